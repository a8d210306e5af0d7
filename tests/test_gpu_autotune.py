"""The launch-shape autotuner: whole-step timing of every 1D tile size on a
copy of the caller's state (which it leaves untouched), and the table it
persists and reuses."""
import json

import numpy as np
import pytest

import swe_inputs as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_tune_1d_picks_a_candidate_and_persists(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_17025_amd import autotune
    case = S.slide_case(n=8192, dx=0.005)
    f = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    state = (f(case.h), f(case.hu), f(case.hw))
    before = [a.clone() for a in state]
    kw = dict(crit=S.CRIT_ETA_D, k_nh=1e-3, enlarge=1, cfl=0.5, precision=0)
    table = tmp_path / "tune.json"
    tile, times = autotune.tune_1d(case, kw, state, case.t0, nsteps=20, warmup=4,
                                   table_path=str(table))
    cands = autotune.candidates_1d(kw)
    assert cands == (114, 128, 242, 256, 498, 512)
    assert tile in cands and set(times) == set(cands)
    assert all(v > 0 for v in times.values()) and times[tile] == min(times.values())
    for a, b in zip(state, before):
        assert torch.equal(a, b)
    saved = json.loads(table.read_text())
    assert len(saved) == 1 and list(saved.values())[0]["tile"] == tile
    # a second call reads the table instead of timing again
    tile2, times2 = autotune.tune_1d(case, kw, state, case.t0, nsteps=20, warmup=4,
                                     table_path=str(table))
    assert tile2 == tile and times2 == times
