"""GPU check of the allocation-free network inference entry point
(swe_nh_cnn_forward_noalloc) against swe_nh_cnn_forward on a caller
workspace: the same kernels on the same inputs, so the outputs must be
identical, bit for bit.  Two calls in a row, the second on a smaller input,
show that what the first left in the library's static scratch does not
reach the second; sizes beyond the scratch's limit and shapes the kernels do
not support are rejected without launching anything."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_17025_amd import swe_nh
    return swe_nh


def net_inputs(B, n, h, w, seed):
    rng = np.random.default_rng(seed)
    npar = B.Net.param_count()
    params = torch.tensor(rng.standard_normal(npar) * 0.1, dtype=torch.float32, device=DEV)
    x = np.zeros((n, h, w, 16), np.float32)
    x[..., :5] = rng.standard_normal((n, h, w, 5))
    u = x.view(np.uint32).astype(np.uint64)
    bits = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)  # BF16, round to nearest even
    xt = torch.from_numpy(bits.view(np.int16).copy()).to(DEV)
    return params, xt


def with_workspace(B, params, x, n, h, w):
    out = torch.empty((n, h, w), dtype=torch.float32, device=DEV)
    B.Net(n, h, w, device=DEV).forward(params, x, out)
    return out


def test_noalloc_forward_matches_workspace_forward(B):
    shapes = [(2, 256, 256, 5), (1, 64, 96, 6)]  # the full scratch, then a smaller input
    for (n, h, w, seed) in shapes:
        print(f"noalloc forward n={n} h={h} w={w} seed={seed}", flush=True)
        assert n * h * w <= B.NOALLOC_MAX_PIXELS
        params, x = net_inputs(B, n, h, w, seed)
        out = torch.full((n, h, w), float("nan"), dtype=torch.float32, device=DEV)
        assert B.cnn_forward_noalloc(params, x, n, h, w, out) == B.OK
        ref = with_workspace(B, params, x, n, h, w)
        torch.cuda.synchronize()
        a, r = out.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(a).all()
        assert np.array_equal(a.view(np.uint32), r.view(np.uint32)), \
            float(np.abs(a - r).max())


def test_noalloc_forward_rejects_what_does_not_fit(B):
    params, x = net_inputs(B, 1, 16, 16, 7)
    out = torch.zeros((1, 16, 16), dtype=torch.float32, device=DEV)
    # beyond the scratch's pixel limit: rejected before any launch
    assert B.cnn_forward_noalloc(params, x, 3, 256, 256, out) == B.ENOMEM
    # shapes the kernels do not take
    assert B.cnn_forward_noalloc(params, x, 1, 24, 16, out) == B.EINVAL
    assert B.cnn_forward_noalloc(params, x, 0, 16, 16, out) == B.EINVAL
    torch.cuda.synchronize()
    assert (out == 0).all()
