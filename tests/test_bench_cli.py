"""bench.py on the CPU: more than one GPU is refused with a message (the
workload runs on one GPU), and the measured traffic is taken from a counter
summary only while its source digest matches."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_pmc_traffic_reads_the_profile_digest(tmp_path):
    """bench.pmc_traffic takes the traffic of a counter summary only when the
    summary's source digest (written with or without its file list) matches
    the sources as they are, and its tile length the one asked for"""
    sys.path.insert(0, ROOT)
    import bench
    dig = bench.sources_sha256(bench.SRC_1D)
    files = ", ".join(bench.SRC_1D)
    cases = [(f"sources_sha256 ({files}): {dig}", 242, 123.0),
             (f"sources_sha256: {dig}", 242, 123.0),
             (f"sources_sha256 ({files}): {dig}", 114, None),
             (f"sources_sha256 ({files}): {'0' * 64}", 242, None)]
    for k, (line, tile, want) in enumerate(cases):
        f = tmp_path / f"p{k}.txt"
        f.write_text(f"# a summary\n\n{line}\ntraffic_bytes_per_launch: 123\ntile1d: 242\n")
        assert bench.pmc_traffic(str(f), bench.SRC_1D, tile) == want, line
