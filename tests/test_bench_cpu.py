"""bench.py on the CPU: more than one GPU is refused with a message before any device work
(the library runs on one GPU), and the roofline entry follows its stated formula."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    for argv, env in ((["--gpus", "2"], {}), (["--gpus", "8", "--steps", "1"], {}), ([], {"WORLD_SIZE": "2"})):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], capture_output=True, text=True,
                           timeout=300, env=dict(os.environ, **env))
        assert r.returncode == 2, (argv, r.stdout, r.stderr)
        assert "one GPU" in r.stderr
        assert r.stdout.strip() == ""            # no JSON line


def test_roofline_entry():
    """The roofline entry prices one launch at its algorithmic bytes (140 B per particle, 56 B per
    contact) over the measured average launch time, against the 8 TB/s HBM peak; traffic only for
    the row-tile kernel."""
    sys.path.insert(0, ROOT)
    import bench
    N, ncell, contacts = 100_000, 33 ** 3, 38_875
    b = bench.pairs_kernel_bytes(N, ncell, contacts, 37)
    assert b == N * 140 + 56 * contacts
    timing = {"k_pairs": (50 * 0.05, 50)}         # 50 launches of 50 us (ms total, launches)
    r = bench.roofline(timing, N, ncell, contacts, 37, traffic=4.9e7)
    assert abs(r["avg_launch_us"] - 50.0) < 1e-9
    assert abs(r["achieved"] - round(b / 50e-6 / 1e9, 2)) < 1e-9 and r["peak"] == 8000.0
    assert abs(r["frac"] - round(r["achieved"] / 8000.0, 5)) < 1e-12 and r["traffic"] == 49_000_000
    timing["name"] = "k_pairs_sized"                # counters taken on the row tiles only
    assert bench.roofline(timing, N, ncell, contacts, 37, traffic=4.9e7)["traffic"] is None
