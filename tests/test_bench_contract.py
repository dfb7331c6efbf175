"""Host-side checks of bench.py's contract (no GPU): the one-GPU refusal and the bookkeeping that
ties the reported HBM traffic to a committed rocprofv3 summary."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_measured_traffic_matches_a_committed_profile():
    """Every (workload, shape) whose traffic bench.py may report has a profile under profiles/
    naming that shape's flags and stating the same bytes per launch."""
    sys.path.insert(0, ROOT)
    import bench
    texts = [open(os.path.join(ROOT, "profiles", f)).read() for f in os.listdir(os.path.join(ROOT, "profiles"))
             if f.endswith(".md")]
    for wl, entries in bench.MEASURED_TRAFFIC.items():
        for family, shape, digest, nbytes in entries:
            if family == "row-lane":
                flags = (f"--sweep diag --diag-rows {shape['rows_per_block']} --diag-k {shape['ordinates_per_lane']} "
                         f"--band {shape['waves_per_group']}")
            else:
                flags = f"--sweep strip --tile {shape['sweep_tile']} --band {shape['band']}"
            hits = [t for t in texts if f"--workload {wl} " in t and flags in t
                    and f"Traffic per launch: **{nbytes / 1e6:.2f} MB**" in t]
            assert hits, (wl, shape, nbytes)
            assert re.fullmatch(r"[0-9a-f]{16}", digest)
