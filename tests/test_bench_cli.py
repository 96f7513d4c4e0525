"""bench.py's contract on the CPU: more than one GPU is refused with a
message, and the algorithmic bytes per cell behind the roofline line are
the compulsory reads and writes of each kernel (FP64, half spectrum of
ny/2 + 1 complex modes per ny reals)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_algorithmic_bytes_per_cell():
    sys.path.insert(0, ROOT)
    import bench
    b = bench.kernel_bytes_per_cell(384)
    half = 16.0 * 193 / 384
    assert b["predict"] == 7 * 8 + 6 * 8            # u v w p H(3) in, H(3) u~(3) out
    assert b["project"] == 5 * 8 + 4 * 8            # u~(3) phi p in, u v w p out
    assert abs(b["div_ffty"] - (24 + half)) < 1e-12
    assert abs(b["fftz_fwd"] - 2 * half) < 1e-12 and abs(b["tri_x"] - 2 * half) < 1e-12
    assert abs(b["iffty"] - (half + 8)) < 1e-12
    # the fluid step moves about 272.3 B per cell
    total = b["predict"] + b["div_ffty"] + b["fftz_fwd"] + b["tri_x"] + b["fftz_inv"] + b["iffty"] + b["project"]
    assert abs(total - 272.3) < 0.1
