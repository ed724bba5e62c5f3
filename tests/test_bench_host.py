"""bench.py's host-side contract, without a GPU: more than one GPU is refused
with a message before anything touches a device, and the workload helpers
match the batched configuration."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_batched_workload_recipe():
    import bench
    frames, llr, out_bytes, bits, scales = bench.batched_workload(256, seed=5)
    assert len(frames) == len(bits) == len(scales) == 256
    assert all(40 <= f[2] <= 6144 and f[1] == 1 and 0 <= f[0] < 3 for f in frames)
    # LLRs back to back, outputs back to back
    assert frames[0][3] == 0 and frames[0][4] == 0
    assert out_bytes == sum((f[2] + 7) // 8 for f in frames)
    k = {0: 7, 1: 7, 2: 9}
    beta = {0: 2, 1: 3, 2: 2}
    assert llr.size == sum((f[2] + k[f[0]] - 1) * beta[f[0]] for f in frames)
    # the work counted for the roofline: stages x states over every block
    tunes = [(512, 35, -1, 1), (512, 35, -1, 1), (256, 64, -1, 2)]
    w = bench.batch_stages(frames, tunes)
    lo = sum((f[2] + k[f[0]] - 1) * (1 << (k[f[0]] - 1)) for f in frames)  # every stage once
    assert lo <= w <= lo * 1.5
