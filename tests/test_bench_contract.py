"""The benchmark script's host-side contract: it refuses more than one GPU
with a message, and its denoiser flop count agrees with the network the
oracle defines (layer shapes, levels, the input's two real channels)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_denoiser_flops_match_the_oracle_layer_shapes():
    sys.path.insert(0, ROOT)
    import bench
    from oracle import unet as U
    shape = (128, 128, 128)
    nvox = shape[0] * shape[1] * shape[2]
    want = 0
    for name, (ci, co) in U.layer_shapes().items():
        level = int(name[3])
        if name == "enc0a":
            ci = 2          # dose and density; the rest is padding
        want += 2 * 27 * ci * co * (nvox >> (3 * level))
    assert bench.unet_forward_flops(shape) == want
