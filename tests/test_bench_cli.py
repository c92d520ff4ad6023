"""Host-side checks of bench.py's command line (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    """The update is measured on one GPU; --gpus N > 1 exits (code 2) and says why,
    before touching any device."""
    out = _bench("--gpus", "2")
    assert out.returncode == 2
    assert "one GPU" in out.stderr and "--gpus 2" in out.stderr
    assert out.stdout == ""


def test_committed_traffic_summaries_match_the_kernel_source_and_default_shapes():
    """The committed rocprofv3 traffic summaries were taken on the current kernel source
    in the launch shapes the benchmark uses, so the bench line carries them; the FP32
    figure is within a few percent of the algorithmic 144 B per node."""
    sys.path.insert(0, ROOT)
    import bench
    single = bench.measured_traffic("step_ab_f32_4096", (2, 2, 2))
    assert single is not None
    alg = 36 * 4 * 4096 * 4096
    assert 1.0 <= single / alg < 1.05
    with open(os.path.join(ROOT, "profiles", "traffic_step_ab_batch_f32_batch64.txt")) as fh:
        kv = dict(line.strip().split("=", 1) for line in fh if "=" in line and not line.startswith("#"))
    assert kv["kernel_source_sha"] == bench.kernel_sha()
    assert kv["launch_shape"].endswith("q0")  # grid mode, as the autotuner picked it
