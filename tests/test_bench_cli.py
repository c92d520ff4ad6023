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
    alg = 36 * 4 * 4096 * 4096
    for shape in ((3, 4, 2), (2, 2, 2)):  # the default, and the earlier default
        single = bench.measured_traffic("step_ab_f32_4096", shape)
        assert single is not None, shape
        assert 1.0 <= single / alg < 1.05
    with open(os.path.join(ROOT, "profiles", "traffic_step_ab_batch_f32_batch64.txt")) as fh:
        kv = dict(line.strip().split("=", 1) for line in fh if "=" in line and not line.startswith("#"))
    assert kv["kernel_source_sha"] == bench.kernel_sha()
    assert kv["launch_shape"].endswith("q0")  # grid mode, as the autotuner picked it
    # the shapes the autotuner has picked between runs each have a summary of their own
    alg_batch = 36 * 4 * 27_590_656
    for rows, waves in ((4, 2), (4, 4), (4, 1), (8, 2)):
        t = bench.measured_traffic("step_ab_batch_f32_batch64", (rows, f"{waves}q0"))
        assert t is not None, (rows, waves)
        assert 1.0 <= t / alg_batch < 1.1
    assert bench.measured_traffic("step_ab_batch_f32_batch64", (2, "2q0")) is None


def test_committed_flop_summary_matches_the_bounded_kernel_source():
    """The Stefan workload's ALU roofline uses executed FP64 FLOPs per step from a committed
    rocprofv3 counter summary taken on the current bounded-kernel source: about 500 FP64
    operations per node of the 1024-node lattice (the pointwise model of the periodic
    update plus the boundary extrapolation)."""
    sys.path.insert(0, ROOT)
    import bench
    fl = bench.measured_flops("step_bounded_f64_1024x1", bench.BOUNDED_SRCS)
    assert fl is not None
    assert 300 * 1024 < fl < 800 * 1024
    assert abs(bench.PEAK_FP64_CU_GFLOPS - 307.03) < 0.01


def test_unet_step_bound_sits_between_the_mfma_and_the_summed_bounds():
    """The U-Net line's per-pass bound takes, pass by pass, the longer of the MFMA time at
    the dense bf16 peak and the HBM time of the activations: at least the whole step's
    FLOPs at peak, at most the MFMA and HBM times added, and 0.61 ms for the 16 x 256^2
    batch (most 256^2 and 128^2 passes are HBM-bound at 32 and 64 channels)."""
    sys.path.insert(0, ROOT)
    import bench
    args = ((32, 64, 128, 256), 8, 16, 256, 256)
    b = bench.unet_step_bound_ms(*args)
    mfma_only = bench.unet_step_flops(*args) / (bench.PEAK_BF16_TFLOPS * 1e12) * 1e3
    assert mfma_only < b < 2.5 * mfma_only
    assert 0.58 < b < 0.65
    # halving the batch halves every term but the optimizer's (about 8 us)
    half = bench.unet_step_bound_ms((32, 64, 128, 256), 8, 8, 256, 256)
    assert 0.006 < 2 * half - b < 0.011


def test_bench_uses_the_oracle_only_in_the_cpu_baseline():
    """The oracle is test infrastructure: in bench.py only the CPU-baseline leg imports it;
    every GPU workload, and its analysis, runs on the library."""
    import ast
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())

    def imports_oracle(node):
        if isinstance(node, ast.ImportFrom):
            mods = [node.module or ""]
        elif isinstance(node, ast.Import):
            mods = [a.name for a in node.names]
        else:
            return False
        return any(m == "oracle" or m.startswith("oracle.") for m in mods)

    assert not any(imports_oracle(n) for n in tree.body)  # nothing at module level
    seen = {fn.name for fn in ast.walk(tree) if isinstance(fn, ast.FunctionDef)
            and any(imports_oracle(n) for n in ast.walk(fn))}
    assert seen == {"cpu_baseline"}, seen
