"""Throughput of the fused liquid-vapour lattice update on one MI355X.

    python bench.py [--steps K] [--warmup W] [--precision f32|f64|f16|bf16] [--scheme ab|aa]
                    [--n 4096] [--no-cpu-baseline] [--gpus 1]

Workload: a static droplet on a periodic 4096 x 4096 D2Q9 lattice, radius 512 at
the domain centre, tanh interface of width 4 nodes, Carnahan-Starling EOS with the
paper's K_EOS/K_INT at T/Tc = 0.75, +-0.5 % seeded (PCG64, seed 1) noise on the
density, fluid at rest, FP32 storage and arithmetic.  One "step" is one time step
of the whole update (density, pair force, moments, EOS, both collisions,
streaming) over the whole lattice, i.e. one launch of the fused kernel.

Prints one JSON line: MLUPS (whole job, inputs resident in HBM), the HBM
roofline of the fused kernel (algorithmic bytes = 36 populations read+written per
node per step, divided by the kernel's average duration from HIP events recorded
on the stream the kernel runs on), the HBM traffic measured by rocprofv3 counters
(if a summary for the current kernel source is committed under profiles/), and the
CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2106_01557_amd", "csrc", "lbm_kernels.hip")
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}


def kernel_sha() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(tag: str, shape: tuple):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it was taken on
    the current kernel source in the same launch shape (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha") != kernel_sha():
        return None
    if kv.get("launch_shape") != f"{shape[0]}x{shape[1]}":
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(seconds: float) -> dict:
    """The FP64 oracle as it stands, on the same recipe scaled to 256 x 256 (R = 32)."""
    import numpy as np
    from oracle import lbm as olbm
    from oracle import thermo
    from paper_2106_01557_amd import inputs

    model = olbm.Model.build(thermo.paper_cs_eos(), thermo.Params(Tr0=0.75))
    d = model.d
    n = 256
    f = inputs.droplet(n, n, d.rho_l, d.rho_v, d.T0, 32, 4, eps=0.005, seed=1)
    st = olbm.init_state(model, *f.as_tuple())
    st = olbm.step(model, st)  # warm-up
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        st = olbm.step(model, st)
        steps += 1
    dt = time.perf_counter() - t0
    assert np.isfinite(st.f).all()
    return {"value": round(n * n * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"FP64 numpy oracle, {n}x{n} droplet R=32 (same recipe), {steps} steps in {dt:.1f} s, "
                      f"single thread (numpy einsum/roll loops, no BLAS)"}


def copy_calibration(nbytes: int = 1 << 30, reps: int = 10) -> int:
    """A plain device copy of known size: read nbytes + write nbytes per launch.  Profiling
    it with the same HBM counters gives the factor that turns counter readings into bytes."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps,
                      "ms": round(dt * 1e3, 4), "GB_s_read_plus_write": round(2 * nbytes / dt / 1e9, 1)}))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--precision", default="f32", choices=list(STORAGE_BYTES))
    ap.add_argument("--scheme", default="ab", choices=["ab", "aa"])
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--rows-per-wave", type=int, default=0)
    ap.add_argument("--waves-per-block", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (for scaling HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported by this build "
              "(the update would shard by slabs with halo exchange, which is not built)", file=sys.stderr)
        return 2

    import torch
    from paper_2106_01557_amd import inputs, lbm

    torch.cuda.set_device(0)
    n = args.n
    params = {"Tr0": 0.75, "precision": args.precision, "scheme": args.scheme,
              "rows_per_wave": args.rows_per_wave, "waves_per_block": args.waves_per_block}
    stream = torch.cuda.Stream()
    solver = lbm.Solver(n, n, params=params, stream=stream)
    d = solver.derived()
    f = inputs.droplet(n, n, d["rho_l"], d["rho_v"], d["T0"], 512, 4, eps=0.005, seed=1)
    solver.set_fields(*f.as_tuple())
    del f
    inv0 = solver.invariants()
    print(f"# workload ready: {n}x{n}, {args.precision}/{args.scheme}, warmup {args.warmup}", file=sys.stderr,
          flush=True)
    solver.step(args.warmup)
    torch.cuda.synchronize()

    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    solver.step(args.steps)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = start.elapsed_time(stop)
    inv1 = solver.invariants()

    nodes = n * n
    launches_per_step = 1 if args.scheme == "ab" else 2
    mlups = nodes * args.steps / wall / 1e6
    ms_per_step = wall * 1e3 / args.steps
    # algorithmic bytes of one fused launch: 18 populations read and 18 written per node
    b_alg = 36 * STORAGE_BYTES[args.precision] * nodes
    if args.scheme == "aa":
        # the AA scheme's collide kernel also reads the density stencil (one FP64 value per node)
        b_alg += 8 * nodes
    kernel_ms = ev_ms / args.steps / launches_per_step if args.scheme == "ab" else ev_ms / args.steps
    achieved = b_alg / (kernel_ms * 1e-3) / 1e9
    tag = f"step_{args.scheme}_{args.precision}_{n}"
    shape = solver.launch_shape()
    traffic = measured_traffic(tag, shape)
    out = {
        "metric": "MLUPS & % HBM roofline",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f16": "f16-storage/f32", "bf16": "bf16-storage/f32"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": f"static droplet {n}x{n} periodic D2Q9, R=512, tanh W=4, CS EOS (a~=1, b~=4, R=1, "
                        f"K_EOS=0.479820, K_INT=2.294922), T/Tc=0.75, +-0.5% noise seed 1",
            "nx": n, "ny": n, "precision": args.precision, "scheme": args.scheme,
            "bytes_per_node_step": 36 * STORAGE_BYTES[args.precision],
            "launch_shape": f"{shape[0]} rows/wave x {shape[1]} waves/block",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "kernel": "k_step_ab (fused f+g update)" if args.scheme == "ab" else "k_density + k_step_aa",
            "kernel_ms": round(kernel_ms, 5),
        },
        "checks": {
            "mass_rel_drift": (inv1["mass"] - inv0["mass"]) / inv0["mass"],
            "bad_nodes": inv1["bad_nodes"],
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
