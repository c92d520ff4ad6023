"""Throughput of the fused liquid-vapour lattice update on one MI355X.

    python bench.py [--steps K] [--warmup W] [--precision f32|f64|f16|bf16] [--scheme ab|aa]
                    [--rounding nearest|stochastic]
                    [--n 4096] [--no-cpu-baseline] [--gpus 1]
    python bench.py --workload batch64 [--steps K] [--coexistence STEPS]
    python bench.py --workload warmstart [--train-runs 2000] [--horizon 5000] [--epochs 20]
    python bench.py --workload stefan [--steps K] [--stefan-physics 40000000]
    python bench.py --workload laplace [--laplace-steps 2000000]  # FP64 Laplace series over long runs

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
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0  # dense bf16 MFMA
# the fused kernel's source: its own file and the pointwise model pieces it includes
KERNEL_SRCS = [os.path.join(ROOT, "paper_2106_01557_amd", "csrc", n) for n in ("lbm_kernels.hip", "lbm_model.hpp")]
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}


# the bounded-domain kernel's source (the Stefan workload)
BOUNDED_SRCS = [os.path.join(ROOT, "paper_2106_01557_amd", "csrc", n) for n in ("lbm_bounded.hip", "lbm_model.hpp")]
PEAK_FP64_CU_GFLOPS = 78.6e3 / 256  # one CU's share of the FP64 vector peak (78.6 TFLOP/s over 256 CUs)


def kernel_sha(srcs=None) -> str:
    h = hashlib.sha256()
    for path in (KERNEL_SRCS if srcs is None else srcs):
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(tag: str, shape: tuple):
    """HBM bytes per launch from a committed rocprofv3 counter summary taken on the current
    kernel source in the same launch shape (profiles/traffic_<tag>.txt, or one file per
    shape, traffic_<tag>_<shape>.txt), else None."""
    import glob
    want = "x".join(str(v) for v in shape)
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"traffic_{tag}*.txt"))):
        kv = {}
        for line in open(path):
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha") != kernel_sha() or kv.get("launch_shape") != want:
            continue
        try:
            return float(kv["hbm_bytes_per_launch"])
        except (KeyError, ValueError):
            return None
    return None


def measured_flops(tag: str, srcs) -> float | None:
    """Executed FP64 FLOPs per step from a committed rocprofv3 counter summary, if it was
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"flops_{tag}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha") != kernel_sha(srcs):
        return None
    try:
        return float(kv["flops_per_step"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(seconds: float) -> dict:
    """The FP64 oracle as it stands, on the same recipe scaled to 256 x 256 (R = 32) and
    512 x 512 (R = 64), one thread, each timed for about half of `seconds` after one
    warm-up step; `value` is the 256 x 256 rate, both are in `sizes`."""
    import numpy as np
    from oracle import lbm as olbm
    from oracle import thermo
    from paper_2106_01557_amd import inputs
    from threadpoolctl import threadpool_limits

    model = olbm.Model.build(thermo.paper_cs_eos(), thermo.Params(Tr0=0.75))
    d = model.d
    rates, notes = {}, []
    for n in (256, 512):
        f = inputs.droplet(n, n, d.rho_l, d.rho_v, d.T0, n // 8, 4, eps=0.005, seed=1)
        st = olbm.init_state(model, *f.as_tuple())
        with threadpool_limits(limits=1):  # one thread: any BLAS call the oracle makes stays serial
            st = olbm.step(model, st)  # warm-up
            steps, t0 = 0, time.perf_counter()
            while time.perf_counter() - t0 < seconds / 2:
                st = olbm.step(model, st)
                steps += 1
            dt = time.perf_counter() - t0
        assert np.isfinite(st.f).all()
        rates[f"{n}x{n}"] = round(n * n * steps / dt / 1e6, 4)
        notes.append(f"{n}x{n} droplet R={n // 8}: {steps} steps in {dt:.1f} s")
    return {"value": rates["256x256"], "unit": "MLUPS", "cores": 1, "kind": "oracle", "sizes": rates,
            "sample": "FP64 numpy oracle, same recipe, " + "; ".join(notes)
                      + f"; one thread (numpy einsum/roll, BLAS pools limited to 1) on {_host_cpu()}"}


def _host_cpu() -> str:
    """The host's CPU model and logical core count, for the baseline's record."""
    import os
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical cores"


def batch_members(seed: int = 2, count: int = 64):
    """The batched workload: `count` periodic domains with side U{128, 256, 512, 1024},
    a droplet (R = side/4) or a slab (middle half liquid) with equal odds, T/Tc in
    U[0.60, 0.95], tanh interface width 4, +-0.5 % density noise; all from PCG64(seed)."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(count):
        side = int(rng.choice([128, 256, 512, 1024]))
        kind = "droplet" if rng.random() < 0.5 else "slab"
        tr = float(rng.uniform(0.60, 0.95))
        out.append({"side": side, "kind": kind, "Tr0": tr, "seed": seed * 1000 + k})
    return out


def _bulk_samples(m, kind, side):
    """Liquid and vapour sample regions (5 x 5 node means): droplet centre and the
    far corner; slab centre row and the row half a period away (5 rows each)."""
    import torch
    rho, T = m["rho"], m["T"]
    c = side // 2
    if kind == "droplet":
        liq = (slice(c - 2, c + 3), slice(c - 2, c + 3))
        vap = (slice(0, 5), slice(0, 5))
    else:
        liq = (slice(c - 2, c + 3), slice(None))
        vap = (slice(0, 5), slice(None))
    vals = torch.stack([rho[liq].mean(), rho[vap].mean(), T[liq].mean(), T[vap].mean()])
    return vals


def run_batch(args) -> dict:
    import torch
    from paper_2106_01557_amd import inputs, lbm

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    spec = batch_members()
    sols = []
    for m in spec:
        eos, params = lbm.Eos(), {"Tr0": m["Tr0"], "precision": args.precision}
        if args.constants == "interface":
            # below T_r 0.8 each domain's K_EOS and K_INT come from the paper's prescribed
            # sigma = 0.01 and W = 10 at its own T_r0 (at the paper's constants, fixed for
            # T_r0 = 0.8, the interface at T_r 0.6 is 6.6 nodes wide with a density ratio
            # of 132, and droplets there blow up); above it the paper's pair already gives
            # W > 10, while recalibrating there (K_EOS 5.5 at T_r 0.94) lets the start-up
            # transient swing T past Tc
            k = lbm.interface_constants(min(m["Tr0"], 0.8), 0.01, 10.0)
            eos, params["K_int"] = lbm.Eos(K_eos=k["K_eos"]), k["K_int"]
        s = lbm.Solver(m["side"], m["side"], eos=eos, params=params, stream=stream)
        d = s.derived()
        n = m["side"]
        if m["kind"] == "droplet":
            f = inputs.droplet(n, n, d["rho_l"], d["rho_v"], d["T0"], n / 4, 4, eps=0.005, seed=m["seed"])
        else:
            f = inputs.slab(n, n, d["rho_l"], d["rho_v"], d["T0"], n // 4, n - n // 4 - 1, width=4, eps=0.005,
                            seed=m["seed"])
        s.set_fields(*f.as_tuple())
        sols.append(s)
    b = lbm.Batch(sols)
    items, nodes = b.size()
    print(f"# batch ready: {len(sols)} domains, {nodes} nodes", file=sys.stderr, flush=True)
    if args.autotune_steps > 0:
        shape, tuned_ms = b.autotune(args.autotune_steps)
        print(f"# autotuned shape {shape}: {tuned_ms:.4f} ms/step", file=sys.stderr, flush=True)
    else:  # fixed shape (grid mode), e.g. for profiling one kernel configuration
        b.set_shape(args.rows_per_wave or 64, args.waves_per_block or 4, queue=False)
        shape, tuned_ms = b.shape(), 0.0
    b.set_graph(args.graph_steps)
    b.step(args.warmup)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    b.step(args.steps)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = start.elapsed_time(stop) / args.steps
    mlups = nodes * args.steps / wall / 1e6
    b_alg = 36 * STORAGE_BYTES[args.precision] * nodes
    achieved = b_alg / (kernel_ms * 1e-3) / 1e9
    bad_each = [s.invariants(raise_on_bad=False)["bad_nodes"] for s in sols]
    bad = sum(bad_each)
    out = {
        "metric": "MLUPS & % HBM roofline (batched)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f16": "f16-storage/f32", "bf16": "bf16-storage/f32"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": "64 periodic domains, side U{128,256,512,1024}, droplet (R=side/4) or slab (middle half), "
                        "T/Tc U[0.60,0.95], CS EOS (a~=1, b~=4, R=1) with "
                        + ("K_EOS, K_INT from sigma=0.01, W=10 at min(T/Tc, 0.8) per domain" if args.constants == "interface"
                           else "the paper's K_EOS=0.479820, K_INT=2.294922")
                        + ", tanh W=4, +-0.5% noise, PCG64 seed 2",
            "nodes": nodes, "work_items": items, "precision": args.precision,
            "launch_shape": shape, "graph_steps": args.graph_steps,
            "autotune_ms_per_step": round(tuned_ms, 5),
        },
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": measured_traffic(f"step_ab_batch_{args.precision}_batch64",
                                                 (shape["rows_per_wave"],
                                                  f"{shape['waves_per_block']}q{int(bool(shape['queue']))}")),
                     "kernel": "k_step_ab_batch", "kernel_ms": round(kernel_ms, 5)},
        "checks": {"bad_nodes": bad,
                   "failed_domains": [(m["side"], m["kind"], round(m["Tr0"], 4))
                                      for m, x in zip(spec, bad_each) if x > 0]},
    }
    if args.coexistence > 0:
        out["coexistence"] = batch_coexistence(b, sols, spec, args.coexistence, args.check_every,
                                               wall * 1e3 / args.steps)
    if args.alone_steps > 0:
        # the plain method on the same domains: each lattice advanced alone by the
        # single-lattice call (one launch per step, its default launch shape), one
        # lattice after another on the same stream.  Every step is bitwise the one the
        # batch computes, so the wall-clock ratio is the time-to-coexistence speed-up.
        k = args.alone_steps
        for sol in sols:
            sol.step(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for sol in sols:
            sol.step(k)
        torch.cuda.synchronize()
        alone_ms = (time.perf_counter() - t0) * 1e3 / k
        out["alone"] = {"ms_per_step": round(alone_ms, 5), "steps": k,
                        "batched_speedup": round(alone_ms / (wall * 1e3 / args.steps), 3),
                        "what": "each domain stepped by the single-lattice call, one domain after another"}
    return out


def batch_coexistence(b, sols, spec, steps, every, ms_per_step) -> dict:
    """Runs the batch `steps` more steps, sampling bulk densities every `every` steps.
    Time to coexistence of a domain: the first sample after which both bulk densities
    stay within 1e-3 (relative) of their final values.  The final values are compared
    with Maxwell's construction at the measured bulk temperature."""
    import numpy as np
    import torch
    from paper_2106_01557_amd import lbm

    hist = []
    done = 0
    t0 = time.perf_counter()
    stream = sols[0].stream
    while done < steps:
        n = min(every, steps - done)
        b.step(n)
        done += n
        # the moments are written on the solvers' stream: sample them on that stream too
        with torch.cuda.stream(stream):
            row = torch.stack([_bulk_samples(s.moments(("rho", "T")), m["kind"], m["side"])
                               for s, m in zip(sols, spec)]).cpu().numpy()
        hist.append((done, row))
        if len(hist) % 10 == 0:
            print(f"# coexistence run: {done}/{steps} steps, {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                  flush=True)
    final = hist[-1][1]
    per = []
    for i, (s, m) in enumerate(zip(sols, spec)):
        rl, rv, Tl, Tv = (float(v) for v in final[i])
        # settled: from this sample on, both bulk densities stay within 1e-3 of the run's
        # final values, and the run goes on for at least ten more samples (a domain that
        # only settles at the end of the run has no time to coexistence within it)
        t_first = None
        for k in range(len(hist) - 10):
            ok = all(abs(h[1][i][0] - rl) <= 1e-3 * rl and abs(h[1][i][1] - rv) <= 1e-3 * rv for h in hist[k:])
            if ok:
                t_first = hist[k][0]
                break
        Tb = 0.5 * (Tl + Tv)
        bad = s.invariants(raise_on_bad=False)["bad_nodes"]
        try:
            mx = lbm.maxwell(Tb / s.derived()["Tc"])
        except lbm.LbmError:
            mx = {"rho_l": float("nan"), "rho_v": float("nan")}
        per.append({"bad_nodes": bad, "side": m["side"], "kind": m["kind"], "Tr0": round(m["Tr0"], 4),
                    "rho_l": rl, "rho_v": rv, "T_bulk_over_Tc": Tb / s.derived()["Tc"],
                    "rel_dev_rho_l": (rl - mx["rho_l"]) / mx["rho_l"], "rel_dev_rho_v": (rv - mx["rho_v"]) / mx["rho_v"],
                    "steps_to_coexistence": t_first, "finite": bool(np.isfinite(final[i]).all())})
    ttc = [p["steps_to_coexistence"] for p in per if p["steps_to_coexistence"] is not None and p["bad_nodes"] == 0]
    slabs = [p for p in per if p["kind"] == "slab"]
    return {
        "steps": steps, "check_every": every,
        "settled_domains": len(ttc), "domains": len(per),
        "finite_domains": sum(1 for p in per if p["bad_nodes"] == 0),
        "failed_domains": [(p["side"], p["kind"], p["Tr0"]) for p in per if p["bad_nodes"] > 0],
        "steps_to_coexistence_median": float(np.median(ttc)) if ttc else None,
        "steps_to_coexistence_max": max(ttc) if ttc else None,
        "seconds_to_coexistence_all": (max(ttc) * ms_per_step / 1e3) if len(ttc) == len(per) else None,
        "slab_max_rel_dev_vs_maxwell": max(max(abs(p["rel_dev_rho_l"]), abs(p["rel_dev_rho_v"])) for p in slabs)
        if slabs else None,
        "per_domain": per,
    }


def unet_step_flops(widths, in_channels, N, H, W) -> float:
    """Dense FLOPs of one training step's 3x3 convolutions: forward, input gradient (all
    layers but the first) and weight gradient, 2 N h w 9 C_in C_out each."""
    from paper_2106_01557_amd import unet
    tot = 0.0
    for name, ci, co in unet.conv_layers(widths, in_channels):
        lvl = int(name[1])
        f = 2.0 * N * (H >> lvl) * (W >> lvl) * 9 * ci * co
        tot += f * (2 if name == "e0a" else 3)
    return tot


def unet_step_bound_ms(widths, in_channels, N, H, W, outputs=2) -> float:
    """Lower bound on one training step's time, pass by pass: each pass takes at least
    the longer of its dense FLOPs at the bf16 MFMA peak and its compulsory HBM bytes
    (bfloat16 activations and gradients read and written once) at the HBM peak, with the
    passes as the step runs them: a decoder convolution reads [upsample2(lower level) |
    skip] as the two tensors (the lower level at half size), and its input gradient
    stores the skip branch's gradient and, through the upsampling's gradient, the lower
    level's (at half size, gated by it); the encoder's second convolution also stores
    its 2x2 max pooling.  The convolutions' weights and partial sums, and launch gaps,
    are left out."""
    from paper_2106_01557_amd import unet
    peak_f, peak_b = PEAK_BF16_TFLOPS * 1e12, PEAK_HBM_GBS * 1e9
    L = len(widths)
    t = 0.0
    for name, ci, co in unet.conv_layers(widths, in_channels):
        lvl = int(name[1])
        P = N * (H >> lvl) * (W >> lvl)
        fl = 2.0 * P * 9 * ci * co
        pass_t = lambda nbytes: max(fl / peak_f, nbytes / peak_b)  # noqa: E731
        if name[0] == "d" and name[2] == "a":                    # input [upsample2(lower) | skip]
            cu = widths[lvl + 1]
            xin = 2.0 * (P // 4 * cu + P * (ci - cu))
            t += pass_t(xin + 2.0 * P * co)                                    # forward
            t += pass_t(2.0 * P * co + 2.0 * P * (ci - cu) + 4.0 * (P // 4) * cu)  # input gradient
            t += pass_t(xin + 2.0 * P * co)                                    # weight gradient
            continue
        io = 2.0 * P * (ci + co)
        pooled = 2.0 * (P // 4) * co if (name[0] == "e" and name[2] == "b" and lvl < L - 1) else 0.0
        t += pass_t(io + pooled)                                 # forward (+ its pooling)
        if name != "e0a":                                        # input gradient (the b layers
            mask = 2.0 * P * ci if name.endswith("b") else 0.0  # read their ReLU mask)
            t += pass_t(io + mask)
        t += pass_t(io)                                          # weight gradient
    bw = 0.0
    for lvl in range(L - 1):
        c = widths[lvl]
        P = N * (H >> lvl) * (W >> lvl)
        bw += 2.0 * (3 * P * c + P // 4 * c)             # max pool gradient (x, skip gradient, dx; dy)
    P0, c0 = N * H * W, widths[0]
    bw += 2 * (8.0 * P0 * 2 + 2.0 * P0 * in_channels + 4.0 * P0 * 2)   # inputs and targets prepared
    bw += 2.0 * P0 * c0 * 2 + 4.0 * P0 * 2 * 2 + 4.0 * P0 * outputs * 2  # head forward and backward in one pass
    nparam = sum(9 * ci * co + co for _, ci, co in unet.conv_layers(widths, in_channels))
    bw += nparam * (4 * 4 + 3 * 4 + 2 + 2 * 2)           # Adam (p, g, m, v in; p, m, v, bf16 out) and flips
    return (t + bw / peak_b) * 1e3


def run_warmstart(args) -> dict:
    """Learned warm start on 256 x 256 problems: generation of training data by the
    batched solver, training of the U-Net on the matrix cores, held-out loss against the
    no-change baseline, and plain against warm-started time to coexistence."""
    import numpy as np
    import torch
    from paper_2106_01557_amd import unet, warmstart as ws

    torch.cuda.set_device(0)
    log = lambda m: print(f"# {m}", file=sys.stderr, flush=True)  # noqa: E731
    side = 256
    specs = ws.sample_specs(args.train_runs + args.test_runs, seed=3, side=side, constants=args.constants)
    t0 = time.perf_counter()
    ds, failed = ws.generate(specs, args.horizon, log=log)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    gen_mlups = len(specs) * side * side * args.horizon / t_gen / 1e6
    n_ok = ds["rho0"].shape[0]
    n_train = n_ok - args.test_runs
    tr = {k: v[:n_train] for k, v in ds.items()}
    te = {k: v[n_train:] for k, v in ds.items()}
    del ds
    bad = set(failed)
    cmp_pool = [s_ for i, s_ in enumerate(specs) if i not in bad][n_train:]
    net = unet.UNet(seed=0, stream=torch.cuda.current_stream())
    base = ws.identity_loss(te)
    before = ws.evaluate_loss(net, te)
    # one timed training step (inputs resident), then the training run
    B = args.batch
    args_b = [tr[k][:B].contiguous() for k in ws.KEYS]
    for _ in range(3):
        net.train_step(*args_b, lr=0.0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        net.train_step(*args_b, lr=0.0)
    e1.record()
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / reps
    flops = unet_step_flops(net.widths, net.in_channels, B, side, side)
    net = unet.UNet(seed=0, stream=torch.cuda.current_stream())  # fresh parameters for the run
    t0 = time.perf_counter()
    hist = ws.train(net, tr, epochs=args.epochs, batch=B, lr=args.lr, seed=4, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    after = ws.evaluate_loss(net, te)
    log(f"held-out loss: no-change {base:.3e}, untrained {before:.3e}, trained {after:.3e}")
    cmp_specs = cmp_pool[: args.compare_runs]
    eq = ws.equal_error_steps(net, cmp_specs, args.horizon, 250, log=log)
    log(f"equal-error steps saved: median {eq['steps_saved_median']:.0f} of {args.horizon}")
    res = ws.compare_warm_start(net, cmp_specs, args.horizon, args.compare_steps, max(args.check_every, 1000), log=log)
    per = res.pop("per_problem")
    samples_s = args.epochs * (n_train // B) * B / t_train
    achieved = flops / (step_ms * 1e-3) / 1e12
    return {
        "metric": "warm-start U-Net training samples/s (256x256, fwd+bwd+Adam)",
        "value": round(samples_s, 2),
        "unit": "samples/s",
        "n_gpus": 1, "steps": args.epochs * (n_train // B), "warmup": 3,
        "ms_per_step": round(step_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 (FP32 accumulate, FP32 master weights)", "data": "synthetic (solver-generated)",
        "config": {
            "workload": "256x256 periodic problems, 1-8 droplets R U[8,48], T/Tc U[0.6,0.9], "
                        + ("K_EOS, K_INT from sigma=0.01, W=10 at min(T/Tc, 0.8) per problem" if args.constants == "interface"
                           else "the paper's K_EOS, K_INT") + ", tanh W=4, +-0.5% "
                        f"noise, PCG64 seed 3; {n_train} train / {args.test_runs} test runs, horizon "
                        f"{args.horizon} steps; U-Net widths {list(net.widths)}, batch {B}, {args.epochs} epochs",
            "batch": B, "epochs": args.epochs,
        },
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_BF16_TFLOPS, 4), "traffic": None,
                     "kernel": "one training step (all 3x3 convolution kernels, dense FLOPs)",
                     "flops_per_step": flops},
        "data_generation": {"runs": len(specs), "non_finite_runs": len(failed),
                            "non_finite_Tr": [round(specs[i].tr, 4) for i in failed],
                            "seconds": round(t_gen, 2), "MLUPS": round(gen_mlups, 1)},
        "training": {"seconds": round(t_train, 2), "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1]},
        "held_out": {"no_change_loss": base, "untrained_loss": before, "trained_loss": after,
                     "ratio_to_no_change": after / base},
        "equal_error": eq,
        "warm_start": res,
        "warm_start_per_problem": per,
    }


def run_unet_step(args) -> dict:
    """Timed U-Net training steps alone (forward, backward, Adam; the same step as the
    warm-start workload's training) on a batch of seeded 256 x 256 droplet problems,
    each its own target: the kernels do the same work whatever the values."""
    import torch
    from paper_2106_01557_amd import unet, warmstart as ws

    torch.cuda.set_device(0)
    specs = ws.sample_specs(args.batch, seed=3, side=256)
    run = ws.Runner(specs)
    rho0, T0f = run.initial_density(), run.uniform_T()
    net = unet.UNet(seed=0, stream=torch.cuda.current_stream(), wgrad_streams=args.wgrad_streams)
    a = [rho0, T0f, rho0, T0f, run.rho_v, run.rho_l, run.T0, run.cond]
    for _ in range(args.warmup):
        net.train_step(*a, lr=args.lr)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        net.train_step(*a, lr=args.lr)
    e1.record()
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / args.steps
    run.close()
    flops = unet_step_flops(net.widths, net.in_channels, args.batch, 256, 256)
    achieved = flops / (step_ms * 1e-3) / 1e12
    bound = unet_step_bound_ms(net.widths, net.in_channels, args.batch, 256, 256, net.K)
    return {
        "metric": "U-Net training samples/s (256x256, fwd+bwd+Adam)",
        "value": round(args.batch / (step_ms * 1e-3), 2), "unit": "samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(step_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 (FP32 accumulate, FP32 master weights)", "data": "synthetic",
        "config": {"workload": f"U-Net widths {list(net.widths)} on {args.batch} seeded 256x256 droplet problems",
                   "batch": args.batch, "weight_gradient_streams": net.wgrad_streams},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_BF16_TFLOPS, 4), "traffic": None,
                     "kernel": "one training step (all 3x3 convolution kernels, dense FLOPs)",
                     "flops_per_step": flops,
                     "step_bound_ms": round(bound, 4), "frac_of_step_bound": round(bound / step_ms, 4)},
    }


def neumann_k(ste: float) -> float:
    """Root of Eq. (21), Ste / (exp(k^2) erf(k)) = k sqrt(pi), by bisection (the left side
    falls and the right side rises with k)."""
    lo, hi = 0.0, 2.0
    g = lambda k: ste / (math.exp(k * k) * math.erf(k)) - k * math.sqrt(math.pi) if k > 0 else math.inf  # noqa: E731
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if g(mid) > 0 else (lo, mid)
    return 0.5 * (lo + hi)


def interface_x(rho_row, rho_v: float, rho_l: float) -> float:
    """Position of the first crossing of (rho_v + rho_l) / 2 from the heated side, linearly
    interpolated, in nodes from the boundary node x = 0."""
    import numpy as np
    mid = 0.5 * (rho_v + rho_l)
    j = int(np.argmax(rho_row >= mid))
    if j == 0 or rho_row[j] < mid:
        return float("nan")
    return (j - 1) + (mid - rho_row[j - 1]) / (rho_row[j] - rho_row[j - 1])


def run_laplace(args) -> dict:
    """Long FP64 runs of the Laplace radius series (droplets R0 = 16, 32, 64 at the
    centre of 256 x 256, T/Tc 0.8, the paper's constants): at every sample, the
    temperature spread over the domain, the droplet's equimolar radius and
    sigma = (p_in - p_out) R against the square-gradient sigma_ref at the droplet's mean
    temperature.  The energy equation is solved, so T is not held fixed: these runs show
    how far the temperature field settles and what sigma does as it does.  The pressures
    and sigma_ref come from the library's host thermodynamics: p_EOS of Eq. (17) with the
    solver's constants, and sigma_ref(T) = 0.01 K_EOS K_INT / (K_EOS' K_INT') with
    (K_EOS', K_INT') the constants that give sigma = 0.01 at T (sigma scales as K_EOS K_INT,
    text after Eq. (19))."""
    import numpy as np
    import torch
    from paper_2106_01557_amd import inputs, lbm

    torch.cuda.set_device(0)
    n, every, total = 256, args.laplace_every, args.laplace_steps
    eos = lbm.Eos()
    K_int = lbm.default_params()["K_int"]
    Tc = lbm.maxwell(0.8, eos)["Tc"]

    def p_eos(rho, T):
        """Eq. (17), Carnahan-Starling with the attraction a~ rho^2, times K_EOS."""
        t = eos.b_t * rho / 4.0
        return eos.K_eos * (rho * eos.R * T * (1 + t + t * t - t ** 3) / (1 - t) ** 3 - eos.a_t * rho * rho)

    def sigma_ref(T):
        k = lbm.interface_constants(T / Tc, 0.01, 10.0, eos)
        return 0.01 * eos.K_eos * K_int / (k["K_eos"] * k["K_int"])
    out = {"metric": "Laplace law over long runs (FP64)", "unit": "sigma / sigma_ref - 1", "n_gpus": 1,
           "data": "synthetic", "config": {"workload": f"FP64 droplets R0 = 16, 32, 64 on {n}x{n}, T/Tc 0.8, "
                                            "CS EOS with the paper's K_EOS, K_INT, tanh W = 4, no noise",
                                            "steps": total, "sample_every": every}, "droplets": []}
    t0 = time.perf_counter()
    for R0 in (16, 32, 64):
        s = lbm.Solver(n, n, params={"Tr0": 0.8, "precision": "f64", "rows_per_wave": 16})
        rows = []
        try:
            c = s.derived()
            f = inputs.droplet(n, n, c["rho_l"], c["rho_v"], c["T0"], R0, 4.0, eps=0.0)
            s.set_fields(*f.as_tuple())
            done = 0
            while done < total:
                k = min(every, total - done)
                s.step(k)
                done += k
                torch.cuda.synchronize()
                m = s.moments_numpy()
                rho, T = m["rho"], m["T"]
                if not (np.isfinite(rho).all() and np.isfinite(T).all()):
                    rows.append({"step": done, "finite": False})
                    break
                i0 = n // 2
                rl, rv = rho[i0, i0], rho[0, 0]
                dp = float(p_eos(rl, T[i0, i0]) - p_eos(rv, T[0, 0]))
                Req = float(np.sqrt(((rho - rv) / (rl - rv)).sum() / np.pi))
                ref = sigma_ref(0.5 * float(T[i0, i0] + T[0, 0]))
                rows.append({"step": done, "T_spread_over_Tc": float((T.max() - T.min()) / Tc),
                             "T_in_over_Tc": float(T[i0, i0] / Tc), "T_out_over_Tc": float(T[0, 0] / Tc),
                             "R_eq": round(Req, 4), "sigma_rel": float(dp * Req / ref - 1)})
                print(f"# laplace R0={R0}: {done} steps, T spread {rows[-1]['T_spread_over_Tc']:.2e} Tc, "
                      f"sigma {rows[-1]['sigma_rel'] * 100:+.2f} %, {time.perf_counter() - t0:.0f} s",
                      file=sys.stderr, flush=True)
        finally:
            s.close()
        out["droplets"].append({"R0": R0, "samples": rows})
    out["seconds"] = round(time.perf_counter() - t0, 1)
    return out


def run_stefan(args) -> dict:
    """The one-dimensional Stefan problem (the paper's Fig. 1 setting): 1024 x rows, heated
    side at T_r1 = 0.85 with outflow at constant pressure, liquid at rest at T_r0 = 0.8
    beyond a 20-node vapour layer, Ste = 0.005.  Times K steps of the bounded update after
    W warm-up steps; with --stefan-physics it then restarts and runs to the paper's four
    output times (1e7 ... 4e7 steps, t = 0.401e7 ... 1.606e7) and reports the interface
    position against Eq. (20)."""
    import numpy as np
    import torch
    from paper_2106_01557_amd import inputs, lbm

    torch.cuda.set_device(0)
    nx, ny = 1024, args.stefan_rows
    stream = torch.cuda.Stream()
    s = lbm.Solver(nx, ny, params={"precision": args.precision, "bc_x": "heated_outflow", "Tr_wall": 0.85},
                   stream=stream)
    d = s.derived()
    start = inputs.heated_layer(nx, ny, d["rho_l"], d["rho_v"], d["T0"], 20.0, 7.0)
    s.set_fields(*start.as_tuple())
    inv0 = s.invariants()
    s.step(args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    s.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    inv1 = s.invariants(raise_on_bad=False)
    out = {
        "metric": "Stefan problem lattice updates (bounded domain)", "value": round(nx * ny * args.steps / wall / 1e6, 2),
        "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 6), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"1-D Stefan problem {nx}x{ny}, heated side T/Tc 0.85 (outflow, p = p_s(T0)), "
                               "liquid at rest at T/Tc 0.8 beyond a 20-node vapour layer (tanh width 7), Ste 0.005, "
                               "CS EOS with the paper's K_EOS/K_INT", "nx": nx, "ny": ny},
        "roofline": None,
        "roofline_note": ("one workgroup advances the whole domain (up to 8192 nodes) for thousands of steps per "
                          "launch, with two workgroup barriers per step, so the peak is one CU's share of the "
                          "FP64 vector peak; executed FP64 FLOPs per step come from a committed counter summary"),
        "kernel_ms_per_step": round(ms, 6),
        "checks": {"mass_out_of_domain_per_step": (inv1["mass"] - inv0["mass"]) / inv0["mass"] / max(1, args.steps + args.warmup),
                   "bad_nodes": inv1["bad_nodes"]},
    }
    flops = measured_flops(f"step_bounded_{args.precision}_{nx}x{ny}", BOUNDED_SRCS) if args.precision == "f64" else None
    if flops is not None:
        achieved = flops / (ms * 1e-3) / 1e9
        out["roofline"] = {"bound": "alu", "achieved": round(achieved, 2), "peak": round(PEAK_FP64_CU_GFLOPS, 2),
                           "unit": "GFLOP/s", "frac": round(achieved / PEAK_FP64_CU_GFLOPS, 4), "traffic": None,
                           "kernel": "k_step_bounded<double> (one workgroup)", "flops_per_step": flops}
    if args.stefan_physics > 0:
        ste = 0.005
        k = neumann_k(ste)
        alpha = d["c"] ** 2 * d["dt"] * d["tau_j_v"] / 3.0
        s.set_fields(*start.as_tuple())
        m = s.moments_numpy()
        X0 = interface_x(m["rho"][0], d["rho_v"], d["rho_l"])
        marks, done, rows = [], 0, []
        every = args.stefan_every
        t_start = time.perf_counter()
        while done < args.stefan_physics:
            n = min(every, args.stefan_physics - done)
            s.step(n)
            done += n
            m = s.moments_numpy()
            t = done * d["dt"]
            X = interface_x(m["rho"][0], d["rho_v"], d["rho_l"])
            XN = math.sqrt(X0 * X0 + 4 * k * k * alpha * t)
            rows.append((done, t, X))
            print(json.dumps({"stefan_step": done, "t": t, "X": X, "X_neumann": XN,
                              "T1_over_Tc": float(m["T"][0, 1] / d["Tc"]), "s": round(time.perf_counter() - t_start, 1)}),
                  file=sys.stderr, flush=True)
            if done % 10_000_000 == 0:
                marks.append({"steps": done, "t": t, "X": X, "X_neumann": XN, "rel_dev": X / XN - 1})
        arr = np.array(rows)
        late = arr[arr[:, 0] > 0.75 * arr[-1, 0]]
        slope = float(np.polyfit(late[:, 1], late[:, 2] ** 2, 1)[0]) if len(late) >= 2 else float("nan")
        out["stefan"] = {"k": k, "alpha_v": alpha, "X_initial": X0, "Fig1_times": marks,
                         "late_dX2_dt": slope, "neumann_dX2_dt": 4 * k * k * alpha,
                         "late_slope_ratio": slope / (4 * k * k * alpha),
                         "seconds": round(time.perf_counter() - t_start, 1),
                         "bad_nodes": s.invariants(raise_on_bad=False)["bad_nodes"]}
    s.close()
    return out


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


def hbm_probe(nbytes: int = 1 << 30, reps: int = 20) -> int:
    """Reference HBM rates on this GPU with plain library kernels over nbytes: a copy
    (nbytes read + nbytes written), a read-only reduction and a write-only fill, each
    timed with events over reps launches after one untimed launch."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = {}
    for name, fn, moved in (("copy", lambda: dst.copy_(src), 2 * nbytes),
                            ("read", lambda: src.sum(), nbytes),
                            ("write", lambda: dst.fill_(0.5), nbytes)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": round(ms, 4), "TB_s": round(moved / (ms * 1e-3) / 1e12, 3)}
    print(json.dumps({"hbm_probe_bytes": nbytes, "reps": reps, **out}))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="droplet4096",
                    choices=["droplet4096", "batch64", "warmstart", "unet_step", "stefan", "laplace"])
    ap.add_argument("--laplace-steps", type=int, default=2_000_000, help="laplace: steps per droplet")
    ap.add_argument("--laplace-every", type=int, default=200_000, help="laplace: steps between samples")
    ap.add_argument("--train-runs", type=int, default=2000)
    ap.add_argument("--test-runs", type=int, default=64)
    ap.add_argument("--horizon", type=int, default=5000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--compare-runs", type=int, default=64)
    ap.add_argument("--compare-steps", type=int, default=120000,
                    help="warmstart: steps of the plain and warm-started runs (256 x 256 runs settle to 1e-3 in about 1e5)")
    ap.add_argument("--autotune-steps", type=int, default=5)
    ap.add_argument("--graph-steps", type=int, default=20)
    ap.add_argument("--alone-steps", type=int, default=200,
                    help="batch64: also time this many steps of each domain stepped alone (0 = skip)")
    ap.add_argument("--coexistence", type=int, default=0,
                    help="batch64: steps of the coexistence run after the timed steps (0 = skip)")
    ap.add_argument("--check-every", type=int, default=500)
    ap.add_argument("--constants", default="interface", choices=["interface", "paper"],
                    help="batch64 / warmstart: K_EOS and K_INT per domain from sigma = 0.01 and W = 10 at "
                         "min(T_r0, 0.8) (interface), or the paper's pair fixed for T_r0 = 0.8 (paper)")
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--precision", default=None, choices=list(STORAGE_BYTES),
                    help="storage and arithmetic precision (default f32; f64 for the Stefan workload)")
    ap.add_argument("--stefan-rows", type=int, default=1,
                    help="stefan: rows of the 1024-wide domain (a y-uniform state evolves identically in each row)")
    ap.add_argument("--stefan-physics", type=int, default=0,
                    help="stefan: after timing, run this many steps from the start and report the interface "
                         "position (4e7 reaches the paper's last output time)")
    ap.add_argument("--stefan-every", type=int, default=1_000_000, help="stefan: steps between position samples")
    ap.add_argument("--scheme", default="ab", choices=["ab", "aa"])
    ap.add_argument("--rounding", default="nearest", choices=["nearest", "stochastic"],
                    help="rounding of the 16-bit stores (f16/bf16 with the ab scheme)")
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--rows-per-wave", type=int, default=0)
    ap.add_argument("--waves-per-block", type=int, default=0)
    ap.add_argument("--columns-per-lane", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--wgrad-streams", type=int, default=2,
                    help="unet_step: streams for the weight gradients beside the input gradients (0: one stream)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--hbm-probe", action="store_true",
                    help="only time a plain 1 GiB copy, read-only reduction and write-only fill (reference HBM rates)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (for scaling HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()
    if args.hbm_probe:
        return hbm_probe()
    if args.precision is None:
        args.precision = "f64" if args.workload == "stefan" else "f32"
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the update would shard by slabs with halo exchange, which is not implemented)", file=sys.stderr)
        return 2

    if args.workload == "batch64":
        print(json.dumps(run_batch(args)), flush=True)
        return 0
    if args.workload == "warmstart":
        print(json.dumps(run_warmstart(args)), flush=True)
        return 0
    if args.workload == "unet_step":
        print(json.dumps(run_unet_step(args)), flush=True)
        return 0
    if args.workload == "stefan":
        print(json.dumps(run_stefan(args)), flush=True)
        return 0
    if args.workload == "laplace":
        print(json.dumps(run_laplace(args)), flush=True)
        return 0

    import torch
    from paper_2106_01557_amd import inputs, lbm

    torch.cuda.set_device(0)
    n = args.n
    params = {"Tr0": 0.75, "precision": args.precision, "scheme": args.scheme,
              "rows_per_wave": args.rows_per_wave, "waves_per_block": args.waves_per_block,
              "columns_per_lane": args.columns_per_lane}
    if args.rounding != "nearest":
        params["rounding"] = args.rounding
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
            "nx": n, "ny": n, "precision": args.precision, "scheme": args.scheme, "rounding": args.rounding,
            "bytes_per_node_step": 36 * STORAGE_BYTES[args.precision],
            "launch_shape": f"{shape[0]} rows/wave x {shape[1]} waves/block x {shape[2]} columns/lane",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "kernel": (("k_step_ab2 (fused f+g update, two columns per lane)" if shape[2] == 2 else
                        "k_step_ab (fused f+g update, one column per lane)")
                       if args.scheme == "ab" else "k_density + k_step_aa"),
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
