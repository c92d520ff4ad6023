"""Learned warm start for the liquid-vapour lattice update.

The solver generates its own training data: seeded periodic fields with several
droplets are advanced `horizon` steps by the batched two-buffer update; a U-Net
(unet.py) learns the map from the initial density and temperature fields (and the
run's reduced temperature) to the density and temperature fields at the horizon;
the solver then starts from the network's prediction (fluid at rest) and finishes
the relaxation, so the lattice model, not the network, decides the final state.
The temperature is part of the prediction because latent heat moves it by up to
about ten percent near interfaces, and the coexistence densities follow it.

Time to coexistence of a run: the first sample after which both bulk densities
(liquid: mean density over nodes whose normalised density exceeds 0.9; vapour:
over nodes below 0.1) stay within a relative 1e-3 of the run's final values.  The
warm-started run's final bulk densities are also compared with the plain run's
(the accuracy of the state the warm start settles in).

All arithmetic of the lattice update, the network and the optimizer runs in the
library's kernels; torch provides memory, the stream and the bookkeeping
reductions of the diagnostics.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import inputs, lbm, unet


@dataclass
class Spec:
    """One problem: droplet centres and radii on a side x side periodic lattice at T/Tc = tr,
    with the scaling constants K_EOS, K_INT of its run (None: the paper's pair)."""
    side: int
    tr: float
    centres: list
    radii: list
    seed: int
    K_eos: float | None = None
    K_int: float | None = None


def sample_specs(n: int, seed: int, side: int = 256, drops=(1, 8), radii=(8.0, 48.0), tr=(0.6, 0.9),
                 constants: str = "interface") -> list:
    """n problems from PCG64(seed): droplet count uniform in drops, radii uniform in
    radii, centres uniform on the lattice, T/Tc uniform in tr.  constants = 'interface'
    gives a problem below T/Tc 0.8 the K_EOS and K_INT for which the flat interface at its
    T/Tc has the paper's surface tension 0.01 and width 10 (at the paper's pair, fixed for
    T/Tc = 0.8, droplets below T/Tc 0.65 blow up) and keeps the paper's pair above 0.8,
    where it already gives a wider interface; 'paper' keeps the paper's pair throughout."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n):
        m = int(rng.integers(drops[0], drops[1] + 1))
        cs = [(float(rng.uniform(0, side)), float(rng.uniform(0, side))) for _ in range(m)]
        rs = [float(rng.uniform(*radii)) for _ in range(m)]
        t = float(rng.uniform(*tr))
        K = lbm.interface_constants(min(t, 0.8), 0.01, 10.0) if constants == "interface" else {"K_eos": None, "K_int": None}
        out.append(Spec(side, t, cs, rs, seed * 100003 + k, K["K_eos"], K["K_int"]))
    return out


def _cond(tr: float) -> float:
    """T/Tc mapped to [-1, 1] over the sampled range [0.6, 0.9]."""
    return (tr - 0.75) / 0.15


class Runner:
    """Advances many problems together with the batched update (one precision, one stream)."""

    def __init__(self, specs, precision="f32", stream=None, width=4.0, eps=0.005):
        import torch
        self.torch = torch
        self.specs = list(specs)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.solvers, self.consts = [], []
        for s in self.specs:
            params, eos = {"Tr0": s.tr, "precision": precision}, lbm.Eos()
            if s.K_eos is not None:
                eos, params["K_int"] = lbm.Eos(K_eos=s.K_eos), s.K_int
            sol = lbm.Solver(s.side, s.side, eos=eos, params=params, stream=self.stream)
            self.solvers.append(sol)
            self.consts.append(sol.derived())
        self.width, self.eps = width, eps
        self.batch = lbm.Batch(self.solvers)  # the precision's default launch shape
        d = lambda key: torch.tensor([c[key] for c in self.consts], dtype=torch.float64, device="cuda")  # noqa: E731
        self.rho_v, self.rho_l, self.T0 = d("rho_v"), d("rho_l"), d("T0")
        self.cond = torch.tensor([_cond(s.tr) for s in self.specs], dtype=torch.float64, device="cuda")

    def initial_density(self):
        """The seeded initial fields [n, side, side] (host FP64, then device)."""
        out = []
        for s, c in zip(self.specs, self.consts):
            f = inputs.droplets(s.side, s.side, c["rho_l"], c["rho_v"], c["T0"], s.centres, s.radii, self.width,
                                eps=self.eps, seed=s.seed)
            out.append(f.rho)
        return self.torch.as_tensor(np.stack(out), dtype=self.torch.float64).cuda()

    def uniform_T(self):
        return self.T0[:, None, None].expand(-1, self.specs[0].side, self.specs[0].side).contiguous()

    def set_fields(self, rho, T=None):
        """Start every problem from density (and temperature) fields [n, side, side]
        (device), fluid at rest; T = None: T0 everywhere."""
        torch = self.torch
        with torch.cuda.stream(self.stream):
            for k, (s, c) in enumerate(zip(self.solvers, self.consts)):
                z = torch.zeros_like(rho[k])
                t = torch.full_like(rho[k], c["T0"]) if T is None else T[k].contiguous()
                s.set_fields(rho[k].contiguous(), z, z, t)
        self.stream.synchronize()

    def step(self, n: int):
        self.batch.step(n)

    def density(self):
        torch = self.torch
        with torch.cuda.stream(self.stream):
            out = torch.stack([s.moments(("rho",))["rho"] for s in self.solvers])
        self.stream.synchronize()
        return out

    def fields(self):
        """Density and temperature [n, side, side] (device FP64)."""
        torch = self.torch
        with torch.cuda.stream(self.stream):
            m = [s.moments(("rho", "T")) for s in self.solvers]
            rho, T = torch.stack([x["rho"] for x in m]), torch.stack([x["T"] for x in m])
        self.stream.synchronize()
        return rho, T

    def bulk(self, rho=None):
        """(liquid, vapour) bulk densities per problem ([n] FP64 host arrays; NaN where a
        phase has no bulk nodes)."""
        torch = self.torch
        rho = self.density() if rho is None else rho
        with torch.cuda.stream(self.stream):
            nu = (rho - self.rho_v[:, None, None]) / (self.rho_l - self.rho_v)[:, None, None]
            liq, vap = (nu > 0.9).double(), (nu < 0.1).double()
            lsum, lcnt = (rho * liq).sum(dim=(1, 2)), liq.sum(dim=(1, 2))
            vsum, vcnt = (rho * vap).sum(dim=(1, 2)), vap.sum(dim=(1, 2))
            res = torch.stack([lsum / lcnt, vsum / vcnt]).cpu().numpy()
        return res[0], res[1]

    def close(self):
        self.batch.close()
        for s in self.solvers:
            s.close()


KEYS = ("rho0", "T0f", "rhoT", "TT", "rho_v", "rho_l", "T0", "cond")


def generate(specs, horizon: int, chunk: int = 64, precision: str = "f32", log=None):
    """Runs every problem `horizon` steps from its seeded initial field (at rest, T0).
    Returns device tensors rho0, T0f, rhoT, TT [n, side, side] (FP64) and rho_v, rho_l,
    T0, cond [n] of the runs that stayed finite, and the indices (into specs) of those
    that did not."""
    import torch
    parts = {k: [] for k in KEYS}
    failed = []
    for i in range(0, len(specs), chunk):
        r = Runner(specs[i:i + chunk], precision=precision)
        rho0 = r.initial_density()
        r.set_fields(rho0)
        r.step(horizon)
        rhoT, TT = r.fields()
        ok = torch.isfinite(rhoT).all(dim=(1, 2)) & torch.isfinite(TT).all(dim=(1, 2))
        failed += [i + j for j in range(len(ok)) if not bool(ok[j])]
        keep = torch.nonzero(ok).flatten()
        for key, v in (("rho0", rho0), ("T0f", r.uniform_T()), ("rhoT", rhoT), ("TT", TT), ("rho_v", r.rho_v),
                       ("rho_l", r.rho_l), ("T0", r.T0), ("cond", r.cond)):
            parts[key].append(v.index_select(0, keep))
        r.close()
        if log:
            log(f"generated {min(i + chunk, len(specs))}/{len(specs)} runs ({len(failed)} non-finite so far)")
    return {k: torch.cat(v) for k, v in parts.items()}, failed


def identity_loss(ds, theta_scale: float = 0.1, outputs: int = 2) -> float:
    """Mean squared error (normalised fields, as the network's loss) of predicting no
    change: the no-net baseline."""
    nu = lambda r: (r - ds["rho_v"][:, None, None]) / (ds["rho_l"] - ds["rho_v"])[:, None, None]  # noqa: E731
    th = lambda t: (t / ds["T0"][:, None, None] - 1) / theta_scale  # noqa: E731
    e = [((nu(ds["rhoT"]) - nu(ds["rho0"])) ** 2).mean()]
    if outputs > 1:
        e.append(((th(ds["TT"]) - th(ds["T0f"])) ** 2).mean())
    return float(sum(e) / len(e))


def train(net: "unet.UNet", ds, epochs: int, batch: int = 16, lr: float = 1e-3, seed: int = 0, log=None,
          lr_final: float | None = None):
    """Adam on the mean squared error of the normalised density; minibatches drawn
    without replacement each epoch from PCG64(seed); cosine decay of the rate to
    lr_final (default lr / 10).  Returns the per-epoch mean losses."""
    import torch
    n = ds["rho0"].shape[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    steps = epochs * (n // batch)
    lr_final = lr / 10 if lr_final is None else lr_final
    hist, k = [], 0
    for ep in range(epochs):
        order = torch.as_tensor(rng.permutation(n), device="cuda")
        losses = []
        for j in range(n // batch):
            idx = order[j * batch:(j + 1) * batch]
            with torch.cuda.stream(net.stream):
                args = [ds[key].index_select(0, idx).contiguous() for key in KEYS]
            rate = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * k / max(steps - 1, 1)))
            loss = net.train_step(*args, lr=rate)
            losses.append(loss.clone())
            k += 1
        mean = float(torch.stack(losses).mean().cpu())
        hist.append(mean)
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {mean:.3e}")
    return hist


def evaluate_loss(net, ds, batch: int = 16) -> float:
    """Mean squared error of the network on a dataset (no parameter update)."""
    import torch
    n = ds["rho0"].shape[0]
    tot = 0.0
    for j in range(0, n - batch + 1, batch):
        sl = slice(j, j + batch)
        _, loss = net.forward(ds["rho0"][sl], ds["T0f"][sl], ds["rho_v"][sl], ds["rho_l"][sl], ds["T0"][sl],
                              ds["cond"][sl], ds["rhoT"][sl], ds["TT"][sl])
        tot += float(loss.cpu()) * batch
    return tot / (n // batch * batch)


def coexistence_times(runner: Runner, start_rho, steps: int, every: int, final=None, start_T=None,
                      settle: int = 10):
    """Runs from (start_rho, start_T) and records the bulk densities every `every` steps.
    final: (liquid, vapour) reference values (default: this run's last sample).  A
    problem's time to coexistence is the first sample from which both bulk densities stay
    within 1e-3 of the reference, provided at least `settle` more samples follow (a run
    that only gets there at its end has none).  Returns the per-problem step counts (None
    where not reached), the last bulk values and the elapsed seconds of the stepping."""
    runner.set_fields(start_rho, start_T)
    hist, t_step = [], 0.0
    done = 0
    while done < steps:
        n = min(every, steps - done)
        t0 = time.perf_counter()
        runner.step(n)
        runner.stream.synchronize()
        t_step += time.perf_counter() - t0
        done += n
        hist.append((done, *runner.bulk()))
    last = (hist[-1][1], hist[-1][2])
    ref = last if final is None else final
    times = []
    for i in range(len(runner.specs)):
        t_hit = None
        for k in range(len(hist) - settle):
            ok = all(abs(h[1][i] - ref[0][i]) <= 1e-3 * abs(ref[0][i]) and
                     abs(h[2][i] - ref[1][i]) <= 1e-3 * abs(ref[1][i]) for h in hist[k:])
            if ok:
                t_hit = hist[k][0]
                break
        times.append(t_hit)
    return times, last, t_step


def guard_prediction(rho, T, rho_v, rho_l, T0, t_band: float = 0.15):
    """Keeps a predicted state inside the range a solver run can start from.  The network
    predicts the normalised density (rho - rho_v) / (rho_l - rho_v), so an error of a few
    hundredths in the vapour gives a negative density at low temperature, and the solver
    diverges from it.  Densities are held in [rho_v / 2, rho_l + (rho_l - rho_v) / 20]
    and temperatures within t_band of T0, per problem ([N, H, W] tensors, [N] bounds)."""
    lo = (0.5 * rho_v)[:, None, None]
    hi = (rho_l + 0.05 * (rho_l - rho_v))[:, None, None]
    t0 = T0[:, None, None]
    rho = rho.clamp_min(0).maximum(lo).minimum(hi)
    T = T.maximum((1 - t_band) * t0).minimum((1 + t_band) * t0)
    return rho, T


def _masses(runner: Runner, rho):
    """Per-problem mass of the density field, as the library's diagnostics sum it."""
    runner.set_fields(rho)
    return np.array([s.invariants(raise_on_bad=False)["mass"] for s in runner.solvers])


def match_mass(runner: Runner, rho0, prho, pT, rounds: int = 3):
    """Puts a guarded prediction back on the initial state's mass, the one invariant the
    update keeps exactly: the density is rescaled per problem to the initial mass and
    re-guarded.  The temperature stays as predicted.  The total energy (sum rho e_k plus
    the discrete potential energy) is not an invariant of the discrete update: it falls
    by about 1.5e-3 of itself in the first 400 steps of a two-droplet 64 x 64 problem
    and 6e-3 in 3000, so the horizon state the network learned already carries that
    loss, and restoring the initial energy would start the run too hot.  Returns (rho,
    relative mass offsets left)."""
    torch = runner.torch
    m0 = _masses(runner, rho0)
    dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    for k in range(rounds + 1):
        m1 = _masses(runner, prho)
        with torch.cuda.stream(runner.stream):
            prho = prho * dev(m0 / m1)[:, None, None]
            if k < rounds:  # the last rescale is not clamped again: it is within a part in 1e6 of 1
                prho, _ = guard_prediction(prho, pT, runner.rho_v, runner.rho_l, runner.T0)
    return prho, np.abs(_masses(runner, prho) / m0 - 1)


def compare_warm_start(net, specs, horizon: int, steps: int, every: int, log=None):
    """Plain runs against warm-started runs on the same problems, at equal final error:
    a warm run's time to coexistence is the first sample after which both its bulk
    densities stay within 1e-3 of the plain run's final values; a warm run whose final
    values are not within 1e-3 of the plain run's (it settled elsewhere, e.g. another
    arrangement of droplets after coarsening) has no time and is counted as not
    reaching the plain run's state.  Returns a summary dict."""
    import torch
    r = Runner(specs)
    rho0 = r.initial_density()
    T0f = r.uniform_T()
    plain, final, t_plain = coexistence_times(r, rho0, steps, every)
    if log:
        log("plain runs done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prho, pT = net.predict_fields(rho0, T0f, r.rho_v, r.rho_l, r.T0, r.cond)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    with torch.cuda.stream(r.stream):  # the runner's stream, which starts the runs
        prho, pT = guard_prediction(prho, pT, r.rho_v, r.rho_l, r.T0)
    prho, dmass = match_mass(r, rho0, prho, pT)
    warm, wlast, t_warm = coexistence_times(r, prho.contiguous(), steps, every, final=final, start_T=pT.contiguous())
    r.close()
    finite = [i for i in range(len(specs)) if all(np.isfinite(v[i]) for v in (final[0], final[1], wlast[0], wlast[1]))]
    dev = {i: max(abs(wlast[0][i] - final[0][i]) / final[0][i], abs(wlast[1][i] - final[1][i]) / final[1][i])
           for i in finite}
    same = [i for i in finite if dev[i] <= 1e-3 and plain[i] is not None and warm[i] is not None]
    p = np.array([plain[i] for i in same], dtype=float)
    w = np.array([warm[i] for i in same], dtype=float)
    return {
        "problems": len(specs), "plain_converged": sum(v is not None for v in plain),
        "same_final_state": len(same), "other_final_state": sum(1 for i in finite if dev[i] > 1e-3),
        "plain_steps_median": float(np.median(p)) if len(p) else None,
        "warm_steps_median": float(np.median(w)) if len(w) else None,
        "plain_steps_mean": float(p.mean()) if len(p) else None,
        "warm_steps_mean": float(w.mean()) if len(w) else None,
        "faster_fraction": float((w < p).mean()) if len(p) else None,
        "speedup_of_means": float(p.mean() / w.mean()) if len(w) and w.mean() > 0 else None,
        "inference_seconds": t_inf, "plain_step_seconds": t_plain, "warm_step_seconds": t_warm,
        "warm_final_rel_dev_median": float(np.median(list(dev.values()))) if dev else None,
        "warm_final_rel_dev_max": float(max(dev.values())) if dev else None,
        "start_mass_offset_max": float(dmass.max()),
        "per_problem": [{"plain": plain[i], "warm": warm[i], "rho_l": float(final[0][i]), "rho_v": float(final[1][i]),
                         "warm_rho_l": float(wlast[0][i]), "warm_rho_v": float(wlast[1][i]), "tr": specs[i].tr}
                        for i in range(len(specs))],
    }


def _mse_fields(rho, T, rho_ref, T_ref, rho_v, rho_l, T0, theta_scale=0.1, outputs=2):
    """Per-problem mean squared difference of the normalised fields (the network's loss)."""
    sc = (rho_l - rho_v)[:, None, None]
    e = ((rho - rho_ref) / sc) ** 2
    e = e.mean(dim=(1, 2))
    if outputs > 1:
        e = 0.5 * (e + (((T - T_ref) / T0[:, None, None] / theta_scale) ** 2).mean(dim=(1, 2)))
    return e


def equal_error_steps(net, specs, horizon: int, every: int, log=None):
    """Steps the warm start saves at equal error: for each problem, the number of plain
    solver steps from the initial field after which the state is as close to the
    horizon state (normalised mean squared difference of density and temperature) as
    the state the solver would start from is (the network's prediction, guarded and put
    back on the initial mass); linear interpolation between samples every `every`
    steps.  Returns a summary with the per-problem values."""
    import torch
    r = Runner(specs)
    rho0 = r.initial_density()
    T0f = r.uniform_T()
    r.set_fields(rho0)
    r.step(horizon)
    rhoT, TT = r.fields()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prho, pT = net.predict_fields(rho0, T0f, r.rho_v, r.rho_l, r.T0, r.cond)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    # score the state the solver would start from: guarded, with the initial mass
    with torch.cuda.stream(r.stream):
        prho, pT = guard_prediction(prho, pT, r.rho_v, r.rho_l, r.T0)
    prho, _ = match_mass(r, rho0, prho, pT)
    ek = dict(rho_v=r.rho_v, rho_l=r.rho_l, T0=r.T0, outputs=net.K)
    e_net = _mse_fields(prho, pT, rhoT, TT, **ek).cpu().numpy()
    r.set_fields(rho0)
    curve = [(0, _mse_fields(rho0, T0f, rhoT, TT, **ek).cpu().numpy())]
    t_step = 0.0
    for s in range(every, horizon + 1, every):
        t1 = time.perf_counter()
        r.step(every)
        r.stream.synchronize()
        t_step += time.perf_counter() - t1
        rho, T = r.fields()
        curve.append((s, _mse_fields(rho, T, rhoT, TT, **ek).cpu().numpy()))
    r.close()
    steps = np.array([c[0] for c in curve], dtype=float)
    errs = np.stack([c[1] for c in curve])  # [samples, problems]
    saved = []
    for i in range(len(specs)):
        e = errs[:, i]
        hit = np.nonzero(e <= e_net[i])[0]
        if len(hit) == 0:
            saved.append(0.0)
            continue
        k = hit[0]
        if k == 0:
            saved.append(0.0)  # no better than the initial field
            continue
        # interpolate in log error between the samples around the crossing
        a, b_ = np.log(max(e[k - 1], 1e-30)), np.log(max(e[k], 1e-30))
        f = (np.log(max(e_net[i], 1e-30)) - a) / (b_ - a) if b_ != a else 1.0
        saved.append(float(steps[k - 1] + f * (steps[k] - steps[k - 1])))
    saved = np.array(saved)
    step_s = t_step / horizon  # seconds per batched step of all problems together
    return {
        "problems": len(specs), "horizon": horizon,
        "net_mse_median": float(np.median(e_net)), "no_change_mse_median": float(np.median(errs[0])),
        "steps_saved_median": float(np.median(saved)), "steps_saved_mean": float(saved.mean()),
        "fraction_of_horizon_median": float(np.median(saved) / horizon),
        "seconds_saved_mean": float(saved.mean() * step_s), "inference_seconds": t_inf,
        "per_problem_steps_saved": [round(float(v), 1) for v in saved],
    }
