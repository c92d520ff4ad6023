"""Shared helpers for the GPU parity tests: run the oracle and the HIP library on
the same seeded inputs and compare their moments.

Error norms (reading: u is near zero in these workloads, so relative errors are
taken against the natural scales of each field):
  rho: max |d rho| / rho_l      u: max |d u| / c_s      T: max |d T| / T0
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

from oracle import lbm as olbm
from oracle import thermo

_LIB_ONLY = {"precision", "scheme", "rows_per_wave", "waves_per_block", "columns_per_lane", "rho_ref", "T_ref",
             "rounding"}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_model(eos_kind="cs", params=None):
    p = {k: v for k, v in (params or {}).items() if k not in _LIB_ONLY}
    e = thermo.paper_cs_eos() if eos_kind == "cs" else thermo.vdw_eos()
    return olbm.Model.build(e, thermo.Params(**p))


def oracle_moments(model, fields, steps):
    st = olbm.init_state(model, *fields.as_tuple())
    st = olbm.run(model, st, steps)
    rho, ux, uy, T = olbm.moments(model, st)
    return {"rho": rho, "ux": ux, "uy": uy, "T": T}, st


def gpu_solver(nx, ny, eos_kind="cs", params=None):
    from paper_2106_01557_amd import lbm
    eos = lbm.Eos() if eos_kind == "cs" else lbm.vdw_eos()
    return lbm.Solver(nx, ny, eos=eos, params=params)


def gpu_moments(nx, ny, fields, steps, eos_kind="cs", params=None, solver=None):
    s = solver or gpu_solver(nx, ny, eos_kind, params)
    s.set_fields(*fields.as_tuple())
    s.step(steps)
    return s.moments_numpy(), s


def errors(a: dict, b: dict, d) -> dict:
    return {
        "rho": float(np.abs(a["rho"] - b["rho"]).max() / d.rho_l),
        "ux": float(np.abs(a["ux"] - b["ux"]).max() / d.cs),
        "uy": float(np.abs(a["uy"] - b["uy"]).max() / d.cs),
        "T": float(np.abs(a["T"] - b["T"]).max() / d.T0),
    }


def assert_close(a, b, d, tol, label=""):
    e = errors(a, b, d)
    say(f"  {label} errors {e}")
    log = os.environ.get("PARITY_LOG")
    if log:
        with open(log, "a") as fh:
            fh.write(json.dumps({"case": label, "tol": tol, **e}) + "\n")
    bad = {k: v for k, v in e.items() if not (v <= tol)}
    assert not bad, f"{label}: {bad} > {tol}"
    return e


def patch(arr, cy, cx, half):
    """Periodic (2 half) x (2 half) window of a [ny, nx] array centred on (cy, cx)."""
    ny, nx = arr.shape[-2:]
    ys = (np.arange(cy - half, cy + half) % ny)[:, None]
    xs = (np.arange(cx - half, cx + half) % nx)[None, :]
    return arr[..., ys, xs]
