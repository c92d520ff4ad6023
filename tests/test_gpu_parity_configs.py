"""GPU parity on the workloads' own parity analogues, through the C ABI.

* The FP32 throughput workload scaled to what the oracle finishes: a 256 x 256 periodic
  droplet, R = 32, tanh width 4, T/Tc = 0.75, +-0.5 % noise (PCG64 seed 1), 1000 steps;
  FP32 within 1e-5 of the FP64 oracle.  The same run with 16-bit deviation storage (the
  precision form) reports its error against the same oracle run, under bars that hold the
  measured errors with margin (no parity claim: the 16-bit forms round the state).
* The flat-slab workload with K_INT = 1 (interface width 4.36 instead of 10, so the bulk
  of the 32-row slab is far from both interfaces): FP64 within 1e-12 after 1000 steps.
Norms: rho max |d rho| / rho_l, u max |d u| / c_s, T max |d T| / T0.
"""
import pytest

from paper_2106_01557_amd import inputs
from tests.parity_helpers import assert_close, errors, gpu_moments, oracle_model, oracle_moments, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def droplet256():
    model = oracle_model("cs", {"Tr0": 0.75})
    d = model.d
    say("case: oracle 256x256 droplet R=32 W=4 T/Tc 0.75, 1000 steps (FP64, CPU)")
    f = inputs.droplet(256, 256, d.rho_l, d.rho_v, d.T0, 32, 4, eps=0.005, seed=1)
    o, _ = oracle_moments(model, f, 1000)
    return model, f, o


def test_fp32_droplet_256_R32_1000_steps(droplet256):
    model, f, o = droplet256
    d = model.d
    say("case: FP32 AB 256x256 droplet R=32, 1000 steps")
    g, s = gpu_moments(256, 256, f, 1000, params={"precision": "f32", "Tr0": 0.75})
    assert s.invariants()["bad_nodes"] == 0
    assert_close(g, o, d, 1e-5, "fp32 droplet 256")


# (rho, u, T) bars of the 16-bit forms on this run; measured errors are printed
BARS16 = {("f16", "nearest"): (3e-2, 1e-2, 3e-2), ("f16", "stochastic"): (2e-2, 5e-3, 2e-2),
          ("bf16", "nearest"): (5e-1, 5e-2, 2.5e-1), ("bf16", "stochastic"): (1e-1, 2e-2, 1e-1)}


@pytest.mark.parametrize("prec,rounding", list(BARS16), ids=lambda v: str(v))
def test_16bit_droplet_256_error_against_oracle(droplet256, prec, rounding):
    model, f, o = droplet256
    d = model.d
    say(f"case: {prec}/{rounding} AB 256x256 droplet R=32, 1000 steps, error vs FP64 oracle")
    g, s = gpu_moments(256, 256, f, 1000, params={"precision": prec, "rounding": rounding, "Tr0": 0.75})
    assert s.invariants()["bad_nodes"] == 0
    e = errors(g, o, d)
    say(f"  {prec}/{rounding} errors {e}")
    br, bu, bT = BARS16[(prec, rounding)]
    assert e["rho"] <= br and max(e["ux"], e["uy"]) <= bu and e["T"] <= bT, e


def test_fp64_flat_slab_kint1_1000_steps():
    model = oracle_model("cs", {"K_int": 1.0})
    d = model.d
    say("case: FP64 AB 64x64 slab, K_INT = 1, 1000 steps")
    f = inputs.slab(64, 64, d.rho_l, d.rho_v, d.T0, 16, 47, eps=0.01, seed=0)
    g, s = gpu_moments(64, 64, f, 1000, params={"precision": "f64", "K_int": 1.0})
    o, _ = oracle_moments(model, f, 1000)
    assert s.invariants()["bad_nodes"] == 0
    assert_close(g, o, d, 1e-12, "fp64 slab K_INT=1")
