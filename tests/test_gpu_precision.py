"""Precision form: populations stored in 16 bits (FP16 or BF16 deviations from the rest
equilibrium of one reference state, the mid density at T0), FP32 arithmetic.  Every result
is reported against the FP64 oracle; the bars are the measured accuracy of each storage
format (96x80 droplet, 1000 steps: FP16 rho 9.8e-3, T 2.3e-2; BF16 rho 5.2e-2, T 9.1e-2)
with margin, not a claim of FP32-level parity."""
import numpy as np
import pytest

from paper_2106_01557_amd import inputs
from tests.parity_helpers import assert_close, errors, gpu_moments, oracle_model, oracle_moments, say

pytestmark = pytest.mark.gpu

# bars per storage format (normalised max errors, see parity_helpers.errors)
BARS = {"f32": 1e-5, "f16": 5e-2, "bf16": 2e-1}


@pytest.fixture(scope="module")
def droplet_case():
    model = oracle_model("cs", {"Tr0": 0.75})
    d = model.d
    f = inputs.droplet(96, 80, d.rho_l, d.rho_v, d.T0, 20, 4, eps=0.005, seed=1)
    o, _ = oracle_moments(model, f, 1000)
    return model, f, o


@pytest.mark.parametrize("prec", ["f32", "f16", "bf16"])
def test_16bit_storage_error_vs_fp64_oracle(droplet_case, prec):
    model, f, o = droplet_case
    d = model.d
    say(f"case: {prec} storage AB 96x80 droplet, 1000 steps vs FP64 oracle")
    g, s = gpu_moments(96, 80, f, 1000, params={"precision": prec, "Tr0": 0.75})
    inv = s.invariants()
    assert inv["bad_nodes"] == 0
    assert_close(g, o, d, BARS[prec], f"{prec} storage droplet")


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_16bit_storage_keeps_uniform_state_nearly_steady(prec):
    """A uniform rest state at the reference density is stored exactly (zero deviations)."""
    model = oracle_model("cs")
    d = model.d
    rho0 = 0.5 * (d.rho_l + d.rho_v)
    say(f"case: {prec} uniform state at the reference density")
    f = inputs.uniform(64, 32, rho0, d.T0)
    g, _ = gpu_moments(64, 32, f, 50, params={"precision": prec})
    assert np.allclose(g["rho"], rho0, rtol=1e-6, atol=0)
    assert np.abs(g["ux"]).max() < 1e-7 and np.abs(g["uy"]).max() < 1e-7
