"""Precision form: populations stored in 16 bits (FP16 or BF16 deviations from the rest
equilibrium of one reference state, the vapour coexistence density at T0), FP32
arithmetic.  Every result is reported against the FP64 oracle; the bars are the measured
accuracy of each storage format with margin, not a claim of FP32-level parity:
  96x80 droplet, 1000 steps: FP16 rho 6.8e-3, T 1.1e-2; BF16 rho 4.7e-2, T 5.9e-2
  64x64 slab, 2000 steps, bulk densities: FP16 rho_l 9.2e-3, rho_v 5.2e-2;
                                          BF16 rho_l 3.3e-2, rho_v 8.7e-2
Rounding to nearest is deterministic, so in a nearly steady state each step rounds the
same values the same way and the errors add up instead of averaging out."""
import numpy as np
import pytest

from paper_2106_01557_amd import inputs
from tests.parity_helpers import assert_close, errors, gpu_moments, oracle_model, oracle_moments, say

pytestmark = pytest.mark.gpu

# bars per storage format (normalised max errors, see parity_helpers.errors)
BARS = {"f32": 1e-5, "f16": 3e-2, "bf16": 1.5e-1}


@pytest.fixture(scope="module")
def droplet_case():
    model = oracle_model("cs", {"Tr0": 0.75})
    d = model.d
    f = inputs.droplet(96, 80, d.rho_l, d.rho_v, d.T0, 20, 4, eps=0.005, seed=1)
    o, _ = oracle_moments(model, f, 1000)
    return model, f, o


@pytest.mark.parametrize("prec,rounding", [("f32", "nearest"), ("f16", "nearest"), ("bf16", "nearest"),
                                            ("f16", "stochastic"), ("bf16", "stochastic")])
def test_16bit_storage_error_vs_fp64_oracle(droplet_case, prec, rounding):
    model, f, o = droplet_case
    d = model.d
    say(f"case: {prec} storage ({rounding} rounding) AB 96x80 droplet, 1000 steps vs FP64 oracle")
    params = {"precision": prec, "Tr0": 0.75}
    if rounding != "nearest":
        params["rounding"] = rounding
    g, s = gpu_moments(96, 80, f, 1000, params=params)
    inv = s.invariants()
    assert inv["bad_nodes"] == 0
    assert_close(g, o, d, BARS[prec], f"{prec} storage ({rounding}) droplet")


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_16bit_storage_keeps_uniform_state_nearly_steady(prec):
    """A uniform rest state at the reference state is stored exactly (zero deviations)."""
    model = oracle_model("cs")
    d = model.d
    rho0 = d.rho_v
    say(f"case: {prec} uniform state at the reference density")
    f = inputs.uniform(64, 32, rho0, d.T0)
    g, _ = gpu_moments(64, 32, f, 50, params={"precision": prec})
    assert np.allclose(g["rho"], rho0, rtol=1e-6, atol=0)
    assert np.abs(g["ux"]).max() < 1e-7 and np.abs(g["uy"]).max() < 1e-7


@pytest.fixture(scope="module")
def slab_case():
    model = oracle_model("cs")
    d = model.d
    f = inputs.slab(64, 64, d.rho_l, d.rho_v, d.T0, 16, 47, eps=0.01, seed=0)
    o, _ = oracle_moments(model, f, 2000)
    return model, f, o


def _bulk(m):
    """Row-mean densities at the slab centre (between rows 31 and 32) and half a period
    away in the vapour (between rows 63 and 0)."""
    r = m["rho"].mean(axis=1)
    return 0.5 * (r[31] + r[32]), 0.5 * (r[63] + r[0])


@pytest.mark.parametrize("prec,bar_l,bar_v", [("f16", 2e-2, 1e-1), ("bf16", 6e-2, 1.5e-1)])
def test_16bit_storage_coexistence_densities_vs_fp64_oracle(slab_case, prec, bar_l, bar_v):
    """Flat-slab coexistence with 16-bit storage: the bulk liquid and vapour densities
    after 2000 steps against the FP64 oracle's, as relative errors."""
    model, f, o = slab_case
    say(f"case: {prec} storage AB 64x64 slab, 2000 steps, bulk densities vs FP64 oracle")
    g, s = gpu_moments(64, 64, f, 2000, params={"precision": prec})
    assert s.invariants()["bad_nodes"] == 0
    (lo, vo), (lg, vg) = _bulk(o), _bulk(g)
    el, ev = abs(lg / lo - 1), abs(vg / vo - 1)
    say(f"  oracle rho_l {lo:.7f} rho_v {vo:.7f}; {prec} rho_l {lg:.7f} ({el:.2e}) rho_v {vg:.7f} ({ev:.2e})")
    assert el <= bar_l and ev <= bar_v


@pytest.mark.parametrize("prec,bar_l,bar_v", [("f16", 2e-3, 2e-3), ("bf16", 1e-2, 1e-2)])
def test_stochastic_rounding_coexistence_densities_vs_fp64_oracle(slab_case, prec, bar_l, bar_v):
    """The same slab with stochastic rounding of the 16-bit stores: rounding up with
    probability equal to the discarded fraction removes the bias that rounding to
    nearest accumulates in a nearly steady state."""
    model, f, o = slab_case
    say(f"case: {prec} storage, stochastic rounding, AB 64x64 slab, 2000 steps, bulk densities vs FP64 oracle")
    g, s = gpu_moments(64, 64, f, 2000, params={"precision": prec, "rounding": "stochastic"})
    assert s.invariants()["bad_nodes"] == 0
    (lo, vo), (lg, vg) = _bulk(o), _bulk(g)
    el, ev = abs(lg / lo - 1), abs(vg / vo - 1)
    e = errors(g, o, model.d)
    say(f"  oracle rho_l {lo:.7f} rho_v {vo:.7f}; {prec} sr rho_l {lg:.7f} ({el:.2e}) rho_v {vg:.7f} ({ev:.2e}); "
        f"max errors {e}")
    assert el <= bar_l and ev <= bar_v


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_stochastic_rounding_is_deterministic_across_forms_and_restarts(droplet_case, prec):
    """The random bits are a hash of the step count and the node, so: two runs agree
    bitwise; the one- and two-column kernel forms agree bitwise (ragged 70x45 and the
    96x80 droplet); a state saved and restored continues bitwise as if never stopped;
    and the result is not that of rounding to nearest."""
    model, f, _ = droplet_case
    d = model.d
    say(f"case: {prec} stochastic rounding determinism, forms, restart")
    base = {"precision": prec, "Tr0": 0.75, "rounding": "stochastic", "rows_per_wave": 16}
    a, _ = gpu_moments(96, 80, f, 300, params=base)
    b, _ = gpu_moments(96, 80, f, 300, params={**base, "columns_per_lane": 1})
    for k in a:
        assert np.array_equal(a[k], b[k]), ("forms", k)
    c, _ = gpu_moments(96, 80, f, 300, params=base)
    for k in a:
        assert np.array_equal(a[k], c[k]), ("rerun", k)
    r, _ = gpu_moments(96, 80, f, 300, params={**base, "rounding": "nearest"})
    assert not np.array_equal(a["rho"], r["rho"])
    g = inputs.random_smooth(70, 45, 0.5 * (d.rho_l + d.rho_v), d.T0, 0.4, 0.04 * d.cs, 0.04, seed=5)
    x, _ = gpu_moments(70, 45, g, 40, params=base)
    y, _ = gpu_moments(70, 45, g, 40, params={**base, "columns_per_lane": 1})
    for k in x:
        assert np.array_equal(x[k], y[k]), ("ragged forms", k)
    from tests.parity_helpers import gpu_solver
    s = gpu_solver(96, 80, params=base)
    s.set_fields(*f.as_tuple())
    s.step(131)
    blob, steps = s.save_state()
    s.step(69)
    want = s.moments_numpy()
    s2 = gpu_solver(96, 80, params=base)
    s2.load_state(blob, steps)
    s2.step(69)
    got = s2.moments_numpy()
    for k in got:
        assert np.array_equal(got[k], want[k]), ("restart", k)


@pytest.mark.parametrize("prec", ["f16", "bf16"])
@pytest.mark.parametrize("nx", [70, 69])
def test_16bit_generic_addressing_path_matches_buffer_path(droplet_case, monkeypatch, prec, nx):
    """The 64-bit addressing path (taken by lattices past the 32-bit buffer-offset range;
    LBM_GENERIC_ADDRESSING=1 forces it) with 16-bit storage, both roundings, in the
    two-column (nx = 70) and one-column (nx = 69) forms, against the buffer path.  The
    paths are compiled separately, so an FP32 result may differ in its last bit and then
    round to the neighbouring 16-bit value: the bar is a few 16-bit steps, far below the
    storage error against the oracle (measured: the two paths agree bitwise)."""
    model, _, _ = droplet_case
    d = model.d
    f = inputs.random_smooth(nx, 45, 0.5 * (d.rho_l + d.rho_v), d.T0, 0.4, 0.04 * d.cs, 0.04, seed=nx)
    for rounding in ("nearest", "stochastic"):
        say(f"case: {prec} {rounding} rounding, generic vs buffer addressing, {nx}x45, 40 steps")
        params = {"precision": prec, "Tr0": 0.75, "rows_per_wave": 8, "rounding": rounding}
        monkeypatch.delenv("LBM_GENERIC_ADDRESSING", raising=False)
        a, _ = gpu_moments(nx, 45, f, 40, params=params)
        monkeypatch.setenv("LBM_GENERIC_ADDRESSING", "1")
        b, s = gpu_moments(nx, 45, f, 40, params=params)
        monkeypatch.delenv("LBM_GENERIC_ADDRESSING")
        assert s.invariants()["bad_nodes"] == 0
        e = errors(a, b, d)
        say(f"  paths differ by {e}")
        assert max(e.values()) <= (2e-3 if prec == "f16" else 1e-2)


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_16bit_storage_aa_scheme_vs_fp64_oracle(droplet_case, prec):
    """The in-place AA scheme with 16-bit storage (density pass, then the in-place
    collide-stream, both through the per-value conversions) meets the same bars as the
    two-buffer form against the FP64 oracle."""
    model, f, o = droplet_case
    say(f"case: {prec} storage AA 96x80 droplet, 1000 steps vs FP64 oracle")
    g, s = gpu_moments(96, 80, f, 1000, params={"precision": prec, "Tr0": 0.75, "scheme": "aa"})
    assert s.invariants()["bad_nodes"] == 0
    assert_close(g, o, model.d, BARS[prec], f"{prec} storage AA droplet")
