"""Pins of the oracle's update against the macroscopic equations the paper recovers, for
terms that only show at the hydrodynamic level, and of the potential-energy diagnostic
against its mean-field limits.

* Linear hydrodynamic modes.  A small sound or temperature wave on a uniform liquid or
  vapour must evolve as the linearised conservation equations (Eq. (6)) say, with the
  transport coefficients stated after Eq. (15) (kinematic viscosity nu, bulk viscosity
  varsigma, heat conductivity lambda), the equation of state of Eq. (17), the
  square-gradient coefficient kappa of the pressure tensor (Eq. (11), kappa from
  Eq. (16)) and the energy equation written for rho e_k with the enthalpy flux
  rho h_k u = (rho e_k + p_BE) u.  Nothing here uses the lattice formulas: the linear
  equations are integrated exactly (matrix exponential per Fourier mode) and the EOS
  derivatives come from the arbitrary-precision thermodynamics.  The differences are the
  lattice's higher-order terms, so they shrink as k^2 when the wavelength doubles; a
  wrong term of the recovered equations would not shrink that way.  This is what fixes
  the heat-flux rows of n^eq (SM Eq. (4a)): their equilibrium enters the energy flux
  through the coupling sigma_q omega_j of L (SM Eq. (5b)), and with rho e_k in place of
  rho h_k the liquid's sound wave is off by 1 % where the lattice leaves 0.1 %.
* The compensation term S Q_m of Eq. (12b) (SM Eq. (6a)).  The text after Eq. (15) says
  that it adds R_add = -(G^2 dx^4/24) div[2 grad rho grad rho + |grad rho|^2 I] to the
  force.  Adding S Q_m after the collision is the same as relaxing towards m^eq + Q_m,
  so the momentum flux gains the second moments of M^-1 Q_m, which must therefore be
  (G^2 dx^4/24)(2 grad rho grad rho + |grad rho|^2 I), with no mass, momentum or heat flux.
  That fixes the e, p_xx and p_xy rows.  The eps row (a fourth-order moment) enters the
  macroscopic equations only beyond the order of the paper's analysis; the printed vector
  has the structure of a second-order Hermite population set, like the u^2 terms of m^eq,
  and that structure is pinned here as such.
* The density gradient in Q_m comes from F_pair (closing remark of the SM), so it must be
  the gradient of the density whatever external acceleration acts.
* The potential-energy diagnostic (a reading; the paper defines no discrete E_p): for a
  uniform density it is exactly -a rho^2 per node with a = G^2 dx^2/2 (Eq. (16): the
  attraction whose pressure is the -a rho^2 of p_EOS = p_BE - a rho^2), and for a slow
  wave the excess over that is (kappa/2) sum |grad rho|^2, the square-gradient energy
  of the same pressure tensor.

The mutation tests at the end plant, one at a time, slips that passed every other CPU
pin (the heat-flux rows of n^eq with rho e_k, the eps or p_xy coefficient of Q_m, the
gradient taken from the total force) and show that a pin here fails for each.
"""
import dataclasses

import mpmath as mp
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import lbm, thermo


@pytest.fixture(scope="module")
def model():
    return lbm.Model.build(thermo.paper_cs_eos(), thermo.Params())


# --- 1. linear hydrodynamic modes ---------------------------------------------------------------

def linear_generator(model, rho0, tau_j, ny):
    """d/dt of the Fourier amplitudes (rho', u_y', T') of mode exp(2 pi i y / ny) for the
    conservation equations (Eq. (6)) linearised about rest at (rho0, T0):
        d rho'/dt = -i k rho0 u'
        rho0 du'/dt = -i k [p_rho rho' + p_T T' + kappa rho0 k^2 rho'] - rho0 (nu + varsigma) k^2 u'
        rho0 c_v dT'/dt = -i k p_BE u' - lambda k^2 T'
    (Pi_yy = rho (nu + varsigma) du/dy for u = u(y) e_y; the energy line is Eq. (6c) minus
    e_k times the continuity equation, rho e_k = rho c_v T to first order)."""
    d, p = model.d, model.params
    k = 2 * np.pi / (ny * p.dx)
    T0 = mp.mpf(d.T0)
    p_rho = float(mp.diff(lambda r: thermo.pressure(model.eos, r, T0), mp.mpf(rho0)))
    p_T = float(mp.diff(lambda t: thermo.pressure(model.eos, mp.mpf(rho0), t), T0))
    p_be = float(thermo.pressure(model.eos, rho0, T0)) + d.a_mf * rho0 * rho0
    cs2 = d.c ** 2 / 3
    nu = cs2 * d.dt * (1 / d.s_p - 0.5)
    zeta = p.varpi * cs2 * d.dt * (1 / d.s_e - 0.5)
    lam = (4 + 3 * p.gamma1 + 2 * p.gamma2) / 6 * d.C_ref * d.c ** 2 * d.dt * tau_j
    return np.array([
        [0, -1j * k * rho0, 0],
        [-1j * k * (p_rho + d.kappa * rho0 * k * k) / rho0, -(nu + zeta) * k * k, -1j * k * p_T / rho0],
        [0, -1j * k * p_be / (rho0 * d.cv), -lam * k * k / (rho0 * d.cv)],
    ])


def _amplitudes(model, st, ny):
    rho, _, uy, T = lbm.moments(model, st)
    e = np.exp(-2j * np.pi * np.arange(ny) / ny) * 2 / ny
    return np.array([np.sum(rho[:, 0] * e), np.sum(uy[:, 0] * e), np.sum(T[:, 0] * e)])


def mode_errors(model, phase, kind, ny, amp=1e-4, t0=20):
    """Per-field |lattice - linear theory| / max(|lattice|, |theory|) of the mode's
    amplitudes after 3 ny steps, the theory started from the lattice's amplitudes at step t0
    (after the initial state's own transient).  `kind` "sound": density wave at uniform T;
    "thermal": temperature wave at uniform density (which also launches sound)."""
    d = model.d
    rho0, tau_j = (d.rho_l, d.tau_j_l) if phase == "liquid" else (d.rho_v, d.tau_j_v)
    s = np.sin(2 * np.pi * np.arange(ny, dtype=float) / ny)[:, None]
    if kind == "sound":
        rho, T = rho0 * (1 + amp * s), d.T0 + 0 * s
    else:
        rho, T = rho0 + 0 * s, d.T0 * (1 + amp * s)
    st = lbm.run(model, lbm.init_state(model, rho, 0 * rho, 0 * rho, T), t0)
    a0 = _amplitudes(model, st, ny)
    steps = 3 * ny
    a1 = _amplitudes(model, lbm.run(model, st, steps), ny)
    pred = sl.expm(linear_generator(model, rho0, tau_j, ny) * steps * d.dt) @ a0
    return np.abs(a1 - pred) / np.maximum(np.abs(a1), np.abs(pred))


# (phase, kind): bar on (rho', u', T') at 128 nodes per wavelength; measured 1.2e-3,
# 3.7e-4, 1.1e-4 for the liquid's sound wave, <= 3e-4 in the vapour.  The liquid's
# temperature wave has decayed 400-fold by the end (lambda / (rho c_v) is large there), so
# its T' is compared at 1.5e-2 (measured 5.9e-3).
MODE_BARS = {
    ("liquid", "sound"): (3e-3, 3e-3, 3e-3),
    ("liquid", "thermal"): (3e-3, 3e-3, 1.5e-2),
    ("vapour", "sound"): (3e-3, 3e-3, 3e-3),
    ("vapour", "thermal"): (3e-3, 3e-3, 3e-3),
}


def check_modes(model, cases=MODE_BARS):
    for (phase, kind), bar in cases.items():
        err = mode_errors(model, phase, kind, 128)
        assert np.all(err < bar), (phase, kind, err)


def check_mode_convergence(model):
    """The liquid's sound wave: the worst field's error falls at least 3x (k^2 would give 4)
    when the wavelength doubles; measured 3.7x."""
    e128 = mode_errors(model, "liquid", "sound", 128).max()
    e256 = mode_errors(model, "liquid", "sound", 256).max()
    assert e128 / e256 > 3.0, (e128, e256)


def test_small_waves_follow_the_linearised_conservation_equations(model):
    check_modes(model)


def test_wave_errors_are_the_lattice_s_higher_order_terms(model):
    check_mode_convergence(model)


# --- 2. the compensation term Q_m ---------------------------------------------------------------

def _random_gradients(n=8, seed=7):
    rng = np.random.default_rng(seed)
    return rng.uniform(-0.05, 0.05, n), rng.uniform(-0.05, 0.05, n)


def check_compensation_stress(model):
    """Second moments of M^-1 Q_m = (G^2 dx^4/24)(2 grad rho grad rho + |grad rho|^2 I);
    zeroth, first and heat-flux moments zero."""
    d, dx = model.d, model.params.dx
    gx, gy = _random_gradients()
    pops = lbm.from_moments(lbm.q_comp(model, gx, gy))
    e = d.c * lbm.EF
    stress = np.einsum("ia,ib,i...->ab...", e, e, pops)
    g = np.stack([gx, gy])
    want = (d.G2 * dx ** 4 / 24) * (2 * np.einsum("a...,b...->ab...", g, g)
                                     + np.einsum("ab,...->ab...", np.eye(2), gx * gx + gy * gy))
    scale = np.abs(want).max()
    assert np.allclose(stress, want, rtol=0, atol=1e-13 * scale)
    mom = lbm.to_moments(pops)
    assert np.allclose(mom[[0, 3, 4, 5, 6]], 0, atol=1e-13 * np.abs(mom).max())


def check_compensation_hermite(model):
    """Q_m equals the moments of the second-order Hermite population set
    w_i (E_i E_i - theta I) : X / (2 theta^2) with theta = 1/3 and X its own lattice-unit
    stress: every row, the eps row included."""
    gx, gy = _random_gradients(seed=8)
    Q = lbm.q_comp(model, gx, gy)
    pops = lbm.from_moments(Q)
    X = np.einsum("ia,ib,i...->ab...", lbm.EF, lbm.EF, pops)
    th = 1.0 / 3.0
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    H = np.einsum("ia,ib->iab", lbm.EF, lbm.EF) - th * np.eye(2)[None]
    herm = w[:, None] * np.einsum("iab,ab...->i...", H, X) / (2 * th * th)
    assert np.allclose(lbm.to_moments(herm), Q, rtol=0, atol=1e-13 * np.abs(Q).max())


def test_compensation_term_carries_the_stress_of_R_add(model):
    check_compensation_stress(model)


def test_compensation_term_is_a_second_order_hermite_set(model):
    check_compensation_hermite(model)


def check_compensation_gradient(model, monkeypatch, nx=128):
    """A density wave rho_v (1 + 0.2 cos kx) under an external acceleration that would
    offset a force-based gradient by 1 % of its amplitude: the gradient handed to Q_m is
    -0.2 rho_v k sin kx within the O(k^2 dx^2 / 6) of the pair-force estimate."""
    d = model.d
    k = 2 * np.pi / nx
    amp = 0.2 * d.rho_v
    a = 0.01 * d.G2 * amp * k
    acc = lbm.Model.build(model.eos, dataclasses.replace(model.params, accel_x=a, accel_y=-a))
    x = np.arange(nx, dtype=float)[None, :]
    rho = d.rho_v + amp * np.cos(k * x)
    seen = {}
    orig = lbm.q_comp

    def spy(m, gx, gy):
        seen["g"] = (gx.copy(), gy.copy())
        return orig(m, gx, gy)

    monkeypatch.setattr(lbm, "q_comp", spy)
    lbm.collide(acc, lbm.init_state(acc, rho, 0 * rho, 0 * rho, 0 * rho + d.T0))
    gx, gy = seen["g"]
    want = -amp * k * np.sin(k * x)
    assert np.abs(gx - want).max() < 1e-3 * amp * k, np.abs(gx - want).max() / (amp * k)
    assert np.abs(gy).max() < 1e-3 * amp * k


def test_compensation_uses_the_density_gradient_under_acceleration(model, monkeypatch):
    check_compensation_gradient(model, monkeypatch)


# --- 3. the potential-energy diagnostic ---------------------------------------------------------

def test_potential_energy_has_its_mean_field_limits(model):
    d = model.d
    a = d.G2 * model.params.dx ** 2 / 2
    for rho0 in (d.rho_v, d.rho_l):
        rho = np.full((4, 6), rho0)
        st = lbm.init_state(model, rho, 0 * rho, 0 * rho, 0 * rho + d.T0)
        Ep = lbm.invariants(model, st)["E_p"]
        assert abs(Ep / (-a * rho0 * rho0 * rho.size) - 1) < 1e-14
    nx = 128
    k = 2 * np.pi / nx
    amp = 0.1 * d.rho_l
    x = np.arange(nx, dtype=float)[None, :]
    rho = d.rho_l + amp * np.cos(k * x)
    st = lbm.init_state(model, rho, 0 * rho, 0 * rho, 0 * rho + d.T0)
    excess = lbm.invariants(model, st)["E_p"] + a * np.sum(rho * rho)
    grad2 = np.sum((amp * k * np.sin(k * x)) ** 2)
    # the discrete excess is (kappa/2) sum |grad rho|^2 times 2(1 - cos k)/k^2 = 1 - k^2/12 + ...
    assert abs(excess / (d.kappa / 2 * grad2) - 1) < 1e-3


# --- 4. mutations: each planted slip fails a pin above ------------------------------------------

def test_mutation_heat_flux_rows_with_energy_instead_of_enthalpy(model, monkeypatch):
    """-rho e_k u-hat in place of -rho h_k u-hat in the q rows of n^eq."""
    orig = lbm.n_eq

    def bad(m, rho_ek, T, rho_hk, uxh, uyh):
        o = orig(m, rho_ek, T, rho_hk, uxh, uyh).copy()
        o[4], o[6] = -rho_ek * uxh, -rho_ek * uyh
        return o

    monkeypatch.setattr(lbm, "n_eq", bad)
    with pytest.raises(AssertionError):
        check_modes(model, {("liquid", "sound"): MODE_BARS[("liquid", "sound")]})


def _plant_q(monkeypatch, row, factor):
    orig = lbm.q_comp

    def bad(m, gx, gy):
        o = orig(m, gx, gy).copy()
        o[row] = factor * o[row]
        return o

    monkeypatch.setattr(lbm, "q_comp", bad)


def test_mutation_compensation_eps_row_halved(model, monkeypatch):
    _plant_q(monkeypatch, 2, 0.5)
    with pytest.raises(AssertionError):
        check_compensation_hermite(model)


def test_mutation_compensation_pxy_row_doubled(model, monkeypatch):
    _plant_q(monkeypatch, 8, 2.0)
    with pytest.raises(AssertionError):
        check_compensation_stress(model)


def test_mutation_gradient_from_the_total_force(model, monkeypatch):
    """grad rho taken from F = F_pair + rho a instead of F_pair."""
    orig = lbm.macros

    def bad(m, st):
        mac = orig(m, st)
        return dataclasses.replace(mac, Fpx=mac.Fx, Fpy=mac.Fy)

    monkeypatch.setattr(lbm, "macros", bad)
    with pytest.raises(AssertionError):
        check_compensation_gradient(model, monkeypatch)
