"""Pins for oracle/thermo.py against what the paper and the mathematics fix.

None of these re-types the formula under test: each compares against a printed
number, a closed form derived independently, or a different route to the same
quantity (quadrature instead of a closed-form antiderivative, etc.).
"""
import mpmath as mp
import pytest

from oracle import thermo


def test_cs_coefficients_match_paper(golden):
    g = golden["cs_coefficients"]
    assert float(thermo.CS_A_COEF) == g["a_coef"]
    assert float(thermo.CS_B_COEF) == g["b_coef"]


@pytest.mark.parametrize("eos", [thermo.paper_cs_eos(), thermo.vdw_eos()], ids=["cs", "vdw"])
def test_critical_point_is_an_inflection_with_zero_slope(eos):
    """At (rho_c, Tc): dp/drho = d2p/drho2 = 0 and p = pc (Eq. (17) definitions of a~, b~)."""
    Tc, pc, rc = thermo.critical_point(eos)
    # the CS coefficients are printed to 16 digits, which bounds how exact the inflection is
    scale = eos.K_eos * eos.R * Tc
    assert abs(thermo.dp_drho(eos, rc, Tc)) < 1e-14 * scale
    assert abs(thermo.d2p_drho2(eos, rc, Tc)) < 1e-14 * scale / rc
    # p(rho_c, Tc) must reproduce pc given by the a~ / b~ definitions; the printed
    # 16-digit coefficients bound the agreement
    assert abs(thermo.pressure(eos, rc, Tc) / pc - 1) < 1e-14


def test_vdw_critical_closed_forms():
    # a = 9/49 and b = 2/21 enter as binary64 numbers, which bounds the agreement
    Tc, pc, rc = thermo.critical_point(thermo.vdw_eos())
    assert abs(Tc / (mp.mpf(4) / 7) - 1) < 1e-15
    assert abs(rc / (mp.mpf(7) / 2) - 1) < 1e-15
    assert abs(pc / (mp.mpf(3) / 4) - 1) < 1e-15


@pytest.mark.parametrize("eos", [thermo.paper_cs_eos(), thermo.vdw_eos()], ids=["cs", "vdw"])
def test_chemical_potential_is_antiderivative_of_dp_over_rho(eos):
    """mu(r2) - mu(r1) = integral (1/rho) dp/drho drho, by quadrature of the pressure's derivative."""
    Tc, _, rc = thermo.critical_point(eos)
    T = mp.mpf("0.8") * Tc
    for r1, r2 in [(rc * mp.mpf("0.1"), rc * mp.mpf("0.5")), (rc * mp.mpf("0.7"), rc * mp.mpf("2.2"))]:
        lhs = thermo.chemical_potential(eos, r2, T) - thermo.chemical_potential(eos, r1, T)
        rhs = mp.quad(lambda r: thermo.dp_drho(eos, r, T) / r, [r1, r2])
        assert abs(lhs - rhs) < mp.mpf(10) ** -20 * (1 + abs(lhs))


@pytest.mark.parametrize("eos", [thermo.paper_cs_eos(), thermo.vdw_eos()], ids=["cs", "vdw"])
@pytest.mark.parametrize("Tr", ["0.6", "0.8", "0.95"])
def test_maxwell_equal_area_in_specific_volume(eos, Tr):
    """Equal-area rule: integral_{v_l}^{v_v} (p(v) - p_s) dv = 0 with v = 1/rho, by quadrature;
    plus p(rho_v) = p(rho_l) = p_s and rho_v < rho_c < rho_l."""
    Tc, _, rc = thermo.critical_point(eos)
    T = mp.mpf(Tr) * Tc
    rv, rl, ps = thermo.maxwell(eos, T)
    assert rv < rc < rl
    assert abs(thermo.pressure(eos, rl, T) - ps) < mp.mpf(10) ** -30
    area = mp.quad(lambda v: thermo.pressure(eos, 1 / v, T) - ps, mp.linspace(1 / rl, 1 / rv, 12))
    scale = ps * (1 / rv - 1 / rl)
    assert abs(area) < mp.mpf(10) ** -20 * scale


def test_paper_sigma_and_width_from_printed_scaling_factors(golden):
    """(K_EOS, K_INT) = (0.479820, 2.294922) give sigma = 0.01 and W = 10 (P1).

    sigma is the square-gradient tension of the pressure tensor Eq. (11) with
    kappa = G^2 dx^4 / 4 (Eq. (16)) and G of Eq. (18); W is the 5%-95% width of the
    flat equilibrium profile (reading: the paper does not define W).  The factors are
    printed to 6 decimals, which bounds the agreement: sigma to 1.2e-6 and W to 2.2e-7
    relative."""
    g = golden["sigma_W_scaling"]
    eos = thermo.paper_cs_eos()
    eos.K_eos = g["K_eos"]
    d = thermo.derive(eos, thermo.Params(K_int=g["K_int"]))
    sigma = thermo.surface_tension(eos, d.T0, d.kappa)
    W = thermo.interface_width(eos, d.T0, d.kappa)
    assert abs(sigma / g["sigma"] - 1) < 1.5e-6
    assert abs(W / g["W"] - 1) < 3e-7


def test_sigma_and_width_scale_as_stated():
    """sigma proportional to K_EOS K_INT and W proportional to K_INT (text after Eq. (19))."""
    base = thermo.paper_cs_eos()
    d0 = thermo.derive(base, thermo.Params())
    s0 = thermo.surface_tension(base, d0.T0, d0.kappa)
    w0 = thermo.interface_width(base, d0.T0, d0.kappa)
    e2 = thermo.paper_cs_eos()
    e2.K_eos = base.K_eos * 1.7
    d2 = thermo.derive(e2, thermo.Params(K_int=2.294922 * 0.6))
    s2 = thermo.surface_tension(e2, d2.T0, d2.kappa)
    w2 = thermo.interface_width(e2, d2.T0, d2.kappa)
    # the factors enter as binary64 numbers, which bounds the agreement
    assert abs(s2 / s0 / (1.7 * 0.6) - 1) < 1e-14
    assert abs(w2 / w0 / 0.6 - 1) < 1e-14


def test_time_step_reproduces_fig1_snapshot_times(golden):
    """P2: with c_s of Eq. (19) at the Maxwell liquid density, c = sqrt(3) c_s and dt = dx / c,
    the Fig. 1 snapshot times are exactly 1, 2, 3, 4 x 10^7 steps (to the 3 printed digits)."""
    d = thermo.derive(thermo.paper_cs_eos(), thermo.Params())
    for n, printed in enumerate(golden["stefan_figure_times"]["times_1e7"], start=1):
        assert round(n * d.dt, 3) == printed
    # and the neighbouring readings do not: c = c_s (no sqrt 3) or c_s at rho_v
    assert round(1 * d.dt * 3 ** 0.5, 3) != 0.401


def test_stefan_root_small_ste_limit():
    """For Ste -> 0, Eq. (21) gives k ~ sqrt(Ste / 2) (erf k ~ 2k/sqrt(pi), exp k^2 ~ 1).
    One order further, sqrt(pi) k exp(k^2) erf(k) = 2k^2 + (4/3) k^4 + O(k^6), so
    k = sqrt(Ste / 2) (1 - Ste / 6) + O(Ste^(5/2)); the root found must agree to that
    order at every small Ste (measured remainder 0.064 Ste^2 relative)."""
    for ste in (1e-4, 1e-3, 0.005, 0.02):
        k = thermo.stefan_root(ste)
        assert abs(k / (ste / 2) ** 0.5 - 1) < 2 * ste
        assert abs(k / ((ste / 2) ** 0.5 * (1 - ste / 6)) - 1) < 0.1 * ste ** 2
    assert thermo.stefan_root(0.05) > thermo.stefan_root(0.005)


def test_latent_heat_matches_clapeyron():
    """h_lv of the text after Eq. (11) equals T (v_v - v_l) dp_s/dT (Clausius-Clapeyron),
    computed by differentiating the Maxwell pressure in T."""
    eos = thermo.paper_cs_eos()
    d = thermo.derive(eos, thermo.Params(K_int=1.0))   # with K_INT = 1 the mean-field a is K_EOS a~
    T0 = mp.mpf(d.T0)
    h = mp.mpf(10) ** -12
    dps = (thermo.maxwell(eos, T0 + h)[2] - thermo.maxwell(eos, T0 - h)[2]) / (2 * h)
    rv, rl, _ = thermo.maxwell(eos, T0)
    clapeyron = T0 * (1 / rv - 1 / rl) * dps
    assert abs(d.h_lv / float(clapeyron) - 1) < 1e-9


def test_derived_relaxation_rates_give_paper_transport():
    """tau_e, tau_q from the constraints make the bulk/shear relation of the text after Eq. (15)
    consistent: nu = c_s^2 dt tau_p and the constraint tau_p tau_q = 1/12 holds for s_p = 1."""
    d = thermo.derive(thermo.paper_cs_eos(), thermo.Params())
    assert d.s_p == 1.0
    assert abs(d.s_q - 1.5) < 1e-15          # tau_q = 1/6
    assert abs(d.s_e - 22.0 / 17.0) < 1e-15   # tau_e = 3/11 with k = 5/6
    assert abs(d.beta + 2.4) < 1e-15
