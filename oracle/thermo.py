"""Oracle thermodynamics and derived model constants, in arbitrary precision.

TEST INFRASTRUCTURE ONLY.  This module is part of the CPU oracle: only the test
suite, the package smoke check and the CPU-baseline leg of the benchmark may
import it.  The product library neither imports nor links anything here, and it
shares no code, tables or constants with it.

Everything is written from the paper (Huang, Wu & Adams, "Mesoscopic lattice
Boltzmann modeling of the liquid-vapor phase transition"):

* the full equation of state: Carnahan-Starling with an attractive term,
  Eq. (17), and the van der Waals form as the second kind;
* the interaction strength G, Eq. (18), and the lattice sound speed, Eq. (19);
* the closure p_BE = p_LBE, rho*h_k = rho*e_k + p_BE, a = G^2 dx^2/2 and
  kappa = G^2 dx^4/4, Eqs. (15)-(16), with p_EOS = p_BE - a rho^2 (text after
  Eq. (11));
* the relaxation-time constraints tau_p tau_q = (k+1) tau_e tau_q = 1/12 of the
  Supplemental Material (after SM Eq. (5b));
* the latent heat h_lv and Stefan number (text after Eq. (11) and Eq. (21)).

Arithmetic is mpmath at MP_DPS decimal digits; results are handed to the
lattice oracle as Python floats.  Derivatives of the pressure are taken
numerically (mpmath.diff) straight from the definition of p, so that no
hand-differentiated formula can hide a mistake.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import mpmath as mp

MP_DPS = 40
mp.mp.dps = MP_DPS

# Eq. (17): a~ = 0.4963880577294099 R^2 Tc^2 / pc,  b~ = 0.1872945669467330 R Tc / pc
CS_A_COEF = mp.mpf("0.4963880577294099")
CS_B_COEF = mp.mpf("0.1872945669467330")


@dataclass
class Eos:
    """Equation of state p_EOS(rho, T).

    kind 'cs'  : Eq. (17), K_eos * [rho R T (1+t+t^2-t^3)/(1-t)^3 - a_t rho^2], t = b_t rho / 4
    kind 'vdw' : K_eos * [rho R T / (1 - b_t rho) - a_t rho^2]
    """
    kind: str = "cs"
    a_t: float = 1.0
    b_t: float = 4.0
    R: float = 1.0
    K_eos: float = 0.479820


def paper_cs_eos() -> Eos:
    """Parameters printed with the numerical tests: a~=1, b~=4, R=1, K_EOS=0.479820."""
    return Eos("cs", 1.0, 4.0, 1.0, 0.479820)


def vdw_eos() -> Eos:
    """The van der Waals workload: a=9/49, b=2/21, R=1 (Tc = 4/7, rho_c = 3.5, pc = 0.75)."""
    return Eos("vdw", 9.0 / 49.0, 2.0 / 21.0, 1.0, 1.0)


def _mpf(x):
    return mp.mpf(x) if not isinstance(x, mp.mpf) else x


def pressure(eos: Eos, rho, T):
    """p_EOS(rho, T), Eq. (17) (or the van der Waals form)."""
    rho, T = _mpf(rho), _mpf(T)
    a, b, R, K = _mpf(eos.a_t), _mpf(eos.b_t), _mpf(eos.R), _mpf(eos.K_eos)
    if eos.kind == "cs":
        t = b * rho / 4
        return K * (rho * R * T * (1 + t + t * t - t ** 3) / (1 - t) ** 3 - a * rho * rho)
    if eos.kind == "vdw":
        return K * (rho * R * T / (1 - b * rho) - a * rho * rho)
    raise ValueError(f"unknown EOS kind {eos.kind!r}")


def dp_drho(eos: Eos, rho, T):
    """(dp_EOS/drho)_T by numerical differentiation of the definition."""
    return mp.diff(lambda r: pressure(eos, r, T), _mpf(rho))


def d2p_drho2(eos: Eos, rho, T):
    return mp.diff(lambda r: pressure(eos, r, T), _mpf(rho), 2)


def chemical_potential(eos: Eos, rho, T):
    """mu(rho, T) up to a T-dependent constant: the antiderivative of (1/rho) dp/drho.

    Closed forms (checked against quadrature of (1/rho) dp/drho in the tests):
      cs : K [R T (ln rho + (8t - 9t^2 + 3t^3)/(1-t)^3) - 2 a rho]
      vdw: K [R T (ln(rho/(1-b rho)) + b rho/(1-b rho)) - 2 a rho]
    """
    rho, T = _mpf(rho), _mpf(T)
    a, b, R, K = _mpf(eos.a_t), _mpf(eos.b_t), _mpf(eos.R), _mpf(eos.K_eos)
    if eos.kind == "cs":
        t = b * rho / 4
        return K * (R * T * (mp.log(rho) + (8 * t - 9 * t * t + 3 * t ** 3) / (1 - t) ** 3) - 2 * a * rho)
    if eos.kind == "vdw":
        return K * (R * T * (mp.log(rho / (1 - b * rho)) + b * rho / (1 - b * rho)) - 2 * a * rho)
    raise ValueError(eos.kind)


def rho_max(eos: Eos):
    """Close-packing limit of the repulsive term (t = 1 for CS, b rho = 1 for vdW)."""
    return 4 / _mpf(eos.b_t) if eos.kind == "cs" else 1 / _mpf(eos.b_t)


def critical_point(eos: Eos):
    """(Tc, pc, rho_c).

    For CS, Tc and pc follow from inverting the a~, b~ definitions under Eq. (17);
    rho_c is then the root of dp/drho = 0 at Tc (tests check d2p/drho2 = 0 there too).
    For vdW: Tc = 8a/(27 b R), pc = a/(27 b^2), rho_c = 1/(3b).
    """
    a, b, R = _mpf(eos.a_t), _mpf(eos.b_t), _mpf(eos.R)
    if eos.kind == "cs":
        Tc = (a / b) * (CS_B_COEF / CS_A_COEF) / R
        pc_raw = CS_B_COEF * R * Tc / b          # p_cr of the bracket, before K_EOS scaling
        # At Tc the inflection point is a double root of dp/drho; minimise dp/drho
        rc = mp.findroot(lambda r: d2p_drho2(eos, r, Tc), 0.13 * 4 / b * mp.mpf(1))
        return Tc, pc_raw * _mpf(eos.K_eos), rc
    if eos.kind == "vdw":
        Tc = 8 * a / (27 * b * R)
        return Tc, _mpf(eos.K_eos) * a / (27 * b * b), 1 / (3 * b)
    raise ValueError(eos.kind)


def spinodals(eos: Eos, T):
    """The two roots of dp/drho = 0 below Tc, found by a sign scan then bisection."""
    rmax = rho_max(eos)
    n = 4000
    prev_r, prev_v = None, None
    roots = []
    for k in range(1, n):
        r = rmax * k / n
        v = dp_drho(eos, r, T)
        if prev_v is not None and (v > 0) != (prev_v > 0):
            roots.append(mp.findroot(lambda x: dp_drho(eos, x, T), (prev_r, r), solver="anderson"))
        prev_r, prev_v = r, v
        if len(roots) == 2:
            break
    if len(roots) != 2:
        raise ValueError("temperature is not below the critical temperature")
    return roots[0], roots[1]


def maxwell(eos: Eos, T):
    """Coexistence (rho_v, rho_l, p_s) at temperature T.

    Conditions: p(rho_v) = p(rho_l) = p_s and mu(rho_v) = mu(rho_l) (equal-area rule).
    Bracketed: for a trial p_s between the spinodal pressures the vapour root lies
    below the first spinodal and the liquid root above the second; bisection on
    mu_l - mu_v in p_s, then a two-variable Newton polish.
    """
    T = _mpf(T)
    s1, s2 = spinodals(eos, T)
    p_hi = pressure(eos, s1, T)
    p_lo = max(pressure(eos, s2, T), mp.mpf(0)) + mp.mpf(10) ** (-(MP_DPS - 5))
    rmax = rho_max(eos)

    def roots_at(ps):
        rv = mp.findroot(lambda r: pressure(eos, r, T) - ps, (mp.mpf(10) ** -30, s1), solver="anderson")
        # liquid branch: p rises without bound towards rmax
        hi = s2 + (rmax - s2) / 2
        while pressure(eos, hi, T) < ps:
            hi = hi + (rmax - hi) / 2
        rl = mp.findroot(lambda r: pressure(eos, r, T) - ps, (s2, hi), solver="anderson")
        return rv, rl

    def dmu(ps):
        rv, rl = roots_at(ps)
        return chemical_potential(eos, rl, T) - chemical_potential(eos, rv, T)

    lo, hi = p_lo, p_hi * (1 - mp.mpf(10) ** -(MP_DPS - 8))
    f_lo, f_hi = dmu(lo), dmu(hi)
    if (f_lo > 0) == (f_hi > 0):
        raise ValueError("could not bracket the coexistence pressure")
    for _ in range(200):
        mid = (lo + hi) / 2
        fm = dmu(mid)
        if (fm > 0) == (f_lo > 0):
            lo, f_lo = mid, fm
        else:
            hi, f_hi = mid, fm
        if hi - lo < abs(mid) * mp.mpf(10) ** -(MP_DPS // 2):
            break
    rv, rl = roots_at((lo + hi) / 2)
    sol = mp.findroot(
        [lambda v, l: pressure(eos, v, T) - pressure(eos, l, T),
         lambda v, l: chemical_potential(eos, v, T) - chemical_potential(eos, l, T)],
        (rv, rl), verify=False)
    rv, rl = sol[0], sol[1]
    scale = abs(pressure(eos, rv, T)) + abs(chemical_potential(eos, rv, T))
    resid = abs(pressure(eos, rv, T) - pressure(eos, rl, T)) + abs(
        chemical_potential(eos, rv, T) - chemical_potential(eos, rl, T))
    if not resid <= scale * mp.mpf(10) ** -(mp.mp.dps - 8):
        raise ValueError("Maxwell construction did not converge")
    return rv, rl, pressure(eos, rv, T)


def grand_potential_excess(eos: Eos, rho, T, rho_v, p_s):
    """Delta Omega(rho) = rho (mu(rho) - mu_s) - (p(rho) - p_s) >= 0 (free-energy excess over the tie line)."""
    mu_s = chemical_potential(eos, rho_v, T)
    return rho * (chemical_potential(eos, rho, T) - mu_s) - (pressure(eos, rho, T) - p_s)


def surface_tension(eos: Eos, T, kappa):
    """Square-gradient surface tension of a flat interface: integral of sqrt(2 kappa dOmega) d rho.

    The pressure tensor of Eq. (11) is that of the free energy f(rho) + kappa/2 |grad rho|^2,
    whose flat profile obeys kappa rho'^2 / 2 = dOmega.
    """
    rv, rl, ps = maxwell(eos, T)
    kappa = _mpf(kappa)
    g = lambda r: mp.sqrt(2 * kappa * max(grand_potential_excess(eos, r, T, rv, ps), 0))
    return mp.quad(g, mp.linspace(rv, rl, 9))


def interface_width(eos: Eos, T, kappa, lo=0.05, hi=0.95):
    """Distance over which the equilibrium flat profile goes from 5% to 95% of (rho_l - rho_v).

    z(rho) = integral sqrt(kappa / (2 dOmega)) d rho.
    """
    rv, rl, ps = maxwell(eos, T)
    kappa = _mpf(kappa)
    r_lo = rv + _mpf(lo) * (rl - rv)
    r_hi = rv + _mpf(hi) * (rl - rv)
    g = lambda r: mp.sqrt(kappa / (2 * grand_potential_excess(eos, r, T, rv, ps)))
    return mp.quad(g, mp.linspace(r_lo, r_hi, 9))


def flat_profile(eos: Eos, T, kappa, z):
    """Equilibrium flat-interface density at signed distance z from the mid-density point
    (liquid for z < 0).  Solves z(rho) = integral_{rho_mid}^{rho} -sqrt(kappa/(2 dOmega)) for rho."""
    rv, rl, ps = maxwell(eos, T)
    kappa = _mpf(kappa)
    rmid = (rv + rl) / 2
    g = lambda r: mp.sqrt(kappa / (2 * grand_potential_excess(eos, r, T, rv, ps)))

    def zof(r):
        return -mp.quad(g, [rmid, r])

    z = _mpf(z)
    lo, hi = rv + (rl - rv) * mp.mpf(10) ** -12, rl - (rl - rv) * mp.mpf(10) ** -12
    if z <= zof(hi):
        return rl
    if z >= zof(lo):
        return rv
    for _ in range(200):
        mid = (lo + hi) / 2
        if zof(mid) > z:
            lo = mid
        else:
            hi = mid
        if hi - lo < mp.mpf(10) ** -20:
            break
    return (lo + hi) / 2


# ---------------------------------------------------------------------------------------
# Model parameters and derived constants
# ---------------------------------------------------------------------------------------

@dataclass
class Params:
    """Model parameters.  Defaults are the paper's numerical-test set (text before Eq. (20))
    plus readings for what the paper leaves open (each marked)."""
    Tr0: float = 0.8              # reference reduced temperature T/Tc
    K_int: float = 2.294922       # K_INT of Eqs. (18)-(19)
    varpi: float = 1.0 / 6.0      # model coefficient in beta, k, h, b (SM Eqs. (3), (5a))
    gamma1: float = -2.0          # SM Eq. (4a,b)
    gamma2: float = 2.0
    tau_p: float = 0.5            # reading: tau_p = 1/s_p - 1/2 (sets s_q, s_e via the SM constraints)
    s_eps: float = 1.0            # reading
    sigma_e: float = 1.0          # reading
    sigma_eps: float = 1.0        # reading
    sigma_q: float = 1.0          # reading
    sigma_p: float = 1.0          # reading
    tau_j_v: float = 0.1          # reading: vapour tau_j = 1/sigma_j - 1/2
    lambda_ratio: float = 10.0    # lambda_l / lambda_v (text before Eq. (20))
    cv: float = 0.0               # <= 0: derive from the Stefan number below (reading)
    ste: float = 0.005            # Stefan number used to derive cv
    dTr_ste: float = 0.05         # T_r1 - T_r0 used to derive cv
    C_ref: float = 0.0            # <= 0: rho_v * cv (reading)
    accel_x: float = 0.0          # external acceleration a of Eq. (14)
    accel_y: float = 0.0
    cs_override: float = 0.0      # > 0: use this c_s instead of Eq. (19)
    dx: float = 1.0


@dataclass
class Derived:
    Tc: float
    pc: float
    rho_c: float
    T0: float
    rho_v: float
    rho_l: float
    p_s: float
    cs: float
    c: float
    dt: float
    G2: float
    a_mf: float
    kappa: float
    cv: float
    C_ref: float
    beta: float
    k: float
    h: float
    bS: float
    s_p: float
    s_q: float
    s_e: float
    s_eps: float
    omega_e: float
    omega_p: float
    tau_j_v: float
    tau_j_l: float
    h_lv: float
    params: dict = field(default_factory=dict)
    eos: dict = field(default_factory=dict)


def derive(eos: Eos, params: Params) -> Derived:
    """All per-run constants, in the order the paper fixes them."""
    Tc, pc, rc = critical_point(eos)
    T0 = _mpf(params.Tr0) * Tc
    rv, rl, ps = maxwell(eos, T0)
    dx = _mpf(params.dx)
    Kint, Keos, at = _mpf(params.K_int), _mpf(eos.K_eos), _mpf(eos.a_t)
    # Eq. (18): G = K_INT sqrt(2 K_EOS a~ / dx^2)
    G2 = Kint ** 2 * 2 * Keos * at / dx ** 2
    # Eq. (19): c_s = K_INT sqrt((dp_EOS/drho)_T + 2 K_EOS a~ rho) at rho = rho_l (reading: at T0)
    if params.cs_override > 0:
        cs = _mpf(params.cs_override)
    else:
        cs = Kint * mp.sqrt(dp_drho(eos, rl, T0) + 2 * Keos * at * rl)
    c = mp.sqrt(3) * cs                   # c_s = c / sqrt(3), text after Eq. (15)
    dt = dx / c                           # c = dx / dt
    a_mf = G2 * dx ** 2 / 2               # Eq. (16)
    kappa = G2 * dx ** 4 / 4
    # latent heat, text after Eq. (11): h_lv = a (rho_l - rho_v) + p_s (1/rho_v - 1/rho_l)
    h_lv = a_mf * (rl - rv) + ps * (1 / rv - 1 / rl)
    if params.cv > 0:
        cv = _mpf(params.cv)
    else:
        # Stefan number (text after Eq. (21)): Ste = rho_v cv Tc (T_r1 - T_r0) / (rho_l h_lv)
        cv = _mpf(params.ste) * rl * h_lv / (rv * Tc * _mpf(params.dTr_ste))
    C_ref = _mpf(params.C_ref) if params.C_ref > 0 else rv * cv
    w = _mpf(params.varpi)
    beta = -2 / (1 - w)                   # SM Eq. (3a,b)
    k = 1 - w                             # after SM Eq. (5b)
    h = 6 * w * (1 - w) / (1 - 3 * w)
    bS = (1 - w) / (1 - 3 * w)
    tau_p = _mpf(params.tau_p)
    tau_q = 1 / (12 * tau_p)              # tau_p tau_q = 1/12
    tau_e = 1 / (12 * (k + 1) * tau_q)    # (k+1) tau_e tau_q = 1/12
    s_p, s_q, s_e = 1 / (tau_p + mp.mpf(1) / 2), 1 / (tau_q + mp.mpf(1) / 2), 1 / (tau_e + mp.mpf(1) / 2)
    return Derived(
        Tc=float(Tc), pc=float(pc), rho_c=float(rc), T0=float(T0), rho_v=float(rv), rho_l=float(rl),
        p_s=float(ps), cs=float(cs), c=float(c), dt=float(dt), G2=float(G2), a_mf=float(a_mf),
        kappa=float(kappa), cv=float(cv), C_ref=float(C_ref), beta=float(beta), k=float(k), h=float(h),
        bS=float(bS), s_p=float(s_p), s_q=float(s_q), s_e=float(s_e), s_eps=float(params.s_eps),
        omega_e=float(s_e / 2 - 1), omega_p=float(s_p / 2 - 1),
        tau_j_v=float(params.tau_j_v), tau_j_l=float(params.tau_j_v * params.lambda_ratio),
        h_lv=float(h_lv), params=asdict(params), eos=asdict(eos))


def stefan_root(ste: float) -> float:
    """Root k of Ste / (exp(k^2) erf(k)) = k sqrt(pi), Eq. (21)."""
    f = lambda k: _mpf(ste) / (mp.exp(k * k) * mp.erf(k)) - k * mp.sqrt(mp.pi)
    return float(mp.findroot(f, (mp.mpf("1e-6"), mp.mpf(3)), solver="anderson"))


def fmt(x) -> str:
    return mp.nstr(x, 15) if isinstance(x, mp.mpf) else repr(x)


__all__ = [
    "Eos", "Params", "Derived", "paper_cs_eos", "vdw_eos", "pressure", "dp_drho", "d2p_drho2",
    "chemical_potential", "critical_point", "spinodals", "maxwell", "surface_tension",
    "interface_width", "flat_profile", "derive", "stefan_root", "grand_potential_excess",
]

if __name__ == "__main__":  # pragma: no cover - quick look
    d = derive(paper_cs_eos(), Params())
    for k_, v_ in asdict(d).items():
        if not isinstance(v_, dict):
            print(f"{k_:10s} {v_!r}")
    print("math check", math.sqrt(3))


def flat_profile_table(eos: Eos, T, kappa, n=400):
    """(z, rho) samples of the equilibrium flat profile (liquid at z < 0), for interpolation.
    z(rho) = -integral_{rho_mid}^{rho} sqrt(kappa / (2 dOmega)) drho, sampled on a grid in rho
    refined towards both bulk values."""
    rv, rl, ps = maxwell(eos, T)
    kappa = _mpf(kappa)
    rmid = (rv + rl) / 2
    g = lambda r: mp.sqrt(kappa / (2 * grand_potential_excess(eos, r, T, rv, ps)))
    zs, rs = [], []
    for k in range(1, n):
        s = mp.mpf(k) / n
        # cosine spacing crowds samples near the bulk values, where z varies fastest
        r = rv + (rl - rv) * (1 - mp.cos(mp.pi * s)) / 2
        zs.append(float(-mp.quad(g, [rmid, r])))
        rs.append(float(r))
    return zs[::-1], rs[::-1]
