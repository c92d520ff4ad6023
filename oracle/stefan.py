"""FP64 CPU oracle of the lattice update on a domain bounded in x: the one-dimensional
Stefan problem of the paper (a 1024 x 4 domain heated from the left side, liquid-vapour
phase change driven by a hotter wall, interface position against the Neumann
solution, Eqs. (20)-(21) and Fig. 1).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the
CPU-baseline leg of the benchmark may import this module.  It shares no code with the
HIP library and never imports it.

Boundary treatment (a reading: the paper applies the improved non-equilibrium
extrapolation scheme of its reference [Huang2019.TLBM], which is not part of the
paper).  Here the plain non-equilibrium extrapolation of Guo, Zheng and Shi (Chinese
Physics 11, 366 (2002); Phys. Fluids 14, 2007 (2002)) stands in for it: the
post-collision populations of a boundary node are the equilibrium at the boundary's
macroscopic state plus the non-equilibrium part of the nearest fluid node,

    l_bar_i(x_b) = l_i^eq(rho_b, u_b, T_b) + [l_bar_i(x_n) - l_i^eq(x_n)],   l = f, g.

Columns x = 0 and x = nx - 1 are boundary nodes; y stays periodic.
  left  (x = 0, heated outflow, Eq. (20) setting): T_b = T_wall, u_b = u(x = 1)
        (zero-gradient outflow), rho_b the vapour root of p_EOS(rho_b, T_wall) = p_out
        (constant pressure; reading: p_out is the saturation pressure at T0, the pressure
        of the liquid at rest);
  right (x = nx - 1, liquid at rest): u_b = 0, T_b = T_far, rho_b = rho(x = nx - 2).
The pair force of Eq. (13) at a fluid node next to a boundary uses rho_b as the density
of the boundary node.  The state at time t is the set of pre-collision populations of
the fluid nodes 1 .. nx - 2; boundary columns carry no state of their own.

The cubic-velocity correction the paper also applies (its reference [Huang2020]) is
left out: with Ste = 0.005 the flow is slow (|u| / c_s ~ 1e-3), where those terms are
negligible.

Pins (tests/test_oracle_stefan.py): the wall density, the imposed boundary state, a
uniform wall state staying steady (at rest, and flowing towards the outflow, which fixes
the velocity-dependent parts of the equilibria the extrapolation uses), steady conduction (linear temperature, no flow), the f populations'
non-equilibrium part through the viscous decay of a shear mode between the walls
(second order in the width), and the g populations' non-equilibrium part through the
conduction profile's slope at the default vapour conductivity (no temperature jump at
either wall).  Dropping either part fails its pin (mutation tests).  The whole bounded
update is compared with the Neumann solution of Eq. (20) on the GPU.
"""
from __future__ import annotations

from dataclasses import dataclass

import mpmath as mp
import numpy as np

from . import lbm, thermo


@dataclass
class Walls:
    """Boundary values of the heated-outflow / wall pair (absolute temperatures)."""
    T_wall: float
    T_far: float
    p_out: float
    rho_wall: float     # vapour root of p_EOS(rho, T_wall) = p_out


def walls(model: lbm.Model, Tr_wall: float, Tr_far: float | None = None, p_out: float | None = None) -> Walls:
    """Wall temperature T_r1 Tc at the heated side, T_far at the far wall (default T0),
    outflow pressure p_out (default the saturation pressure p_s at T0)."""
    d = model.d
    T_wall = Tr_wall * d.Tc
    T_far = d.T0 if Tr_far is None else Tr_far * d.Tc
    p = d.p_s if p_out is None else p_out
    # vapour branch: p_EOS rises with rho up to the first spinodal at T_wall
    lo, hi = mp.mpf("1e-30"), thermo.spinodals(model.eos, mp.mpf(T_wall))[0]
    f = lambda r: thermo.pressure(model.eos, r, T_wall) - p
    if not f(hi) > 0:
        raise ValueError("p_out is above the vapour spinodal pressure at the wall temperature")
    for _ in range(400):
        mid = (lo + hi) / 2
        if f(mid) > 0:
            hi = mid
        else:
            lo = mid
    return Walls(float(T_wall), float(T_far), float(p), float((lo + hi) / 2))


def _eq_pops(model: lbm.Model, rho, ux, uy, T):
    """(f^eq, g^eq) = M^-1 m^eq, M^-1 n^eq of a macroscopic state (SM Eqs. (3a), (4a))."""
    d = model.d
    uxh, uyh = ux / d.c, uy / d.c
    pbe = lbm.p_be(model, rho, T)
    eta = pbe / (d.cs * d.cs) - rho
    rho_ek = rho * (d.cv * T + 0.5 * (ux * ux + uy * uy))
    f = lbm.from_moments(lbm.m_eq(model, rho, uxh, uyh, eta))
    g = lbm.from_moments(lbm.n_eq(model, rho_ek, T, rho_ek + pbe, uxh, uyh))
    return f, g


def macros(model: lbm.Model, w: Walls, st: lbm.State):
    """Eq. (14) at the fluid nodes with the boundary densities of the walls in the stencil;
    returns (macroscopic fields, state with stand-in populations at the boundary columns).
    Boundary columns of the returned fields hold the imposed boundary state."""
    d, p = model.d, model.params
    f = st.f.copy()
    g = st.g.copy()
    rho_in = f[:, :, 1:-1].sum(axis=0)
    ny = f.shape[1]
    rho_b = np.full(ny, w.rho_wall), rho_in[:, -1]
    # stand-in populations at the boundary columns: only their density enters the stencil
    for col, rb, T in ((0, rho_b[0], w.T_wall), (-1, rho_b[1], w.T_far)):
        fe, ge = _eq_pops(model, rb, 0 * rb, 0 * rb, 0 * rb + T)
        f[:, :, col], g[:, :, col] = fe, ge
    mac = lbm.macros(model, lbm.State(f, g, st.step))
    # boundary velocity and temperature (the stencil values there are not used)
    mac.ux[:, 0], mac.uy[:, 0] = mac.ux[:, 1], mac.uy[:, 1]
    mac.ux[:, -1] = mac.uy[:, -1] = 0.0
    mac.T[:, 0], mac.T[:, -1] = w.T_wall, w.T_far
    return mac, lbm.State(f, g, st.step)


def step(model: lbm.Model, w: Walls, st: lbm.State) -> lbm.State:
    d = model.d
    mac, full = macros(model, w, st)
    fbar, gbar = lbm.collide(model, full, mac)
    for col, nb in ((0, 1), (-1, -2)):
        rho_b, ux_b, uy_b, T_b = mac.rho[:, col], mac.ux[:, col], mac.uy[:, col], mac.T[:, col]
        fe_b, ge_b = _eq_pops(model, rho_b, ux_b, uy_b, T_b)
        # equilibrium of the neighbour at the state its collision used
        uxh, uyh = mac.ux[:, nb] / d.c, mac.uy[:, nb] / d.c
        rho_n = mac.rho[:, nb]
        pbe = lbm.p_be(model, rho_n, mac.T[:, nb])
        eta = pbe / (d.cs * d.cs) - rho_n
        fe_n = lbm.from_moments(lbm.m_eq(model, rho_n, uxh, uyh, eta))
        ge_n = lbm.from_moments(lbm.n_eq(model, mac.rho_ek[:, nb], mac.T[:, nb], mac.rho_ek[:, nb] + pbe, uxh, uyh))
        fbar[:, :, col] = fe_b + fbar[:, :, nb] - fe_n
        gbar[:, :, col] = ge_b + gbar[:, :, nb] - ge_n
    f = lbm.stream(fbar)
    g = lbm.stream(gbar)
    # boundary columns carry no state (what wrapped around is not used)
    f[:, :, 0] = f[:, :, -1] = np.nan
    g[:, :, 0] = g[:, :, -1] = np.nan
    return lbm.State(f, g, st.step + 1)


def run(model: lbm.Model, w: Walls, st: lbm.State, n: int) -> lbm.State:
    for _ in range(n):
        st = step(model, w, st)
    return st


def init_state(model: lbm.Model, rho, ux, uy, T) -> lbm.State:
    """Same reading as the periodic oracle: f = M^-1 m^eq, g = M^-1 n^eq of the given fields."""
    st = lbm.init_state(model, rho, ux, uy, T)
    st.f[:, :, 0] = st.f[:, :, -1] = np.nan
    st.g[:, :, 0] = st.g[:, :, -1] = np.nan
    return st


def moments(model: lbm.Model, w: Walls, st: lbm.State):
    """(rho, ux, uy, T) at time t; boundary columns hold the imposed boundary state."""
    mac, _ = macros(model, w, st)
    return mac.rho, mac.ux, mac.uy, mac.T


def interface_position(rho_row: np.ndarray, rho_v: float, rho_l: float) -> float:
    """First crossing of (rho_v + rho_l)/2 from the vapour side, linearly interpolated, in
    node units from the heated boundary node x = 0."""
    mid = 0.5 * (rho_v + rho_l)
    k = int(np.argmax(rho_row >= mid))
    if k == 0 or rho_row[k] < mid:
        raise ValueError("no vapour-liquid crossing")
    return (k - 1) + (mid - rho_row[k - 1]) / (rho_row[k] - rho_row[k - 1])


def neumann_position(k: float, alpha: float, t: np.ndarray, t0: float) -> np.ndarray:
    """Eq. (20): X_i(t) = 2 k sqrt(alpha_v (t + t0))."""
    return 2 * k * np.sqrt(alpha * (t + t0))


__all__ = ["Walls", "walls", "step", "run", "init_state", "moments", "macros", "interface_position",
           "neumann_position"]
