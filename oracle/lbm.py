"""FP64 CPU oracle of the lattice update: D2Q9 double-distribution MRT step with the
pairwise interaction force, the dense-gas equation of state and the total kinetic
energy distribution.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the
CPU-baseline leg of the benchmark may import this module.  It shares no code with
the HIP library and never imports it.

The step is written in moment space exactly as the paper states it, with explicit
9x9 matrices built per node (S depends on the local velocity, L on the local
density), and numpy.roll for the periodic stencil and the streaming.  Each piece
cites its source:

  velocities            SM Eq. (1)
  moment matrix M       SM Eq. (2)
  m^eq, F_m             SM Eq. (3a), (3b)
  n^eq, q_m             SM Eq. (4a), (4b)
  S, L                  SM Eq. (5a), (5b) and the constants listed after them
  Q_m, Y                SM Eq. (6a), (6b); grad(rho) from F_pair (last SM remark)
  streaming             Eq. (12a)
  collisions            Eq. (12b), (12c)
  pair force            Eq. (13)
  moments               Eq. (14), with F = F_pair + rho a and q = F . u
  closure               Eqs. (15)-(16): p_LBE = c_s^2 (rho + eta) = p_BE = p_EOS + a rho^2,
                        rho h_k = rho e_k + p_BE
  temperature           rho e_k = rho c_v T + rho |u|^2 / 2 (text after Eq. (11))

Readings of points the paper leaves open (initial state, lambda between phases,
the discrete potential energy) are marked where they are used.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import thermo

# --- SM Eq. (1): e_i / c for i = 0..8 -------------------------------------------------
def _velocities() -> np.ndarray:
    e = np.zeros((9, 2))
    for i in range(1, 5):
        ang = (i - 1) * np.pi / 2
        e[i] = (np.cos(ang), np.sin(ang))
    for i in range(5, 9):
        ang = (2 * i - 1) * np.pi / 4
        e[i] = (np.sqrt(2) * np.cos(ang), np.sqrt(2) * np.sin(ang))
    return np.rint(e)


E = _velocities().astype(np.int64)          # integer lattice vectors e_i / c
EF = E.astype(np.float64)

# --- SM Eq. (2): orthogonal moment matrix (rows rho, e, eps, jx, qx, jy, qy, pxx, pxy) --
M = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1],
], dtype=np.float64)
# M is orthogonal (SM Eq. (2)): M M^T = D = diag(9, 36, 36, 6, 12, 6, 12, 4, 4), so
# M^-1 = M^T D^-1 exactly, with every entry a correctly rounded k/D_j.  (A numerical
# inverse misses this by an ulp or so, enough to leak mass from the momentum rows.)
MINV = M.T / np.diag(M @ M.T)[None, :]

# --- Eq. (13): omega(|e_i dt|^2) = 1/3 on axes, 1/12 on diagonals --------------------
OMEGA = np.array([0.0] + [1.0 / 3.0] * 4 + [1.0 / 12.0] * 4)


@dataclass
class Model:
    """Numbers the step needs, all float64.  Built from oracle.thermo.derive()."""
    eos: thermo.Eos
    d: thermo.Derived
    params: thermo.Params

    @classmethod
    def build(cls, eos: thermo.Eos, params: thermo.Params) -> "Model":
        return cls(eos, thermo.derive(eos, params), params)


# ---------------------------------------------------------------------------------------
# pointwise physics
# ---------------------------------------------------------------------------------------

def p_eos(model: Model, rho, T):
    """Eq. (17) (or the van der Waals form), vectorised in float64."""
    e = model.eos
    if e.kind == "cs":
        t = e.b_t * rho / 4.0
        return e.K_eos * (rho * e.R * T * (1 + t + t * t - t ** 3) / (1 - t) ** 3 - e.a_t * rho * rho)
    return e.K_eos * (rho * e.R * T / (1 - e.b_t * rho) - e.a_t * rho * rho)


def p_be(model: Model, rho, T):
    """p_BE = p_EOS + a rho^2 with a = G^2 dx^2 / 2 (text after Eq. (11), Eq. (16))."""
    return p_eos(model, rho, T) + model.d.a_mf * rho * rho


def tau_j(model: Model, rho):
    """Reading: lambda (hence tau_j = 1/sigma_j - 1/2) linear in rho between the
    coexistence densities at T0, clamped outside; lambda_l = ratio * lambda_v."""
    d = model.d
    s = np.clip((rho - d.rho_v) / (d.rho_l - d.rho_v), 0.0, 1.0)
    return d.tau_j_v + (d.tau_j_l - d.tau_j_v) * s


def shifted(a: np.ndarray, ex: int, ey: int) -> np.ndarray:
    """Periodic a(x + ex dx, y + ey dx).  Arrays are indexed [y, x]."""
    return np.roll(a, shift=(-ey, -ex), axis=(0, 1))


def pair_force(model: Model, rho: np.ndarray):
    """Eq. (13): F_pair = G^2 rho(x) sum_i omega(|e_i dt|^2) rho(x + e_i dt) e_i dt,
    with e_i dt = dx * (integer lattice vector)."""
    d, dx = model.d, model.params.dx
    sx = np.zeros_like(rho)
    sy = np.zeros_like(rho)
    for i in range(1, 9):
        nb = shifted(rho, E[i, 0], E[i, 1])
        sx += OMEGA[i] * nb * E[i, 0] * dx
        sy += OMEGA[i] * nb * E[i, 1] * dx
    return d.G2 * rho * sx, d.G2 * rho * sy


# ---------------------------------------------------------------------------------------
# moment-space building blocks (SM Eqs. (3)-(6)); arrays carry a leading axis of 9
# ---------------------------------------------------------------------------------------

def m_eq(model: Model, rho, uxh, uyh, eta):
    """SM Eq. (3a)."""
    d = model.d
    u2 = uxh * uxh + uyh * uyh
    return np.stack([
        rho,
        -2 * rho + 2 * eta + 3 * rho * u2,
        rho + d.beta * eta - 3 * rho * u2,
        rho * uxh,
        -rho * uxh,
        rho * uyh,
        -rho * uyh,
        rho * (uxh * uxh - uyh * uyh),
        rho * uxh * uyh,
    ])


def f_m(Fxh, Fyh, uxh, uyh):
    """SM Eq. (3b)."""
    fu = Fxh * uxh + Fyh * uyh
    z = np.zeros_like(Fxh)
    return np.stack([
        z, 6 * fu, -6 * fu, Fxh, -Fxh, Fyh, -Fyh,
        2 * Fxh * uxh - 2 * Fyh * uyh,
        Fxh * uyh + Fyh * uxh,
    ])


def n_eq(model: Model, rho_ek, T, rho_hk, uxh, uyh):
    """SM Eq. (4a)."""
    p, d = model.params, model.d
    z = np.zeros_like(rho_ek)
    return np.stack([
        rho_ek,
        -4 * rho_ek + (4 + p.gamma1) * d.C_ref * T,
        4 * rho_ek - (4 - p.gamma2) * d.C_ref * T,
        rho_hk * uxh, -rho_hk * uxh, rho_hk * uyh, -rho_hk * uyh,
        z, z,
    ])


def q_m(model: Model, q, uxh, uyh):
    """SM Eq. (4b)."""
    p = model.params
    z = np.zeros_like(q)
    return np.stack([q, p.gamma1 * q, p.gamma2 * q, q * uxh, -q * uxh, q * uyh, -q * uyh, z, z])


def s_matrix(model: Model, uxh, uyh):
    """SM Eq. (5a), one 9x9 matrix per node: shape (9, 9, ny, nx).
    s_0 and s_j multiply identically vanishing entries; they are set to 1."""
    d = model.d
    S = np.zeros((9, 9) + uxh.shape)
    s0 = sj = 1.0
    S[0, 0] = s0
    S[1, 1] = d.s_e
    S[1, 2] = d.k * d.s_eps * d.omega_e
    S[1, 4] = d.h * uxh * d.s_q * d.omega_e
    S[1, 6] = d.h * uyh * d.s_q * d.omega_e
    S[2, 2] = d.s_eps
    S[3, 3] = sj
    S[4, 4] = d.s_q
    S[5, 5] = sj
    S[6, 6] = d.s_q
    S[7, 4] = 2 * d.bS * uxh * d.s_q * d.omega_p
    S[7, 6] = -2 * d.bS * uyh * d.s_q * d.omega_p
    S[7, 7] = d.s_p
    S[8, 4] = d.bS * uyh * d.s_q * d.omega_p
    S[8, 6] = d.bS * uxh * d.s_q * d.omega_p
    S[8, 8] = d.s_p
    return S


def l_matrix(model: Model, rho):
    """SM Eq. (5b) with sigma_j = 1/(tau_j(rho) + 1/2) per node; sigma_0 multiplies zero."""
    p = model.params
    sj = 1.0 / (tau_j(model, rho) + 0.5)
    wj = sj / 2 - 1
    L = np.zeros((9, 9) + rho.shape)
    L[0, 0] = 1.0
    L[1, 1] = p.sigma_e
    L[2, 2] = p.sigma_eps
    L[3, 3] = sj
    L[3, 4] = p.sigma_q * wj
    L[4, 4] = p.sigma_q
    L[5, 5] = sj
    L[5, 6] = p.sigma_q * wj
    L[6, 6] = p.sigma_q
    L[7, 7] = p.sigma_p
    L[8, 8] = p.sigma_p
    return L


def q_comp(model: Model, gx, gy):
    """SM Eq. (6a)."""
    d, dx = model.d, model.params.dx
    pre = d.G2 * dx * dx * d.dt * d.dt / 12.0
    g2 = gx * gx + gy * gy
    z = np.zeros_like(gx)
    return pre * np.stack([z, 6 * g2, -6 * g2, z, z, z, z, gx * gx - gy * gy, gx * gy])


def y_matrix(uxh, uyh):
    """SM Eq. (6b), one 9x9 matrix per node."""
    Y = np.zeros((9, 9) + uxh.shape)
    Y[3, 1], Y[3, 7], Y[3, 8] = uxh / 3, uxh, 2 * uyh
    Y[4, 1], Y[4, 7], Y[4, 8] = -uxh / 3, -uxh, -2 * uyh
    Y[5, 1], Y[5, 7], Y[5, 8] = uyh / 3, -uyh, 2 * uxh
    Y[6, 1], Y[6, 7], Y[6, 8] = -uyh / 3, uyh, -2 * uxh
    return Y


def matvec(A, v):
    """Per-node 9x9 matrix times 9-vector."""
    return np.einsum("ij...,j...->i...", A, v)


def to_moments(pops):
    """m = M (f_i)^T at every node."""
    return np.einsum("ij,j...->i...", M, pops)


def from_moments(mom):
    """(f_i)^T = M^-1 m at every node."""
    return np.einsum("ij,j...->i...", MINV, mom)


# ---------------------------------------------------------------------------------------
# state, initialisation, moments, step
# ---------------------------------------------------------------------------------------

@dataclass
class State:
    f: np.ndarray      # (9, ny, nx)
    g: np.ndarray      # (9, ny, nx)
    step: int = 0


def init_state(model: Model, rho, ux, uy, T) -> State:
    """Reading: f = M^-1 m^eq and g = M^-1 n^eq of the given fields, with no force shift
    (the paper states no initialisation)."""
    d = model.d
    rho = np.asarray(rho, np.float64)
    ux = np.asarray(ux, np.float64)
    uy = np.asarray(uy, np.float64)
    T = np.asarray(T, np.float64)
    uxh, uyh = ux / d.c, uy / d.c
    pbe = p_be(model, rho, T)
    eta = pbe / (d.cs * d.cs) - rho
    f = from_moments(m_eq(model, rho, uxh, uyh, eta))
    rho_ek = rho * (d.cv * T + 0.5 * (ux * ux + uy * uy))
    rho_hk = rho_ek + pbe
    g = from_moments(n_eq(model, rho_ek, T, rho_hk, uxh, uyh))
    return State(f, g, 0)


@dataclass
class Macro:
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    T: np.ndarray
    Fx: np.ndarray
    Fy: np.ndarray
    q: np.ndarray
    rho_ek: np.ndarray
    Fpx: np.ndarray
    Fpy: np.ndarray


def macros(model: Model, st: State) -> Macro:
    """Eq. (14) and the temperature: everything at time t before collision."""
    d, p = model.d, model.params
    rho = st.f.sum(axis=0)
    Fpx, Fpy = pair_force(model, rho)
    Fx = Fpx + rho * p.accel_x
    Fy = Fpy + rho * p.accel_y
    # rho u = sum_i e_i f_i + dt/2 F, with e_i = c * E_i
    jx = d.c * np.einsum("i,i...->...", EF[:, 0], st.f)
    jy = d.c * np.einsum("i,i...->...", EF[:, 1], st.f)
    ux = (jx + 0.5 * d.dt * Fx) / rho
    uy = (jy + 0.5 * d.dt * Fy) / rho
    q = Fx * ux + Fy * uy
    rho_ek = st.g.sum(axis=0) + 0.5 * d.dt * q
    T = (rho_ek / rho - 0.5 * (ux * ux + uy * uy)) / d.cv
    return Macro(rho, ux, uy, T, Fx, Fy, q, rho_ek, Fpx, Fpy)


def collide(model: Model, st: State, mac: Macro | None = None):
    """Eqs. (12b), (12c) at every node; returns post-collision (f_bar, g_bar)."""
    d, p = model.d, model.params
    if mac is None:
        mac = macros(model, st)
    rho = mac.rho
    uxh, uyh = mac.ux / d.c, mac.uy / d.c
    Fxh, Fyh = mac.Fx / d.c, mac.Fy / d.c
    pbe = p_be(model, rho, mac.T)
    eta = pbe / (d.cs * d.cs) - rho
    rho_hk = mac.rho_ek + pbe

    # f: density distribution
    m = to_moments(st.f)
    meq = m_eq(model, rho, uxh, uyh, eta)
    Fm = f_m(Fxh, Fyh, uxh, uyh)
    S = s_matrix(model, uxh, uyh)
    # grad rho computed locally from F_pair (last remark of the SM): F_pair = G^2 dx^2 rho grad(rho)
    gx = mac.Fpx / (d.G2 * p.dx * p.dx * rho)
    gy = mac.Fpy / (d.G2 * p.dx * p.dx * rho)
    Qm = q_comp(model, gx, gy)
    mbar = m + d.dt * Fm - matvec(S, m - meq + 0.5 * d.dt * Fm) + matvec(S, Qm)

    # g: total kinetic energy distribution
    n = to_moments(st.g)
    neq = n_eq(model, mac.rho_ek, mac.T, rho_hk, uxh, uyh)
    qm = q_m(model, mac.q, uxh, uyh)
    L = l_matrix(model, rho)
    Y = y_matrix(uxh, uyh)
    nbar = (n + d.dt * qm - matvec(L, n - neq + 0.5 * d.dt * qm)
            + d.c * d.c * matvec(Y, 0.5 * (m + mbar) - meq))
    return from_moments(mbar), from_moments(nbar)


def stream(pops: np.ndarray) -> np.ndarray:
    """Eq. (12a): l_i(x + e_i dt, t + dt) = l_bar_i(x, t), periodic."""
    out = np.empty_like(pops)
    for i in range(9):
        out[i] = np.roll(pops[i], shift=(E[i, 1], E[i, 0]), axis=(0, 1))
    return out


def step(model: Model, st: State) -> State:
    fbar, gbar = collide(model, st)
    return State(stream(fbar), stream(gbar), st.step + 1)


def run(model: Model, st: State, n: int) -> State:
    for _ in range(n):
        st = step(model, st)
    return st


# ---------------------------------------------------------------------------------------
# diagnostics
# ---------------------------------------------------------------------------------------

def invariants(model: Model, st: State) -> dict:
    """Global sums.  mass and momentum are exact invariants on periodic domains with no
    external acceleration; sum_g obeys sum_g(t+dt) = sum_g(t) + dt * sum_q(t) (row 0 of
    Eq. (12c)); E_p is the reading of the discrete potential energy
    -(G^2 dx^2 / 2) sum_x [rho^2/6 + rho(x)/2 * sum_i omega_i rho(x + e_i dx)],
    which equals the integral of rho V_mean / 2 with V_mean of Eq. (8) to O(dx^4)."""
    d = model.d
    mac = macros(model, st)
    rho = mac.rho
    nb = np.zeros_like(rho)
    for i in range(1, 9):
        nb += OMEGA[i] * shifted(rho, E[i, 0], E[i, 1])
    Ep = -(d.G2 * model.params.dx ** 2 / 2) * np.sum(rho * rho / 6 + 0.5 * rho * nb)
    return {
        "mass": float(st.f.sum()),
        "mom_x": float(d.c * np.einsum("i,i...->...", EF[:, 0], st.f).sum()),
        "mom_y": float(d.c * np.einsum("i,i...->...", EF[:, 1], st.f).sum()),
        "sum_g": float(st.g.sum()),
        "dt_sum_q": float(d.dt * mac.q.sum()),
        "E_p": float(Ep),
        "E_kin": float(mac.rho_ek.sum()),
    }


def moments(model: Model, st: State):
    """(rho, ux, uy, T) at time t, Eq. (14)."""
    mac = macros(model, st)
    return mac.rho, mac.ux, mac.uy, mac.T


__all__ = ["E", "M", "MINV", "OMEGA", "Model", "State", "Macro", "init_state", "macros",
           "collide", "stream", "step", "run", "invariants", "moments", "pair_force",
           "p_eos", "p_be", "tau_j", "m_eq", "n_eq", "f_m", "q_m", "s_matrix", "l_matrix",
           "y_matrix", "q_comp", "to_moments", "from_moments", "shifted"]
