// Pointwise pieces of the lattice update shared by the HIP kernels (the periodic
// fused update and diagnostics in lbm_kernels.hip, the bounded-domain update in
// lbm_bounded.hip): the equation of state, the pair-force stencil, the moment
// transforms, the macroscopic quantities of Eq. (14) and the two collisions.
// Device code only; every translation unit gets its own copy.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_internal.hpp"

namespace lbm_dev {
namespace {

// Velocity order (SM Eq. (1)): 0 rest, 1 (+x), 2 (+y), 3 (-x), 4 (-y),
// 5 (+x,+y), 6 (-x,+y), 7 (-x,-y), 8 (+x,-y).
__device__ constexpr int kEx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kEy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

__device__ inline double rcp(double x) { return 1.0 / x; }
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Block -> work-item remap so that the blocks one XCD receives (hardware
// dispatches block b to XCD b mod 8) cover a contiguous range of work items.
__device__ inline int remap_xcd(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7, slot = b >> 3;
    return x * q + min(x, r) + slot;
}

__device__ inline int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Element index of slot s (0..17) at node (x, y) in the row-interleaved layout.
__device__ inline size_t slot_index(int s, int x, int y, int nx) { return ((size_t)y * 18 + s) * (size_t)nx + x; }

// ---------------------------------------------------------------------------
// pointwise model pieces
// ---------------------------------------------------------------------------

// p_BE = p_EOS + a rho^2 (text after Eq. (11) with a = G^2 dx^2 / 2, Eq. (16));
// p_EOS is Eq. (17) (or the van der Waals form).
template <typename C>
__device__ inline C p_be(const Consts<C>& P, C rho, C T) {
    C rep;
    if (P.eos_kind == 0) {
        const C t = P.bq * rho, s = C(1) - t;
        const C z = (C(1) + t * (C(1) + t * (C(1) - t))) * rcp(s * s * s);
        rep = P.KR * rho * T * z;
    } else {
        rep = P.KR * rho * T * rcp(C(1) - P.bq * rho);
    }
    return rep + P.a_diff * rho * rho;
}

// Isotropic stencil sums s = sum_i w_i rho(x + e_i dx) e_i / c with w = 1/3 (axes),
// 1/12 (diagonals): Eq. (13).
template <typename C>
__device__ inline void stencil(C rE, C rN, C rW, C rS, C rNE, C rNW, C rSW, C rSE, C& sx, C& sy) {
    const C third = C(1) / C(3), twelfth = C(1) / C(12);
    sx = third * (rE - rW) + twelfth * ((rNE - rSW) + (rSE - rNW));
    sy = third * (rN - rS) + twelfth * ((rNE - rSW) + (rNW - rSE));
}

// Moment transform m = M f (SM Eq. (2)) done with sums and differences.
template <typename C>
__device__ inline void to_moments(const C* f, C* m) {
    const C A = (f[1] + f[2]) + (f[3] + f[4]);
    const C D = (f[5] + f[6]) + (f[7] + f[8]);
    m[0] = f[0] + A + D;
    m[1] = C(-4) * f[0] - A + C(2) * D;
    m[2] = C(4) * f[0] - C(2) * A + D;
    const C x1 = f[1] - f[3], y1 = f[2] - f[4];
    const C dp = f[5] - f[7], dm = f[8] - f[6];
    m[3] = x1 + dp + dm;
    m[4] = C(-2) * x1 + dp + dm;
    m[5] = y1 + dp - dm;
    m[6] = C(-2) * y1 + dp - dm;
    m[7] = (f[1] + f[3]) - (f[2] + f[4]);
    m[8] = (f[5] + f[7]) - (f[6] + f[8]);
}

// Inverse transform f = M^T D^-1 m with D = diag(9, 36, 36, 6, 12, 6, 12, 4, 4).
// The conserved moments are reproduced up to unbiased rounding: 1/9 and 1/6 are
// inexact in binary, and a product with their rounded values would scale the mass or
// the momentum by the same factor every step (with 1/6 rounded to FP32, momentum grew
// by 3e-8 of itself per step, which moved a translating droplet by 4e-4 nodes in 1000
// steps).  Row 0 of M is all ones, so f_0 = m_0 - sum_{i>0} f_i, and the axis and
// diagonal populations sum to 4 ba and 4 bd: f_0 = m_0 - 4 (ba + bd).  Likewise the
// x-momentum is (f_1 - f_3) + (f_5 - f_6 - f_7 + f_8) = 2 xx + 4 dx, so the diagonal
// part is taken as dx = (m_3 - 2 xx) / 4 (equal to a_3 + a_4 in exact arithmetic).
template <typename C>
__device__ inline void from_moments(const C* m, C* f) {
    const C a0 = m[0] * (C(1) / C(9)), a1 = m[1] * (C(1) / C(36)), a2 = m[2] * (C(1) / C(36));
    const C a3 = m[3] * (C(1) / C(6)), a4 = m[4] * (C(1) / C(12));
    const C a5 = m[5] * (C(1) / C(6)), a6 = m[6] * (C(1) / C(12));
    const C a7 = m[7] * C(0.25), a8 = m[8] * C(0.25);
    const C ba = a0 - a1 - C(2) * a2;          // axis populations
    const C bd = a0 + C(2) * a1 + a2;          // diagonal populations
    const C xx = a3 - C(2) * a4, yy = a5 - C(2) * a6;
    const C dx = (m[3] - C(2) * xx) * C(0.25), dy = (m[5] - C(2) * yy) * C(0.25);
    f[1] = ba + xx + a7;
    f[2] = ba + yy - a7;
    f[3] = ba - xx + a7;
    f[4] = ba - yy - a7;
    f[5] = bd + dx + dy + a8;
    f[6] = bd - dx + dy - a8;
    f[7] = bd - dx - dy + a8;
    f[8] = bd + dx - dy - a8;
    f[0] = m[0] - C(4) * (ba + bd);
}

// Macroscopic quantities at time t (Eq. (14)) from rho, the first moments of f
// (m3 = sum e_x f / c, m5 = sum e_y f / c), n0 = sum g and the stencil sums.
template <typename C>
struct Macro {
    C inv_rho, uxh, uyh, Fxh, Fyh, q, rho_ek, T, gx, gy;
};

template <typename C>
__device__ inline Macro<C> macros(const Consts<C>& P, C rho, C m3, C m5, C n0, C sx, C sy) {
    Macro<C> M;
    M.inv_rho = rcp(rho);
    // F = F_pair + rho a
    const C Fx = P.G2dx * rho * sx + rho * P.ax;
    const C Fy = P.G2dx * rho * sy + rho * P.ay;
    // rho u / c = sum e_i f_i / c + dt F / (2c)
    M.uxh = (m3 + P.hdt_c * Fx) * M.inv_rho;
    M.uyh = (m5 + P.hdt_c * Fy) * M.inv_rho;
    M.Fxh = Fx * P.inv_c;
    M.Fyh = Fy * P.inv_c;
    // q = F . u
    M.q = P.c * (Fx * M.uxh + Fy * M.uyh);
    M.rho_ek = n0 + P.hdt * M.q;
    // rho e_k = rho cv T + rho |u|^2 / 2
    M.T = (M.rho_ek * M.inv_rho - C(0.5) * P.c2 * (M.uxh * M.uxh + M.uyh * M.uyh)) * P.inv_cv;
    // grad rho = F_pair / (G^2 dx^2 rho) = s / dx (the SM's local evaluation)
    M.gx = sx * P.inv_dx;
    M.gy = sy * P.inv_dx;
    return M;
}

// Post-collision moments for f (Eq. (12b)) and g (Eq. (12c)).  f, g: pre-collision
// populations at the node; on return fo, go hold the post-collision populations.
template <typename C>
__device__ inline void collide(const Consts<C>& P, const C* f, const C* g, C rho, C sx, C sy, C* fo,
                               C* go) {
    C m[9], n[9];
    to_moments(f, m);
    to_moments(g, n);
    const Macro<C> M = macros(P, rho, m[3], m[5], n[0], sx, sy);
    const C ux = M.uxh, uy = M.uyh, Fx = M.Fxh, Fy = M.Fyh;

    // closure: eta = p_BE / c_s^2 - rho, rho h_k = rho e_k + p_BE
    const C pbe = p_be(P, rho, M.T);
    const C eta = pbe * P.inv_cs2 - rho;
    const C rho_hk = M.rho_ek + pbe;

    // --- f: SM Eqs. (3a), (3b), (5a), (6a) ---------------------------------
    const C u2 = ux * ux + uy * uy;
    const C ru2 = rho * u2;
    const C meq1 = C(-2) * rho + C(2) * eta + C(3) * ru2;
    const C meq2 = rho + P.beta * eta - C(3) * ru2;
    const C meq4 = -rho * ux, meq6 = -rho * uy;
    const C meq7 = rho * (ux * ux - uy * uy), meq8 = rho * ux * uy;
    const C Fu = Fx * ux + Fy * uy;
    const C Fm1 = C(6) * Fu, Fm2 = C(-6) * Fu, Fm4 = -Fx, Fm6 = -Fy;
    const C Fm7 = C(2) * (Fx * ux - Fy * uy), Fm8 = Fx * uy + Fy * ux;
    const C g2 = M.gx * M.gx + M.gy * M.gy;
    const C Q1 = P.Qpre * C(6) * g2, Q2 = -Q1;
    const C Q7 = P.Qpre * (M.gx * M.gx - M.gy * M.gy), Q8 = P.Qpre * M.gx * M.gy;
    // X = m - m_eq + dt/2 F_m - Q_m; rows 0, 3, 5 vanish identically
    const C X1 = m[1] - meq1 + P.hdt * Fm1 - Q1;
    const C X2 = m[2] - meq2 + P.hdt * Fm2 - Q2;
    const C X4 = m[4] - meq4 + P.hdt * Fm4;
    const C X6 = m[6] - meq6 + P.hdt * Fm6;
    const C X7 = m[7] - meq7 + P.hdt * Fm7 - Q7;
    const C X8 = m[8] - meq8 + P.hdt * Fm8 - Q8;
    C mb[9];
    mb[0] = rho;
    mb[1] = m[1] + P.dt * Fm1 - (P.s_e * X1 + P.ks * X2 + P.hs * (ux * X4 + uy * X6));
    mb[2] = m[2] + P.dt * Fm2 - P.s_eps * X2;
    mb[3] = m[3] + P.dt * Fx;
    mb[4] = m[4] + P.dt * Fm4 - P.s_q * X4;
    mb[5] = m[5] + P.dt * Fy;
    mb[6] = m[6] + P.dt * Fm6 - P.s_q * X6;
    mb[7] = m[7] + P.dt * Fm7 - (C(2) * P.bs * (ux * X4 - uy * X6) + P.s_p * X7);
    mb[8] = m[8] + P.dt * Fm8 - (P.bs * (uy * X4 + ux * X6) + P.s_p * X8);

    // --- g: SM Eqs. (4a), (4b), (5b), (6b) ---------------------------------
    const C T = M.T, q = M.q, rek = M.rho_ek;
    const C neq1 = C(-4) * rek + P.g1C * T;
    const C neq2 = C(4) * rek - P.g2C * T;
    const C neq3 = rho_hk * ux, neq5 = rho_hk * uy;
    const C qx = q * ux, qy = q * uy;
    // sigma_j from tau_j(rho), linear between the coexistence densities at T0
    C sfrac = (rho - P.rho_v) * P.inv_drho;
    sfrac = sfrac < C(0) ? C(0) : (sfrac > C(1) ? C(1) : sfrac);
    const C sig_j = rcp(P.tau_jv + P.dtau_j * sfrac + C(0.5));
    const C wq = P.sig_q * (C(0.5) * sig_j - C(1));
    const C D1 = n[1] - neq1 + P.hdt * P.gamma1 * q;
    const C D2 = n[2] - neq2 + P.hdt * P.gamma2 * q;
    const C D3 = n[3] - neq3 + P.hdt * qx;
    const C D4 = n[4] + neq3 - P.hdt * qx;
    const C D5 = n[5] - neq5 + P.hdt * qy;
    const C D6 = n[6] + neq5 - P.hdt * qy;
    // Y acts on Z = (m + m_bar)/2 - m_eq, rows 1, 7, 8
    const C Z1 = C(0.5) * (m[1] + mb[1]) - meq1;
    const C Z7 = C(0.5) * (m[7] + mb[7]) - meq7;
    const C Z8 = C(0.5) * (m[8] + mb[8]) - meq8;
    const C Yx = P.c2 * (ux * (Z1 * (C(1) / C(3)) + Z7) + C(2) * uy * Z8);
    const C Yy = P.c2 * (uy * (Z1 * (C(1) / C(3)) - Z7) + C(2) * ux * Z8);
    C nb[9];
    nb[0] = n[0] + P.dt * q;
    nb[1] = n[1] + P.dt * P.gamma1 * q - P.sig_e * D1;
    nb[2] = n[2] + P.dt * P.gamma2 * q - P.sig_eps * D2;
    nb[3] = n[3] + P.dt * qx - (sig_j * D3 + wq * D4) + Yx;
    nb[4] = n[4] - P.dt * qx - P.sig_q * D4 - Yx;
    nb[5] = n[5] + P.dt * qy - (sig_j * D5 + wq * D6) + Yy;
    nb[6] = n[6] - P.dt * qy - P.sig_q * D6 - Yy;
    nb[7] = n[7] - P.sig_p * n[7];
    nb[8] = n[8] - P.sig_p * n[8];

    from_moments(mb, fo);
    from_moments(nb, go);
}

}  // namespace
}  // namespace lbm_dev
