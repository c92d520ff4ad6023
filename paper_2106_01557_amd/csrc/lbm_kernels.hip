// HIP kernels for gfx950 (MI355X): the lattice update of the liquid-vapour
// double-distribution model and its diagnostics.
//
// Layout in HBM: structure of arrays, 18 planes of nx*ny values (plane i < 9 is
// f_i, plane 9 + i is g_i), each plane row-major [y][x] with x fastest.
// Velocity order (SM Eq. (1)): 0 rest, 1 (+x), 2 (+y), 3 (-x), 4 (-y),
// 5 (+x,+y), 6 (-x,+y), 7 (-x,-y), 8 (+x,-y).
//
// The per-node arithmetic follows the paper's moment-space form: M of SM Eq. (2)
// applied as sums and differences, the equilibria and sources of SM Eqs. (3)-(4),
// the collision matrices S and L of SM Eq. (5) (only their non-trivial rows),
// the compensation Q_m and dissipation Y of SM Eq. (6), the moments of Eq. (14)
// and the closure p_LBE = c_s^2 (rho + eta) = p_BE (Eq. (15)).  No MFMA: the
// update is not a contraction; it is bound by HBM traffic (36 values per node
// per step in the fused two-buffer scheme).

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lbm_internal.hpp"

namespace lbm_dev {
namespace {

// ---------------------------------------------------------------------------
// storage <-> arithmetic conversions; 16-bit formats store deviations from a
// per-population reference (the rest equilibrium of a reference state)
// ---------------------------------------------------------------------------
template <typename S, typename C>
struct Io;

template <>
struct Io<double, double> {
    __device__ static double ld(const double* p, int k, double) { return p[k]; }
    __device__ static void st(double* p, int k, double v, double) { p[k] = v; }
};
template <>
struct Io<float, float> {
    __device__ static float ld(const float* p, int k, float) { return p[k]; }
    __device__ static void st(float* p, int k, float v, float) { p[k] = v; }
};
template <>
struct Io<__half, float> {
    __device__ static float ld(const __half* p, int k, float ref) { return __half2float(p[k]) + ref; }
    __device__ static void st(__half* p, int k, float v, float ref) { p[k] = __float2half(v - ref); }
};
template <>
struct Io<__hip_bfloat16, float> {
    __device__ static float ld(const __hip_bfloat16* p, int k, float ref) {
        return __bfloat162float(p[k]) + ref;
    }
    __device__ static void st(__hip_bfloat16* p, int k, float v, float ref) {
        p[k] = __float2bfloat16(v - ref);
    }
};

__device__ inline double rcp(double x) { return 1.0 / x; }
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Block -> work-item remap so that the blocks one XCD receives (hardware
// dispatches block b to XCD b mod 8) cover a contiguous range of work items.
__device__ inline int remap_xcd(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7, slot = b >> 3;
    return x * q + min(x, r) + slot;
}

__device__ inline int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

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
// Row 0 of M is all ones, so f_0 = m_0 - sum_{i>0} f_i, and the axis and diagonal
// populations sum to 4 ba and 4 bd; taking f_0 = m_0 - 4 (ba + bd) keeps the sum of
// the populations equal to m_0 up to unbiased rounding (1/9 is inexact in binary
// and would otherwise bias the mass in the same direction every step).
template <typename C>
__device__ inline void from_moments(const C* m, C* f) {
    const C a0 = m[0] * (C(1) / C(9)), a1 = m[1] * (C(1) / C(36)), a2 = m[2] * (C(1) / C(36));
    const C a3 = m[3] * (C(1) / C(6)), a4 = m[4] * (C(1) / C(12));
    const C a5 = m[5] * (C(1) / C(6)), a6 = m[6] * (C(1) / C(12));
    const C a7 = m[7] * C(0.25), a8 = m[8] * C(0.25);
    const C ba = a0 - a1 - C(2) * a2;          // axis populations
    const C bd = a0 + C(2) * a1 + a2;          // diagonal populations
    const C xx = a3 - C(2) * a4, yy = a5 - C(2) * a6;
    const C dx = a3 + a4, dy = a5 + a6;
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

// Velocity components per population (integer lattice vectors).
__device__ constexpr int kEx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kEy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// ---------------------------------------------------------------------------
// fused two-buffer step (push streaming)
// ---------------------------------------------------------------------------
// A wavefront owns a strip of 62 columns and marches through `rows` rows.  Lane
// L holds column x0 - 1 + L (lanes 0 and 63 are halo columns that only supply
// rho).  Each row's density is computed once from the 9 f values the lane
// loads anyway; neighbour densities in x come from the adjacent lanes (wave
// shuffles), in y from the rows kept in registers, so every f value is read
// from HBM once per step (plus two halo rows per strip of `rows`).
//
// Software pipeline: while row y is collided, the g values of row y+1 and the f
// values of row y+2 are already in flight (vector memory returns in order, so the
// loads for later rows are issued before the registers of earlier rows are used).
// The last row of a strip is peeled so the pipelined rows need no selects.
//
// Addressing: with kBuf every access is a raw buffer instruction on one resource
// per state buffer whose record count covers all 18 planes; the plane offset goes
// in the scalar offset, the lane's row/column byte offset in the vector offset.  A
// lane that must not store (halo columns) gets the vector offset
// drop = 2^32 - 1 - 17 * plane_bytes: for every plane the total offset then lies at
// or past the record count without leaving 32 bits, so the hardware drops the
// store whether or not it counts the scalar offset in its range check.  That needs
// 35 * plane_bytes < 2^32, which the launcher checks; larger lattices use 64-bit
// plane addresses and branch around the halo stores.
template <typename S>
struct Bits;
template <>
struct Bits<float> {
    __device__ static float ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
    }
    __device__ static void st(float x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, v, s, 0);
    }
};
template <>
struct Bits<double> {
    using V2 = unsigned __attribute__((ext_vector_type(2)));
    __device__ static double ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
    }
    __device__ static void st(double x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, x), r, v, s, 0);
    }
};
template <>
struct Bits<__half> {
    __device__ static __half ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        return __builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
    }
    __device__ static void st(__half x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, v, s, 0);
    }
};
template <>
struct Bits<__hip_bfloat16> {
    __device__ static __hip_bfloat16 ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        return __builtin_bit_cast(__hip_bfloat16, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
    }
    __device__ static void st(__hip_bfloat16 x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, v, s, 0);
    }
};

template <typename S, bool kBuf>
struct Planes;

template <typename S>
struct Planes<S, true> {
    __amdgpu_buffer_rsrc_t r;
    unsigned pb, drop;
    __device__ Planes(const void* base, size_t plane_bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)(unsigned)(18 * plane_bytes),
                                              0x00020000)),
          pb((unsigned)plane_bytes),
          drop((0xFFFFFFFFu - 17u * (unsigned)plane_bytes) & ~(unsigned)(sizeof(S) - 1)) {}
    template <typename C>
    __device__ C ld(int i, unsigned off, C ref) const {
        const S v = Bits<S>::ld(r, off, pb * (unsigned)i);
        return Io<S, C>::ld(&v, 0, ref);
    }
    template <typename C>
    __device__ void st(int i, unsigned off, C v, C ref, bool valid) const {
        S t;
        Io<S, C>::st(&t, 0, v, ref);
        Bits<S>::st(t, r, valid ? off : drop, pb * (unsigned)i);
    }
};

template <typename S>
struct Planes<S, false> {
    char* base;
    size_t pb;
    __device__ Planes(const void* b, size_t plane_bytes) : base((char*)b), pb(plane_bytes) {}
    template <typename C>
    __device__ C ld(int i, unsigned off, C ref) const {
        return Io<S, C>::ld(reinterpret_cast<const S*>(base + pb * i + off), 0, ref);
    }
    template <typename C>
    __device__ void st(int i, unsigned off, C v, C ref, bool valid) const {
        if (valid) Io<S, C>::st(reinterpret_cast<S*>(base + pb * i + off), 0, v, ref);
    }
};

template <typename S, typename C, bool kBuf>
__device__ inline void load_row9(const Planes<S, kBuf>& B, int first, unsigned off, const C* ref, C* v) {
#pragma unroll
    for (int i = 0; i < 9; ++i) v[i] = B.template ld<C>(first + i, off, ref[i]);
}

template <typename C>
__device__ inline C sum9(const C* f) {
    return f[0] + ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]));
}

struct StripGeom {
    int nx, ny;
    unsigned xc, xe, xw, rowb, esz;
    bool owner;
    __device__ unsigned off(int y, unsigned x) const { return (unsigned)y * rowb + x * esz; }
};

// One row of the marching update.  kStage = 2: issue the loads two rows ahead
// (g of row y+2, f of row y+3), collide row y, rotate the register ring; kStage = 1:
// collide and rotate without new loads; kStage = 0: collide only (last row).
template <int kStage, typename S, typename C, bool kBuf>
__device__ __forceinline__ void ab_row(const Consts<C>& P, const Planes<S, kBuf>& in, const Planes<S, kBuf>& out,
                                       const StripGeom& G, int y, C (&fA)[9], C (&fB)[9], C (&fC)[9], C (&gA)[9],
                                       C (&gB)[9], C& rm, C& rc, C& rp) {
    C fD[9], gC[9];
    if (kStage == 2) {
        load_row9<S, C, kBuf>(in, 9, G.off(wrap(y + 2, G.ny), G.xc), P.ref_g, gC);
        load_row9<S, C, kBuf>(in, 0, G.off(wrap(y + 3, G.ny), G.xc), P.ref_f, fD);
    }
    // neighbour densities: lane L-1 is x-1 (west), lane L+1 is x+1 (east)
    const C rW = __shfl_up(rc, 1), rE = __shfl_down(rc, 1);
    const C rSW = __shfl_up(rm, 1), rSE = __shfl_down(rm, 1);
    const C rNW = __shfl_up(rp, 1), rNE = __shfl_down(rp, 1);
    auto body = [&]() {
        C sx, sy;
        stencil(rE, rp, rW, rm, rNE, rNW, rSW, rSE, sx, sy);
        C fo[9], go[9];
        collide(P, fA, gA, rc, sx, sy, fo, go);
        const int yn = y + 1 == G.ny ? 0 : y + 1, ys = y == 0 ? G.ny - 1 : y - 1;
        const unsigned dst[9] = {G.off(y, G.xc), G.off(y, G.xe), G.off(yn, G.xc), G.off(y, G.xw), G.off(ys, G.xc),
                                 G.off(yn, G.xe), G.off(yn, G.xw), G.off(ys, G.xw), G.off(ys, G.xe)};
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            out.template st<C>(i, dst[i], fo[i], P.ref_f[i], G.owner);
            out.template st<C>(9 + i, dst[i], go[i], P.ref_g[i], G.owner);
        }
    };
    if (kBuf) body();          // every lane runs the row; halo lanes' stores are dropped
    else if (G.owner) body();
    if (kStage >= 1) {
        rm = rc;
        rc = rp;
        rp = sum9(fC);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            fA[i] = fB[i];
            fB[i] = fC[i];
            gA[i] = gB[i];
            if (kStage == 2) {
                fC[i] = fD[i];
                gB[i] = gC[i];
            }
        }
    }
}

template <typename S, typename C, int WPB, bool kBuf>
__global__ void __launch_bounds__(64 * WPB)
k_step_ab(const S* __restrict__ in, S* __restrict__ out, const Consts<C> P, const int nstrips,
          const int rows, const int nitems) {
    const int lane = threadIdx.x & 63;
    const int w = remap_xcd(blockIdx.x, gridDim.x) * WPB + (threadIdx.x >> 6);
    if (w >= nitems) return;
    const int strip = w % nstrips, chunk = w / nstrips;
    const int nx = P.nx, ny = P.ny;
    const int x0 = strip * 62;
    const int owned = min(62, nx - x0);
    const bool active = lane <= owned + 1;
    StripGeom G;
    G.nx = nx;
    G.ny = ny;
    G.owner = lane >= 1 && lane <= owned;
    // inactive lanes read column 0 (a valid address) and never store
    G.xc = active ? (unsigned)wrap(x0 - 1 + lane, nx) : 0u;
    G.xe = G.xc + 1 == (unsigned)nx ? 0u : G.xc + 1;
    G.xw = G.xc == 0 ? (unsigned)nx - 1 : G.xc - 1;
    G.rowb = (unsigned)nx * sizeof(S);
    G.esz = sizeof(S);
    const size_t pb = (size_t)nx * ny * sizeof(S);
    const Planes<S, kBuf> Pin(in, pb);
    const Planes<S, kBuf> Pout(out, pb);
    const int y0 = chunk * rows, y1 = min(ny, y0 + rows);

    // register ring: f of rows y, y+1, y+2 and g of rows y, y+1; densities of rows y-1..y+1
    C fA[9], fB[9], fC[9], gA[9], gB[9];
    C rm, rc, rp;
    {
        C t[9];
        load_row9<S, C, kBuf>(Pin, 0, G.off(wrap(y0 - 1, ny), G.xc), P.ref_f, t);
        rm = sum9(t);
    }
    load_row9<S, C, kBuf>(Pin, 0, G.off(y0, G.xc), P.ref_f, fA);
    load_row9<S, C, kBuf>(Pin, 0, G.off(wrap(y0 + 1, ny), G.xc), P.ref_f, fB);
    load_row9<S, C, kBuf>(Pin, 9, G.off(y0, G.xc), P.ref_g, gA);
    load_row9<S, C, kBuf>(Pin, 9, G.off(wrap(y0 + 1, ny), G.xc), P.ref_g, gB);
    load_row9<S, C, kBuf>(Pin, 0, G.off(wrap(y0 + 2, ny), G.xc), P.ref_f, fC);
    rc = sum9(fA);
    rp = sum9(fB);
    // Let the prologue's loads land before the loop: the loop header then sees only
    // the pipelined state, and the memory-counter waits inside the loop cover just the
    // loads issued in earlier rows (not the stores of the previous row).
#pragma unroll
    for (int i = 0; i < 9; ++i) asm volatile("" ::"v"(gA[i]), "v"(gB[i]), "v"(fC[i]));
    int y = y0;
    for (; y < y1 - 2; ++y) ab_row<2, S, C, kBuf>(P, Pin, Pout, G, y, fA, fB, fC, gA, gB, rm, rc, rp);
    if (y < y1 - 1) ab_row<1, S, C, kBuf>(P, Pin, Pout, G, y++, fA, fB, fC, gA, gB, rm, rc, rp);
    ab_row<0, S, C, kBuf>(P, Pin, Pout, G, y, fA, fB, fC, gA, gB, rm, rc, rp);
}

// ---------------------------------------------------------------------------
// AA pattern (one buffer, in place).  Even step: node x reads slot i of x and
// writes its post-collision f_i to slot opp(i) of x.  Odd step: node x reads
// slot opp(i) of x - e_i and writes slot i of x + e_i.  Each node's read set
// equals its write set, so the update is race-free in place; the density
// stencil reads a separate array written by k_density beforehand.
// ---------------------------------------------------------------------------
template <typename S, typename C>
__device__ inline void aa_offsets(int parity, int x, int y, int nx, int ny, int* rd_slot, int* rd_off,
                                  int* wr_slot, int* wr_off) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if (parity == 0) {
            rd_slot[i] = i;
            rd_off[i] = y * nx + x;
            wr_slot[i] = kOpp[i];
            wr_off[i] = rd_off[i];
        } else {
            rd_slot[i] = kOpp[i];
            rd_off[i] = wrap(y - kEy[i], ny) * nx + wrap(x - kEx[i], nx);
            wr_slot[i] = i;
            wr_off[i] = wrap(y + kEy[i], ny) * nx + wrap(x + kEx[i], nx);
        }
    }
}

template <typename S, typename C>
__global__ void __launch_bounds__(256)
k_step_aa(S* __restrict__ st, const double* __restrict__ rho_arr, const Consts<C> P, const int parity) {
    using IO = Io<S, C>;
    const int nx = P.nx, ny = P.ny, N = nx * ny;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    int rs[9], ro[9], ws[9], wo[9];
    aa_offsets<S, C>(parity, x, y, nx, ny, rs, ro, ws, wo);
    C f[9], g[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        f[i] = IO::ld(st + (size_t)rs[i] * N, ro[i], P.ref_f[i]);
        g[i] = IO::ld(st + (size_t)(9 + rs[i]) * N, ro[i], P.ref_g[i]);
    }
    const int xe = wrap(x + 1, nx), xw = wrap(x - 1, nx);
    const int yn = wrap(y + 1, ny) * nx, ys = wrap(y - 1, ny) * nx, yc = y * nx;
    const C rho = (C)rho_arr[yc + x];
    C sx, sy;
    stencil((C)rho_arr[yc + xe], (C)rho_arr[yn + x], (C)rho_arr[yc + xw], (C)rho_arr[ys + x],
            (C)rho_arr[yn + xe], (C)rho_arr[yn + xw], (C)rho_arr[ys + xw], (C)rho_arr[ys + xe], sx, sy);
    C fo[9], go[9];
    collide(P, f, g, rho, sx, sy, fo, go);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        IO::st(st + (size_t)ws[i] * N, wo[i], fo[i], P.ref_f[i]);
        IO::st(st + (size_t)(9 + ws[i]) * N, wo[i], go[i], P.ref_g[i]);
    }
}

// Populations of node (x, y) at the current time, for either scheme: AA parity
// 0 is also the layout of the two-buffer scheme.
template <typename S, typename C>
__device__ inline void load_node(const S* st, const Consts<C>& P, int parity, int x, int y, C* f, C* g) {
    using IO = Io<S, C>;
    const int nx = P.nx, ny = P.ny, N = nx * ny;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int slot = i, off = y * nx + x;
        if (parity) {
            slot = kOpp[i];
            off = wrap(y - kEy[i], ny) * nx + wrap(x - kEx[i], nx);
        }
        f[i] = IO::ld(st + (size_t)slot * N, off, P.ref_f[i]);
        g[i] = IO::ld(st + (size_t)(9 + slot) * N, off, P.ref_g[i]);
    }
}

template <typename S, typename C>
__global__ void __launch_bounds__(256)
k_init(S* __restrict__ st, const double* __restrict__ rho_in, const double* __restrict__ ux_in,
       const double* __restrict__ uy_in, const double* __restrict__ T_in, const Consts<C> P) {
    using IO = Io<S, C>;
    const int N = P.nx * P.ny;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= N) return;
    const C rho = (C)rho_in[k], u = (C)ux_in[k], v = (C)uy_in[k], T = (C)T_in[k];
    const C ux = u * P.inv_c, uy = v * P.inv_c;
    const C pbe = p_be(P, rho, T);
    const C eta = pbe * P.inv_cs2 - rho;
    const C ru2 = rho * (ux * ux + uy * uy);
    C m[9], f[9];
    m[0] = rho;
    m[1] = C(-2) * rho + C(2) * eta + C(3) * ru2;
    m[2] = rho + P.beta * eta - C(3) * ru2;
    m[3] = rho * ux;
    m[4] = -rho * ux;
    m[5] = rho * uy;
    m[6] = -rho * uy;
    m[7] = rho * (ux * ux - uy * uy);
    m[8] = rho * ux * uy;
    from_moments(m, f);
    const C rek = rho * (P.cv * T + C(0.5) * (u * u + v * v));
    const C rhk = rek + pbe;
    C n[9], g[9];
    n[0] = rek;
    n[1] = C(-4) * rek + P.g1C * T;
    n[2] = C(4) * rek - P.g2C * T;
    n[3] = rhk * ux;
    n[4] = -rhk * ux;
    n[5] = rhk * uy;
    n[6] = -rhk * uy;
    n[7] = C(0);
    n[8] = C(0);
    from_moments(n, g);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        IO::st(st + (size_t)i * N, k, f[i], P.ref_f[i]);
        IO::st(st + (size_t)(9 + i) * N, k, g[i], P.ref_g[i]);
    }
}

template <typename S, typename C>
__global__ void __launch_bounds__(256)
k_density(const S* __restrict__ st, const Consts<C> P, const int parity, double* __restrict__ rho) {
    const int N = P.nx * P.ny;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= N) return;
    const int y = k / P.nx, x = k - y * P.nx;
    C f[9], g[9];
    load_node(st, P, parity, x, y, f, g);
    rho[k] = (double)(f[0] + ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8])));
}

template <typename C>
__device__ inline void neighbour_sums(const double* rho, const Consts<C>& P, int x, int y, C& sx, C& sy,
                                      C& wsum) {
    const int nx = P.nx, ny = P.ny;
    const int xe = wrap(x + 1, nx), xw = wrap(x - 1, nx);
    const int yn = wrap(y + 1, ny) * nx, ys = wrap(y - 1, ny) * nx, yc = y * nx;
    const C rE = (C)rho[yc + xe], rN = (C)rho[yn + x], rW = (C)rho[yc + xw], rS = (C)rho[ys + x];
    const C rNE = (C)rho[yn + xe], rNW = (C)rho[yn + xw], rSW = (C)rho[ys + xw], rSE = (C)rho[ys + xe];
    stencil(rE, rN, rW, rS, rNE, rNW, rSW, rSE, sx, sy);
    wsum = (C(1) / C(3)) * ((rE + rN) + (rW + rS)) + (C(1) / C(12)) * ((rNE + rNW) + (rSW + rSE));
}

template <typename S, typename C>
__global__ void __launch_bounds__(256)
k_moments(const S* __restrict__ st, const Consts<C> P, const int parity, const double* __restrict__ rho,
          double* __restrict__ ux, double* __restrict__ uy, double* __restrict__ T) {
    const int N = P.nx * P.ny;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= N) return;
    const int y = k / P.nx, x = k - y * P.nx;
    C f[9], g[9], m[9], n[9];
    load_node(st, P, parity, x, y, f, g);
    to_moments(f, m);
    to_moments(g, n);
    C sx, sy, ws;
    neighbour_sums(rho, P, x, y, sx, sy, ws);
    const Macro<C> M = macros(P, (C)rho[k], m[3], m[5], n[0], sx, sy);
    if (ux) ux[k] = (double)(P.c * M.uxh);
    if (uy) uy[k] = (double)(P.c * M.uyh);
    if (T) T[k] = (double)M.T;
}

// Per-block FP64 partial sums of the 8 diagnostics, in a fixed order.
template <typename S, typename C>
__global__ void __launch_bounds__(256)
k_invariants(const S* __restrict__ st, const Consts<C> P, const int parity, const double* __restrict__ rho,
             double* __restrict__ partials) {
    const int N = P.nx * P.ny;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = blockIdx.x * 256 + threadIdx.x; k < N; k += gridDim.x * 256) {
        const int y = k / P.nx, x = k - y * P.nx;
        C f[9], g[9], m[9], n[9];
        load_node(st, P, parity, x, y, f, g);
        to_moments(f, m);
        to_moments(g, n);
        C sx, sy, ws;
        neighbour_sums(rho, P, x, y, sx, sy, ws);
        const C r = (C)rho[k];
        const Macro<C> M = macros(P, r, m[3], m[5], n[0], sx, sy);
        double mass = 0, sg = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            mass += (double)f[i];
            sg += (double)g[i];
        }
        acc[0] += mass;
        acc[1] += (double)P.c * (double)m[3];
        acc[2] += (double)P.c * (double)m[5];
        acc[3] += sg;
        acc[4] += (double)P.dt * (double)M.q;
        acc[5] += (double)P.Ep_pre * ((double)r * (double)r / 6.0 + 0.5 * (double)r * (double)ws);
        acc[6] += (double)M.rho_ek;
        bool bad = !(r > C(0)) || !(M.T > C(0)) || !isfinite((double)M.T) || !isfinite((double)M.rho_ek);
        if (P.eos_kind == 0) bad = bad || !(P.bq * r < C(1));
        else bad = bad || !(P.bq * r < C(1));
        acc[7] += bad ? 1.0 : 0.0;
    }
    __shared__ double sm[8][256];
#pragma unroll
    for (int j = 0; j < 8; ++j) sm[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int j = 0; j < 8; ++j) sm[j][threadIdx.x] += sm[j][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x < 8) partials[blockIdx.x * 8 + threadIdx.x] = sm[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_reduce_partials(const double* __restrict__ partials, int nblocks,
                                                         double* __restrict__ out) {
    __shared__ double sm[8][256];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += 256) {
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] += partials[b * 8 + j];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) sm[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int j = 0; j < 8; ++j) sm[j][threadIdx.x] += sm[j][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x < 8) out[threadIdx.x] = sm[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename S, typename C>
struct Launch {
    static hipError_t init(const void* cv, void* st, const double* r, const double* u, const double* v,
                           const double* T, hipStream_t s) {
        const Consts<C>& P = *static_cast<const Consts<C>*>(cv);
        const int N = P.nx * P.ny;
        hipLaunchKernelGGL((k_init<S, C>), dim3((N + 255) / 256), dim3(256), 0, s, static_cast<S*>(st), r,
                           u, v, T, P);
        return hipGetLastError();
    }
    template <bool kBuf>
    static hipError_t step_ab_wpb(const S* i, S* o, const Consts<C>& P, int nstrips, int rows, int nitems, int wpb,
                                  int nblocks, hipStream_t s) {
        switch (wpb) {
            case 1: hipLaunchKernelGGL((k_step_ab<S, C, 1, kBuf>), dim3(nblocks), dim3(64), 0, s, i, o, P, nstrips, rows, nitems); break;
            case 2: hipLaunchKernelGGL((k_step_ab<S, C, 2, kBuf>), dim3(nblocks), dim3(128), 0, s, i, o, P, nstrips, rows, nitems); break;
            case 4: hipLaunchKernelGGL((k_step_ab<S, C, 4, kBuf>), dim3(nblocks), dim3(256), 0, s, i, o, P, nstrips, rows, nitems); break;
            case 8: hipLaunchKernelGGL((k_step_ab<S, C, 8, kBuf>), dim3(nblocks), dim3(512), 0, s, i, o, P, nstrips, rows, nitems); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    static hipError_t step_ab(const void* cv, const void* in, void* out, LaunchShape sh, hipStream_t s) {
        const Consts<C>& P = *static_cast<const Consts<C>*>(cv);
        const int nstrips = (P.nx + 61) / 62;
        const int rows = sh.rows_per_wave;
        const int nchunks = (P.ny + rows - 1) / rows;
        const int nitems = nstrips * nchunks;
        const int wpb = sh.waves_per_block;
        const int nblocks = (nitems + wpb - 1) / wpb;
        const S* i = static_cast<const S*>(in);
        S* o = static_cast<S*>(out);
        // raw buffer addressing needs every plane offset and the drop offset in 32 bits
        const bool kBuf = (size_t)35 * P.nx * P.ny * sizeof(S) < ((size_t)1 << 32);
        if (kBuf) return step_ab_wpb<true>(i, o, P, nstrips, rows, nitems, wpb, nblocks, s);
        return step_ab_wpb<false>(i, o, P, nstrips, rows, nitems, wpb, nblocks, s);
    }
    static hipError_t step_aa(const void* cv, void* st, double* rho, int parity, LaunchShape, hipStream_t s) {
        const Consts<C>& P = *static_cast<const Consts<C>*>(cv);
        const int N = P.nx * P.ny;
        hipLaunchKernelGGL((k_density<S, C>), dim3((N + 255) / 256), dim3(256), 0, s,
                           static_cast<const S*>(st), P, parity, rho);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_step_aa<S, C>), dim3((P.nx + 63) / 64, (P.ny + 3) / 4), dim3(256), 0, s,
                           static_cast<S*>(st), rho, P, parity);
        return hipGetLastError();
    }
    static hipError_t density(const void* cv, const void* st, int parity, double* rho, hipStream_t s) {
        const Consts<C>& P = *static_cast<const Consts<C>*>(cv);
        const int N = P.nx * P.ny;
        hipLaunchKernelGGL((k_density<S, C>), dim3((N + 255) / 256), dim3(256), 0, s,
                           static_cast<const S*>(st), P, parity, rho);
        return hipGetLastError();
    }
    static hipError_t moments(const void* cv, const void* st, int parity, const double* rho, double* ux,
                              double* uy, double* T, hipStream_t s) {
        const Consts<C>& P = *static_cast<const Consts<C>*>(cv);
        const int N = P.nx * P.ny;
        hipLaunchKernelGGL((k_moments<S, C>), dim3((N + 255) / 256), dim3(256), 0, s,
                           static_cast<const S*>(st), P, parity, rho, ux, uy, T);
        return hipGetLastError();
    }
    static hipError_t invariants(const void* cv, const void* st, int parity, const double* rho,
                                 double* partials, double* result, hipStream_t s) {
        const Consts<C>& P = *static_cast<const Consts<C>*>(cv);
        const int N = P.nx * P.ny;
        int nb = (N + 255) / 256;
        if (nb > kMaxPartialBlocks) nb = kMaxPartialBlocks;
        hipLaunchKernelGGL((k_invariants<S, C>), dim3(nb), dim3(256), 0, s, static_cast<const S*>(st), P,
                           parity, rho, partials);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, partials, nb, result);
        return hipGetLastError();
    }
};

}  // namespace

#define LBM_DISPATCH(prec, call)                                        \
    switch (prec) {                                                     \
        case kF64: return Launch<double, double>::call;                 \
        case kF32: return Launch<float, float>::call;                   \
        case kF16: return Launch<__half, float>::call;                  \
        case kBF16: return Launch<__hip_bfloat16, float>::call;         \
        default: return hipErrorInvalidValue;                           \
    }

hipError_t launch_init(int prec, const void* c, void* state, const double* rho, const double* ux,
                       const double* uy, const double* T, hipStream_t stream) {
    LBM_DISPATCH(prec, init(c, state, rho, ux, uy, T, stream));
}
hipError_t launch_step_ab(int prec, const void* c, const void* in, void* out, LaunchShape shape,
                          hipStream_t stream) {
    LBM_DISPATCH(prec, step_ab(c, in, out, shape, stream));
}
hipError_t launch_step_aa(int prec, const void* c, void* state, double* rho_scratch, int parity,
                          LaunchShape shape, hipStream_t stream) {
    LBM_DISPATCH(prec, step_aa(c, state, rho_scratch, parity, shape, stream));
}
hipError_t launch_density(int prec, const void* c, const void* state, int aa_parity, double* rho,
                          hipStream_t stream) {
    LBM_DISPATCH(prec, density(c, state, aa_parity, rho, stream));
}
hipError_t launch_moments(int prec, const void* c, const void* state, int aa_parity, const double* rho,
                          double* ux, double* uy, double* T, hipStream_t stream) {
    LBM_DISPATCH(prec, moments(c, state, aa_parity, rho, ux, uy, T, stream));
}
hipError_t launch_invariants(int prec, const void* c, const void* state, int aa_parity, const double* rho,
                             double* partials, double* result, hipStream_t stream) {
    LBM_DISPATCH(prec, invariants(c, state, aa_parity, rho, partials, result, stream));
}

size_t consts_size(int prec) { return prec == kF64 ? sizeof(Consts<double>) : sizeof(Consts<float>); }
size_t storage_bytes(int prec) { return prec == kF64 ? 8 : (prec == kF32 ? 4 : 2); }

}  // namespace lbm_dev
