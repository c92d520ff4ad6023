// HIP kernels for lattices bounded in x: the one-dimensional Stefan problem of the paper
// (a long, narrow domain heated from one side, Eqs. (20)-(21)), with y periodic.
//
// Boundary treatment: non-equilibrium extrapolation (Guo, Zheng and Shi 2002) stands in
// for the improved scheme the paper cites: the post-collision populations of a boundary
// node are the equilibrium at the boundary's macroscopic state plus the non-equilibrium
// part of the neighbouring fluid node,
//     l_bar_i(x_b) = l_i^eq(rho_b, u_b, T_b) + [l_bar_i(x_n) - l_i^eq(x_n)],  l = f, g.
// x = 0 is a heated wall with vapour outflow at constant pressure (T_b = T_wall, rho_b
// the vapour density at p_out and T_wall, u_b = u of column 1); x = nx - 1 is a wall at
// rest (u_b = 0, T_b = T_far, rho_b = rho of column nx - 2).  The pair force of Eq. (13)
// at a fluid node next to a boundary takes rho_b as the boundary node's density.
// Boundary columns carry no state: the thread of the neighbouring fluid column writes
// their post-collision populations every step, and nothing reads what streams into them.
//
// These domains are small (the paper's is 1024 x 4 nodes) and are stepped millions of
// times, so one workgroup marches the whole lattice through many steps per launch, with
// the densities of each step in LDS and a workgroup barrier between the density pass
// and the collide-stream pass.  Same state layout and pull convention as the periodic
// two-buffer update.

#include <hip/hip_runtime.h>

#include "lbm_internal.hpp"
#include "lbm_model.hpp"

namespace lbm_dev {
namespace {

// Populations of fluid node (x, y), pulled: slot i at (x - e_ix, y - e_iy), y periodic.
template <typename C>
__device__ inline void pull_node(const C* st, int nx, int ny, int x, int y, C* f, C* g) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int xs = x - kEx[i], ys = wrap(y - kEy[i], ny);
        f[i] = st[slot_index(i, xs, ys, nx)];
        g[i] = st[slot_index(9 + i, xs, ys, nx)];
    }
}

template <typename C>
__device__ inline C density(const C* f) {
    return f[0] + ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]));
}

// Density of node (x, y) for the stencil: the fluid density, or the boundary's.
template <typename C>
__device__ inline C node_density(const C* st, const Walls<C>& W, int nx, int ny, int x, int y) {
    C f[9], g[9];
    if (x == 0) return W.rho_wall;
    pull_node(st, nx, ny, x == nx - 1 ? nx - 2 : x, y, f, g);
    return density(f);
}

template <typename C>
__device__ inline void stencil_at(const C* rho, int nx, int ny, int x, int y, C& sx, C& sy) {
    const int yn = wrap(y + 1, ny) * nx, ys = wrap(y - 1, ny) * nx, yc = y * nx;
    stencil(rho[yc + x + 1], rho[yn + x], rho[yc + x - 1], rho[ys + x], rho[yn + x + 1], rho[yn + x - 1],
            rho[ys + x - 1], rho[ys + x + 1], sx, sy);
}

// Equilibrium populations M^-1 m^eq and M^-1 n^eq (SM Eqs. (3a), (4a)) of a state given
// by rho, u/c, T, rho e_k and p_BE.
template <typename C>
__device__ inline void equilibria(const Consts<C>& P, C rho, C uxh, C uyh, C T, C rek, C pbe, C* f, C* g) {
    const C eta = pbe * P.inv_cs2 - rho;
    const C ru2 = rho * (uxh * uxh + uyh * uyh);
    C m[9];
    m[0] = rho;
    m[1] = C(-2) * rho + C(2) * eta + C(3) * ru2;
    m[2] = rho + P.beta * eta - C(3) * ru2;
    m[3] = rho * uxh;
    m[4] = -rho * uxh;
    m[5] = rho * uyh;
    m[6] = -rho * uyh;
    m[7] = rho * (uxh * uxh - uyh * uyh);
    m[8] = rho * uxh * uyh;
    from_moments(m, f);
    const C rhk = rek + pbe;
    C n[9];
    n[0] = rek;
    n[1] = C(-4) * rek + P.g1C * T;
    n[2] = C(4) * rek - P.g2C * T;
    n[3] = rhk * uxh;
    n[4] = -rhk * uxh;
    n[5] = rhk * uyh;
    n[6] = -rhk * uyh;
    n[7] = C(0);
    n[8] = C(0);
    from_moments(n, g);
}

// Macroscopic state of fluid node (x, y) at the current time (Eq. (14)).
template <typename C>
__device__ inline Macro<C> node_macros(const Consts<C>& P, const C* f, const C* g, C rho, C sx, C sy) {
    C m[9], n[9];
    to_moments(f, m);
    to_moments(g, n);
    return macros(P, rho, m[3], m[5], n[0], sx, sy);
}

template <typename C>
__global__ void __launch_bounds__(kBoundedThreads)
k_step_bounded(const Consts<C> P, const Walls<C> W, C* __restrict__ b0, C* __restrict__ b1, int first, int steps) {
    __shared__ C rho_s[kMaxBoundedNodes];
    const int nx = P.nx, ny = P.ny, N = nx * ny;
    for (int k = 0; k < steps; ++k) {
        const C* in = ((first + k) & 1) ? b1 : b0;
        C* out = ((first + k) & 1) ? b0 : b1;
        for (int n = threadIdx.x; n < N; n += kBoundedThreads) {
            const int y = n / nx, x = n - y * nx;
            rho_s[n] = node_density(in, W, nx, ny, x, y);
        }
        __syncthreads();
        for (int n = threadIdx.x; n < N; n += kBoundedThreads) {
            const int y = n / nx, x = n - y * nx;
            if (x == 0 || x == nx - 1) continue;
            C f[9], g[9], fo[9], go[9];
            pull_node(in, nx, ny, x, y, f, g);
            const C rho = rho_s[n];
            C sx, sy;
            stencil_at(rho_s, nx, ny, x, y, sx, sy);
            collide(P, f, g, rho, sx, sy, fo, go);
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                out[slot_index(i, x, y, nx)] = fo[i];
                out[slot_index(9 + i, x, y, nx)] = go[i];
            }
            if (x != 1 && x != nx - 2) continue;
            // non-equilibrium extrapolation to the boundary column(s) next to this node
            const Macro<C> M = node_macros(P, f, g, rho, sx, sy);
            const C pbe = p_be(P, rho, M.T);
            C fe[9], ge[9];
            equilibria(P, rho, M.uxh, M.uyh, M.T, M.rho_ek, pbe, fe, ge);
            for (int side = 0; side < 2; ++side) {
                const bool left = side == 0;
                if ((left && x != 1) || (!left && x != nx - 2)) continue;
                const int xb = left ? 0 : nx - 1;
                const C rb = left ? W.rho_wall : rho;
                const C Tb = left ? W.T_wall : W.T_far;
                const C ub = left ? M.uxh : C(0), vb = left ? M.uyh : C(0);
                const C rek_b = rb * (P.cv * Tb + C(0.5) * P.c2 * (ub * ub + vb * vb));
                C fb[9], gb[9];
                equilibria(P, rb, ub, vb, Tb, rek_b, p_be(P, rb, Tb), fb, gb);
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    out[slot_index(i, xb, y, nx)] = fb[i] + (fo[i] - fe[i]);
                    out[slot_index(9 + i, xb, y, nx)] = gb[i] + (go[i] - ge[i]);
                }
            }
        }
        // the next step's density pass reads what the other threads wrote
        __threadfence_block();
        __syncthreads();
    }
}

// Moments of the current state; boundary columns report the imposed boundary state
// (heated side: u of column 1).
template <typename C>
__global__ void __launch_bounds__(kBoundedThreads)
k_moments_bounded(const Consts<C> P, const Walls<C> W, const C* __restrict__ st, double* __restrict__ rho,
                  double* __restrict__ ux, double* __restrict__ uy, double* __restrict__ T) {
    __shared__ C rho_s[kMaxBoundedNodes];
    const int nx = P.nx, ny = P.ny, N = nx * ny;
    for (int n = threadIdx.x; n < N; n += kBoundedThreads) {
        const int y = n / nx, x = n - y * nx;
        rho_s[n] = node_density(st, W, nx, ny, x, y);
    }
    __syncthreads();
    for (int n = threadIdx.x; n < N; n += kBoundedThreads) {
        const int y = n / nx, x = n - y * nx;
        rho[n] = (double)rho_s[n];
        if (x == nx - 1) {
            if (ux) ux[n] = 0.0;
            if (uy) uy[n] = 0.0;
            if (T) T[n] = (double)W.T_far;
            continue;
        }
        const int xf = x == 0 ? 1 : x;  // the heated side reports column 1's velocity
        C f[9], g[9];
        pull_node(st, nx, ny, xf, y, f, g);
        C sx, sy;
        stencil_at(rho_s, nx, ny, xf, y, sx, sy);
        const Macro<C> M = node_macros(P, f, g, rho_s[y * nx + xf], sx, sy);
        if (ux) ux[n] = (double)(P.c * M.uxh);
        if (uy) uy[n] = (double)(P.c * M.uyh);
        if (T) T[n] = x == 0 ? (double)W.T_wall : (double)M.T;
    }
}

// The 8 diagnostics of the periodic lbm_invariants over the fluid columns: each thread
// sums its nodes in order, then a fixed-order tree in LDS.
template <typename C>
__global__ void __launch_bounds__(kBoundedThreads)
k_invariants_bounded(const Consts<C> P, const Walls<C> W, const C* __restrict__ st, double* __restrict__ out) {
    // the densities, then (after the node loop) the reduction tree, in one LDS buffer
    constexpr int kWords = (kMaxBoundedNodes * (int)sizeof(C) > 8 * (kBoundedThreads / 4) * 8)
                               ? kMaxBoundedNodes * (int)sizeof(C) / 8 : 8 * (kBoundedThreads / 4);
    __shared__ double lds[kWords];
    C* rho_s = reinterpret_cast<C*>(lds);
    double (*sm)[kBoundedThreads / 4] = reinterpret_cast<double (*)[kBoundedThreads / 4]>(lds);
    const int nx = P.nx, ny = P.ny, N = nx * ny;
    for (int n = threadIdx.x; n < N; n += kBoundedThreads) {
        const int y = n / nx, x = n - y * nx;
        rho_s[n] = node_density(st, W, nx, ny, x, y);
    }
    __syncthreads();
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int n = threadIdx.x; n < N; n += kBoundedThreads) {
        const int y = n / nx, x = n - y * nx;
        if (x == 0 || x == nx - 1) continue;
        C f[9], g[9], m[9], nn[9];
        pull_node(st, nx, ny, x, y, f, g);
        to_moments(f, m);
        to_moments(g, nn);
        const C r = rho_s[n];
        C sx, sy;
        stencil_at(rho_s, nx, ny, x, y, sx, sy);
        const Macro<C> M = macros(P, r, m[3], m[5], nn[0], sx, sy);
        const int yn = wrap(y + 1, ny) * nx, ys = wrap(y - 1, ny) * nx, yc = y * nx;
        const C ws = (C(1) / C(3)) * ((rho_s[yc + x + 1] + rho_s[yn + x]) + (rho_s[yc + x - 1] + rho_s[ys + x])) +
                     (C(1) / C(12)) * ((rho_s[yn + x + 1] + rho_s[yn + x - 1]) + (rho_s[ys + x - 1] + rho_s[ys + x + 1]));
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
        const bool bad = !(r > C(0)) || !(M.T > C(0)) || !isfinite((double)M.T) || !isfinite((double)M.rho_ek) ||
                         !(P.bq * r < C(1));
        acc[7] += bad ? 1.0 : 0.0;
    }
    __syncthreads();  // every density read is done before the buffer becomes the tree
    // four threads' sums per LDS slot first (fixed pairing), then a tree
    const int t = threadIdx.x, slot = t >> 2;
    for (int q = 0; q < 4; ++q) {
        if ((t & 3) == q) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (q == 0) sm[j][slot] = acc[j];
                else sm[j][slot] += acc[j];
            }
        }
        __syncthreads();
    }
    for (int s = kBoundedThreads / 8; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int j = 0; j < 8; ++j) sm[j][t] += sm[j][t + s];
        }
        __syncthreads();
    }
    if (t < 8) out[t] = sm[t][0];
}

template <typename C>
hipError_t step_bounded(const void* c, const void* w, void* b0, void* b1, int first, int steps, hipStream_t s) {
    hipLaunchKernelGGL((k_step_bounded<C>), dim3(1), dim3(kBoundedThreads), 0, s,
                       *static_cast<const Consts<C>*>(c), *static_cast<const Walls<C>*>(w), static_cast<C*>(b0),
                       static_cast<C*>(b1), first, steps);
    return hipGetLastError();
}

template <typename C>
hipError_t moments_bounded(const void* c, const void* w, const void* st, double* rho, double* ux, double* uy,
                           double* T, hipStream_t s) {
    hipLaunchKernelGGL((k_moments_bounded<C>), dim3(1), dim3(kBoundedThreads), 0, s,
                       *static_cast<const Consts<C>*>(c), *static_cast<const Walls<C>*>(w),
                       static_cast<const C*>(st), rho, ux, uy, T);
    return hipGetLastError();
}

template <typename C>
hipError_t invariants_bounded(const void* c, const void* w, const void* st, double* out, hipStream_t s) {
    hipLaunchKernelGGL((k_invariants_bounded<C>), dim3(1), dim3(kBoundedThreads), 0, s,
                       *static_cast<const Consts<C>*>(c), *static_cast<const Walls<C>*>(w),
                       static_cast<const C*>(st), out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step_bounded(int prec, const void* c, const void* walls, void* buf0, void* buf1, int first,
                               int steps, hipStream_t stream) {
    if (prec == kF64) return step_bounded<double>(c, walls, buf0, buf1, first, steps, stream);
    if (prec == kF32) return step_bounded<float>(c, walls, buf0, buf1, first, steps, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_moments_bounded(int prec, const void* c, const void* walls, const void* state, double* rho,
                                  double* ux, double* uy, double* T, hipStream_t stream) {
    if (prec == kF64) return moments_bounded<double>(c, walls, state, rho, ux, uy, T, stream);
    if (prec == kF32) return moments_bounded<float>(c, walls, state, rho, ux, uy, T, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_invariants_bounded(int prec, const void* c, const void* walls, const void* state,
                                     double* result, hipStream_t stream) {
    if (prec == kF64) return invariants_bounded<double>(c, walls, state, result, stream);
    if (prec == kF32) return invariants_bounded<float>(c, walls, state, result, stream);
    return hipErrorInvalidValue;
}

}  // namespace lbm_dev
