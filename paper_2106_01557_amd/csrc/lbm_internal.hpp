// Internal interface between the C ABI (lbm_api.cpp) and the HIP kernels
// (lbm_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lbm_dev {

// Per-run constants in the arithmetic type C of the kernels.  Built once on the
// host; passed by value to every launch.
template <typename C>
struct Consts {
    int32_t nx, ny;
    int32_t eos_kind;      // 0 CS, 1 vdW
    uint32_t step;         // steps completed before this launch (the stochastic-rounding stream)
    C G2dx;                // G^2 dx: F_pair = G^2 dx rho sum_i w_i rho(x + e_i dx) e_i/c (Eq. (13))
    C inv_dx;              // grad rho = sum_i w_i rho_i (e_i/c) / dx
    C ax, ay;              // external acceleration
    C c, inv_c, c2;        // lattice speed c = dx/dt
    C dt, hdt, hdt_c;      // dt, dt/2, dt/(2c)
    C inv_cv, cv, C_ref;
    C KR, Ka, bq;          // K_EOS R, K_EOS a~, b~/4 (CS) or b (vdW)
    C a_diff;              // a - K_EOS a~ with a = G^2 dx^2/2, so that p_BE = K R rho T Z + a_diff rho^2
    C inv_cs2;
    C beta;
    C g1C, g2C;            // (4 + gamma1) C_ref and (4 - gamma2) C_ref (SM Eq. (4a))
    C gamma1, gamma2;
    C s_e, s_eps, s_q, s_p;
    C ks;                  // k s_eps omega_e        (S(1,2))
    C hs;                  // h s_q omega_e          (S(1,4)/u_x, S(1,6)/u_y)
    C bs;                  // b s_q omega_p          (S(8,4)/u_y; S(7,4) = 2 bs u_x)
    C sig_e, sig_eps, sig_q, sig_p;
    C rho_v, inv_drho, tau_jv, dtau_j;  // tau_j(rho) interpolation
    C Qpre;                // G^2 dx^2 dt^2 / 12 (SM Eq. (6a))
    C Ep_pre;              // -(G^2 dx^2)/2 for the potential-energy diagnostic
    C ref_f[9], ref_g[9];  // deviation reference for 16-bit storage (zero otherwise)
};

enum Precision { kF64 = 0, kF32 = 1, kF16 = 2, kBF16 = 3 };

struct LaunchShape {
    int rows_per_wave;     // rows a wavefront marches through
    int waves_per_block;   // independent wavefronts per workgroup
    int columns_per_lane;  // 0 auto (two where the form allows), 1 or 2
};

// Default work items of the two-buffer kernel per storage precision (rows per wavefront,
// wavefronts per workgroup), measured on a 4096^2 lattice: FP32 3 x 4, FP64 4 x 2,
// 16-bit 16 x 4.  For FP32, three rows per item spend less per-item set-up per node than
// two, which matters most during the shader-clock dip of a run's first ~30 dispatches
// (3 % faster there than 2 x 2, 0.5 % at the steady clock), and unlike four rows they
// still find the rows they share with the items above and below in L2.
inline int default_rows(int prec) { return prec == kF32 ? 3 : (prec == kF64 ? 4 : 16); }
inline int default_waves(int prec) { return prec == kF64 ? 2 : 4; }

// All launchers enqueue on `stream` and return the hipError_t of the launch.
// `state` points at the 18 planes of nx*ny values (9 for f then 9 for g).
// layout of the state (see load_node): 0 AA even parity, 1 AA odd parity, 2 two-buffer pull
hipError_t launch_init(int prec, const void* c, void* state, const double* rho, const double* ux,
                       const double* uy, const double* T, int layout, hipStream_t stream);
// stochastic: 16-bit stores round stochastically (random bits from P.step and the node)
hipError_t launch_step_ab(int prec, const void* c, const void* in, void* out, LaunchShape shape, bool stochastic,
                          hipStream_t stream);
// In-place AA pattern: `parity` 0 = even step (own-node slots), 1 = odd step.
hipError_t launch_step_aa(int prec, const void* c, void* state, double* rho_scratch, int parity,
                          LaunchShape shape, hipStream_t stream);
hipError_t launch_density(int prec, const void* c, const void* state, int layout, double* rho,
                          hipStream_t stream);
hipError_t launch_moments(int prec, const void* c, const void* state, int layout, const double* rho,
                          double* ux, double* uy, double* T, hipStream_t stream);
// Writes 8 FP64 sums to `result` (device), using `partials` (>= kMaxPartialBlocks * 8 doubles).
hipError_t launch_invariants(int prec, const void* c, const void* state, int layout, const double* rho,
                             double* partials, double* result, hipStream_t stream);

constexpr int kMaxPartialBlocks = 1024;

// ---- batched form: many independent lattices advanced by one launch per step ----
// One descriptor per lattice, in device memory.  The work items of lattice b (strips of
// 64 columns times `rows` rows, strip-major within each row chunk) are numbered
// starts[b] .. starts[b+1]-1 in one global range.  A launch of parity p reads buf[p]
// and writes buf[p ^ 1].
template <typename C>
struct BatchDesc {
    Consts<C> P;
    const void* buf[2];
    int32_t nstrips;
    int32_t rows;
    int32_t cols;          // columns per lane of the two-buffer kernel (1 or 2)
    int32_t pad_;
};

// Work distribution of a batched launch.
struct BatchLaunch {
    int waves_per_block;
    int blocks;            // grid size
    int queue;             // 0: one wavefront per work item; 1: persistent grid on per-XCD tile queues
    int groups;            // queue mode: number of queues (min(8, blocks))
};

// `queue` holds 2 x 8 unsigned counters (zero before the first launch).  A queue-mode
// launch of parity p takes items from counters [p*8, p*8+8) and clears the other eight
// for the next launch.  `steps` holds 2 counters per lattice: a launch of parity p reads
// lattice b's step count from steps[2b + p] and writes it plus one to steps[2b + (p ^ 1)]
// (so graph replays advance the stochastic-rounding stream without host writes).
hipError_t launch_step_ab_batch(int prec, const void* desc, const int32_t* starts, unsigned* queue,
                                uint32_t* steps, int nlat, int nitems, int parity, BatchLaunch bl, bool stochastic,
                                hipStream_t stream);
// Resident blocks per CU of the batched kernel for the given precision and block size.
int batch_blocks_per_cu(int prec, int waves_per_block, int queue, bool stochastic);
size_t batch_desc_size(int prec);

// ---- lattices bounded in x (lbm_bounded.hip) ----
// Boundary state of the heated-outflow / wall pair: the heated side at x = 0 holds
// rho_wall (vapour at p_out and T_wall) and T_wall with the velocity of column 1; the far
// side at x = nx - 1 holds the density of column nx - 2, zero velocity and T_far.
template <typename C>
struct Walls {
    C rho_wall, T_wall, T_far;
};
// One workgroup steps the whole lattice, with each step's densities in LDS.
constexpr int kMaxBoundedNodes = 8192;
constexpr int kBoundedThreads = 1024;
// Advances `steps` steps of the two-buffer pull scheme: step k reads buf[(first + k) & 1]
// and writes the other buffer.
hipError_t launch_step_bounded(int prec, const void* c, const void* walls, void* buf0, void* buf1, int first,
                               int steps, hipStream_t stream);
// rho, u, T of the current state (rho may not be NULL; the others may); boundary columns
// report the imposed boundary state.
hipError_t launch_moments_bounded(int prec, const void* c, const void* walls, const void* state, double* rho,
                                  double* ux, double* uy, double* T, hipStream_t stream);
// The 8 FP64 diagnostics of launch_invariants over the fluid columns 1 .. nx - 2, in a
// fixed summation order.
hipError_t launch_invariants_bounded(int prec, const void* c, const void* walls, const void* state,
                                     double* result, hipStream_t stream);
size_t consts_size(int prec);
size_t storage_bytes(int prec);

}  // namespace lbm_dev
