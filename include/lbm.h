/*
 * lbm.h - C ABI of the MI355X (gfx950) lattice Boltzmann update for the
 * liquid-vapour phase transition of Huang, Wu & Adams (arXiv 2106.01557).
 *
 * One call of lbm_step() advances the double-distribution D2Q9 model by whole
 * time steps: streaming Eq. (12a), the moment-space collisions Eqs. (12b)-(12c)
 * with the matrices of SM Eqs. (2)-(6), the pairwise interaction force Eq. (13),
 * the moment sums Eq. (14), and the closure Eqs. (15)-(17) (built-in variable
 * eta from the dense-gas equation of state).  The lattice is periodic in x and y.
 *
 * Conventions shared by every call
 *  - Every function returns int: LBM_OK (0) or a negative LBM_E* code.  Nothing
 *    aborts or throws across the ABI.  lbm_last_error() holds a message.
 *  - Fields are row-major [ny][nx] (x fastest), one value per node, FP64.
 *  - Device pointers are HIP device addresses on the device that was current
 *    when lbm_init() ran.  The library never allocates device memory: the
 *    caller passes a workspace of at least lbm_workspace_bytes() bytes and keeps
 *    it alive until lbm_destroy().  Host memory for the context itself is owned
 *    by the library.
 *  - All device work is enqueued on the stream given to lbm_init() (NULL = the
 *    default stream) and is asynchronous unless marked "synchronising".  Device
 *    faults surface as LBM_EHIP at the next synchronising call.
 *  - Units are the paper's lattice units (dx = 1 by default, R = 1); the time
 *    step dt is derived from Eq. (19) and reported by lbm_derived().
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes --------------------------------------------------------- */
#define LBM_OK          0
#define LBM_EINVAL     (-1)  /* bad parameter, shape or pointer                          */
#define LBM_ESPACE     (-2)  /* workspace too small                                      */
#define LBM_EHIP       (-3)  /* HIP runtime error (launch failure, device fault, ...)     */
#define LBM_ENONFINITE (-4)  /* state check found NaN/Inf, rho <= 0, T <= 0 or a packing
                                fraction >= 1                                            */
#define LBM_ESTATE     (-5)  /* call out of order (e.g. lbm_step before lbm_set_fields,
                                or a device call on a host-only context)                 */
#define LBM_EIO        (-6)  /* checkpoint file cannot be opened, read or written, or its
                                header or checksum does not match                         */

/* ---- equation of state kinds (p_EOS of the text after Eq. (11)) --------- */
#define LBM_EOS_CS  0  /* Eq. (17): K[rho R T (1+t+t^2-t^3)/(1-t)^3 - a rho^2], t = b rho/4 */
#define LBM_EOS_VDW 1  /* K[rho R T / (1 - b rho) - a rho^2]                             */

/* ---- storage precision of the distributions (arithmetic is FP64 for F64 and
 *      FP32 otherwise) ------------------------------------------------------ */
#define LBM_F64  0
#define LBM_F32  1
#define LBM_F16  2  /* FP16 deviations from the rest equilibrium of (rho_ref, T_ref) */
#define LBM_BF16 3  /* BF16 deviations from the rest equilibrium of (rho_ref, T_ref) */

/* ---- rounding of the 16-bit storage formats --------------------------------- */
#define LBM_ROUND_NEAREST    0  /* round to nearest even (default)                          */
#define LBM_ROUND_STOCHASTIC 1  /* unbiased stochastic rounding; see lbm_params.rounding    */

/* ---- update schemes ------------------------------------------------------- */
#define LBM_SCHEME_AB 0  /* fused single pass, two state buffers (pull streaming)      */
#define LBM_SCHEME_AA 1  /* in-place AA pattern, one state buffer, plus a density pass */

/* ---- boundaries in x (y is always periodic) -------------------------------- */
#define LBM_BC_PERIODIC       0  /* periodic in x (the default)                          */
#define LBM_BC_HEATED_OUTFLOW 1  /* the one-dimensional Stefan problem (Eqs. (20)-(21)):
                                    x = 0 is a heated wall (T_r1 = lbm_params.Tr_wall) with
                                    vapour outflow at constant pressure (lbm_params.p_out),
                                    x = nx-1 a wall at rest (lbm_params.Tr_far); both by
                                    non-equilibrium extrapolation from the neighbouring
                                    fluid column (Guo, Zheng & Shi 2002, standing in for
                                    the improved scheme the paper cites).  Columns 0 and
                                    nx-1 are boundary nodes.  Needs the two-buffer scheme,
                                    LBM_F64 or LBM_F32, nx >= 4 and nx*ny <= 8192 (one
                                    workgroup steps the lattice); not a batch member.    */

typedef struct lbm_ctx lbm_ctx;   /* opaque; owned by the library */

/* Lattice: D2Q9 velocities of SM Eq. (1), periodic in y, and in x unless bc_x says
 * otherwise (a zero-initialised bc_x is periodic). */
typedef struct {
    int32_t nx, ny;   /* nodes, each >= 1 and nx*ny < 2^31                           */
    double  dx;       /* lattice spacing delta_x (> 0; the paper uses 1)              */
    int32_t bc_x;     /* LBM_BC_PERIODIC or LBM_BC_HEATED_OUTFLOW                     */
} lbm_lattice;

/* Equation of state, Eq. (17).  For LBM_EOS_CS, a_t and b_t are a~ and b~ (Tc, pc
 * follow from their definitions under Eq. (17)); for LBM_EOS_VDW they are a and b. */
typedef struct {
    int32_t kind;                    /* LBM_EOS_CS or LBM_EOS_VDW                   */
    double  a_t, b_t, R, K_eos;      /* all > 0                                      */
} lbm_eos;

/* Model parameters (text before Eq. (20), SM Eqs. (3)-(5)).  Fields marked
 * "reading" are not fixed by the paper; their defaults are set by
 * lbm_default_params(). */
typedef struct {
    double Tr0;           /* reference reduced temperature T0/Tc: sets rho_l in Eq. (19) and
                             the density range of the conductivity interpolation       */
    double K_int;         /* K_INT of Eqs. (18)-(19)                                    */
    double varpi;         /* model coefficient (SM Eq. (3), (5a)), 0 < varpi < 1/3      */
    double gamma1, gamma2;/* model coefficients (SM Eq. (4))                            */
    double tau_p;         /* tau_p = 1/s_p - 1/2 > 0; s_q, s_e follow from
                             tau_p tau_q = (k+1) tau_e tau_q = 1/12 (after SM Eq. (5b)) */
    double s_eps;         /* reading                                                    */
    double sigma_e, sigma_eps, sigma_q, sigma_p; /* L entries (SM Eq. (5b)); reading    */
    double tau_j_v;       /* vapour tau_j = 1/sigma_j - 1/2 (reading)                   */
    double lambda_ratio;  /* lambda_l / lambda_v; tau_j is linear in rho between the
                             coexistence densities at T0 and clamped outside (reading) */
    double cv;            /* specific heat; <= 0: derived from ste and dTr_ste          */
    double ste, dTr_ste;  /* Stefan number and T_r1 - T_r0 used to derive cv (reading) */
    double C_ref;         /* reference volumetric heat capacity; <= 0: rho_v * cv       */
    double accel_x, accel_y; /* external acceleration a of Eq. (14)                     */
    double cs_override;   /* > 0: use this lattice sound speed instead of Eq. (19)      */
    double rho_ref, T_ref;/* deviation reference for LBM_F16/LBM_BF16 storage;
                             <= 0: rho_v at T0 (vapour coexistence) and T0            */
    double Tr_wall;       /* LBM_BC_HEATED_OUTFLOW: T/Tc of the heated wall (T_r1; the
                             paper's 0.85); > 0                                       */
    double Tr_far;        /* LBM_BC_HEATED_OUTFLOW: T/Tc of the far wall; <= 0: Tr0     */
    double p_out;         /* LBM_BC_HEATED_OUTFLOW: outflow pressure; <= 0: the
                             saturation pressure at T0 (reading: the pressure of the
                             liquid at rest).  The boundary density is the vapour root
                             of p_EOS(rho, T_wall) = p_out                            */
    int32_t precision;    /* LBM_F64, LBM_F32, LBM_F16, LBM_BF16                        */
    int32_t scheme;       /* LBM_SCHEME_AB or LBM_SCHEME_AA                             */
    int32_t rows_per_wave;/* rows one wavefront marches through per launch; 0 = auto
                             (LBM_F32 2, LBM_F64 4, LBM_F16/LBM_BF16 16)               */
    int32_t waves_per_block; /* 1, 2, 4 or 8; 0 = auto (2; 4 for 16-bit storage)        */
    int32_t columns_per_lane;/* two-buffer kernel: columns per lane, 1 or 2; 0 = auto
                                (2 for 4- and 2-byte storage with an even nx, else 1);
                                2 is taken only where allowed                           */
    int32_t rounding;     /* LBM_F16/LBM_BF16 stores of the two-buffer update:
                             LBM_ROUND_NEAREST or LBM_ROUND_STOCHASTIC.  Rounding to
                             nearest is deterministic per value, so in a nearly steady
                             state the same values round the same way every step and the
                             errors accumulate into a bias (coexistence densities move by
                             percents); stochastic rounding rounds up with probability equal
                             to the discarded fraction, which removes that bias.  Its random
                             bits are a hash of the step count and the node, so runs stay
                             deterministic, and restarts (lbm_load_state) and batched
                             members stay bitwise equal to uninterrupted single runs.
                             LBM_EINVAL for other precisions or the AA scheme.
                             lbm_set_fields rounds to nearest.                       */
    int32_t check_every;  /* failure detection: > 0 makes lbm_step run the state check of
                             lbm_invariants (NaN/Inf, rho <= 0, T <= 0, packing fraction
                             >= 1) after every step whose count is a multiple of
                             check_every; that check synchronises the stream.  On a
                             failure lbm_step stops there and returns LBM_ENONFINITE, and
                             lbm_last_error() names the step count and the number of
                             failing nodes.  0 (default): no checks inside lbm_step.     */
} lbm_params;

/* Fills *p with the paper's numerical-test parameters (varpi = 1/6, gamma1 = -2,
 * gamma2 = 2, T_r0 = 0.8, K_INT = 2.294922, lambda_l = 10 lambda_v) and the
 * readings listed above; precision LBM_F64, scheme LBM_SCHEME_AB.  Never fails
 * for a non-NULL p. */
int lbm_default_params(lbm_params* p);

/* Fills *e with the paper's Carnahan-Starling set (a~ = 1, b~ = 4, R = 1,
 * K_EOS = 0.479820), text before Eq. (20). */
int lbm_default_eos(lbm_eos* e);

/* Device workspace needed for this lattice and these parameters (state buffers,
 * a density scratch array and reduction partials).  LBM_EINVAL on bad input. */
int lbm_workspace_bytes(const lbm_lattice* lat, const lbm_params* p, size_t* bytes);

/* Validates everything (LBM_EINVAL with a message on any bad value, before any
 * HIP call), derives the per-run constants (Maxwell coexistence at T0, c_s of
 * Eq. (19), dt = dx/c with c = sqrt(3) c_s, G^2 of Eq. (18), a and kappa of
 * Eq. (16), relaxation rates, cv, C_ref) and binds the caller's workspace and
 * stream.  workspace == NULL creates a host-only context whose constants can be
 * queried with lbm_derived() but which refuses device calls (LBM_ESTATE).
 * Otherwise workspace must be device memory of at least lbm_workspace_bytes()
 * bytes, 256-byte aligned (LBM_ESPACE / LBM_EINVAL).  On success *out owns a new
 * context; on failure *out is NULL and the message is available through
 * lbm_last_error(NULL). */
int lbm_init(lbm_ctx** out, const lbm_lattice* lat, const lbm_eos* eos,
             const lbm_params* p, void* workspace, size_t workspace_bytes,
             void* hip_stream);

/* Sets the state from macroscopic fields (device FP64 arrays [ny][nx]; u is
 * the velocity in lattice units, T the temperature): f = M^-1 m^eq and
 * g = M^-1 n^eq of SM Eqs. (3a), (4a) with rho e_k = rho (cv T + |u|^2/2),
 * eta and rho h_k from the closure Eq. (15) (reading: no force shift at t = 0).
 * Resets the step counter to 0.  Asynchronous. */
int lbm_set_fields(lbm_ctx* ctx, const double* rho, const double* ux,
                   const double* uy, const double* T);

/* Advances n >= 0 time steps.  Asynchronous; launches only (no host sync), except for
 * the state checks that lbm_params.check_every > 0 asks for (see there). */
int lbm_step(lbm_ctx* ctx, int64_t n);

/* Writes rho, u and T at the current time (Eq. (14); u includes the dt/2 F
 * correction, T from rho e_k = rho cv T + rho |u|^2/2) into caller-owned device
 * FP64 arrays [ny][nx].  Any of ux, uy, T may be NULL; rho may not (it also
 * serves as scratch for the force stencil).  Asynchronous. */
int lbm_moments(lbm_ctx* ctx, double* rho, double* ux, double* uy, double* T);

/* Global diagnostics in FP64, reduced on the device in a fixed order
 * (deterministic), then copied to host (synchronising):
 *   out[0] mass            sum_x sum_i f_i                    (exact invariant)
 *   out[1] momentum x      sum_x sum_i e_ix f_i               (invariant if a = 0)
 *   out[2] momentum y
 *   out[3] sum_g           sum_x sum_i g_i; obeys sum_g(t+dt) = sum_g(t) + out[4]
 *   out[4] dt sum_x q      (row 0 of Eq. (12c))
 *   out[5] E_p             -(G^2 dx^2/2) sum_x [rho^2/6 + rho/2 sum_i w_i rho(x+e_i dx)]
 *   out[6] sum_x rho e_k
 *   out[7] number of nodes failing the state check (NaN/Inf, rho <= 0, T <= 0,
 *          packing fraction >= 1); when > 0 the call returns LBM_ENONFINITE.
 * n_out must be >= 8. */
int lbm_invariants(lbm_ctx* ctx, double* out, int n_out);

/* Per-run constants, in this order (n <= 27 values are written):
 *  0 Tc   1 pc   2 T0   3 rho_v  4 rho_l  5 p_s   6 c_s  7 c   8 dt   9 G^2
 * 10 a   11 kappa 12 cv 13 C_ref 14 beta 15 k  16 h  17 b (SM Eq. (5a))
 * 18 s_p 19 s_q 20 s_e 21 omega_e 22 omega_p 23 tau_j_v 24 tau_j_l 25 h_lv
 * 26 rho_wall (LBM_BC_HEATED_OUTFLOW: the boundary density of the heated side; else 0) */
int lbm_derived(const lbm_ctx* ctx, double* out, int n);

/* Effective launch shape of the fused two-buffer kernel (after resolving the
 * 0 = auto values of lbm_params): rows each wavefront marches through,
 * wavefronts per workgroup and columns per lane (columns_per_lane may be NULL).
 * Host-only; never fails for a valid context. */
int lbm_launch_shape(const lbm_ctx* ctx, int32_t* rows_per_wave, int32_t* waves_per_block,
                     int32_t* columns_per_lane);

/* Number of completed steps since lbm_set_fields(). */
int lbm_step_count(const lbm_ctx* ctx, int64_t* steps);

/* Raw state copy for checkpoint/restart: the distributions in storage
 * precision, in the layout of the current step (scheme and parity included),
 * to/from caller device memory of lbm_state_bytes() bytes.  Restoring a saved
 * state and stepping is bitwise identical to never having stopped. */
int lbm_state_bytes(const lbm_ctx* ctx, size_t* bytes);
int lbm_save_state(lbm_ctx* ctx, void* dst_device, int64_t* steps);
int lbm_load_state(lbm_ctx* ctx, const void* src_device, int64_t steps);

/* Checkpoint to a file and restart from one (synchronising).  The file holds a
 * 256-byte header (magic "LBMSTATE", format version, lattice, EOS, every model
 * parameter that enters the update, storage precision, scheme, rounding, the step count
 * and an FNV-1a 64-bit checksum of the payload) followed by the raw state of
 * lbm_save_state (little-endian, storage precision, state_bytes of lbm_state_bytes()).
 * The state is staged through host memory the library allocates for the call.
 * lbm_load() accepts only a file written for the same lattice, EOS, parameters,
 * precision, scheme and rounding (launch-shape fields may differ) and restores the step
 * count with the state, so that stepping on is bitwise identical to never having
 * stopped.  LBM_EIO when the file cannot be opened, read or written, is truncated, or
 * its magic, version or checksum is wrong; LBM_EINVAL when it was written for a
 * different configuration (the message names the first field that differs); the
 * context is unchanged on any failure of lbm_load(). */
int lbm_save(lbm_ctx* ctx, const char* path);
int lbm_load(lbm_ctx* ctx, const char* path);

/* Releases the context (never the caller's workspace).  NULL is allowed. */
int lbm_destroy(lbm_ctx* ctx);

/* Coexisting densities of the equation of state alone (Maxwell equal-area
 * construction on p_EOS of Eq. (17); the pressure at coexistence is p_s) at the
 * reduced temperature Tr = T/Tc, 0 < Tr < 1.  Host-only: out[0] rho_v,
 * out[1] rho_l, out[2] p_s, out[3] Tc.  LBM_EINVAL on bad input or when no
 * coexistence is found. */
int lbm_maxwell(const lbm_eos* eos, double Tr, double out[4]);

/* The paper's procedure for the two scaling constants (text before Eq. (20)): a
 * prescribed surface tension sigma and 5 %-95 % interface width W of the flat interface
 * at T = Tr Tc fix K_EOS and K_INT.  With kappa = G^2 dx^4 / 4 and G of Eq. (18), the
 * square-gradient tension int sqrt(2 kappa dOmega) drho scales as K_INT K_EOS and the
 * width int sqrt(kappa / (2 dOmega)) drho as K_INT, so both follow from the integrals at
 * K_EOS = K_INT = 1 (dOmega: grand-potential excess over the Maxwell tie line of p_EOS).
 * eos->K_eos is ignored.  Host-only: out[0] K_EOS, out[1] K_INT.  LBM_EINVAL on bad input
 * or when there is no coexistence at Tr.  (sigma = 0.01, W = 10 at Tr = 0.8 give the
 * paper's 0.479820 and 2.294922.) */
int lbm_interface_constants(const lbm_eos* eos, double Tr, double sigma, double W, double dx, double out[2]);

/* ---- batched form -----------------------------------------------------------
 * Many independent lattices (each its own size, EOS, temperature and constants,
 * created by lbm_init with the two-buffer scheme) advanced together by one kernel
 * launch per time step.  Each step of a member is bitwise identical to what
 * lbm_step on that member alone computes.  The members stay usable through the
 * single-lattice calls (moments, invariants, save/load, even lbm_step); the
 * batch notices a member stepped alone and re-reads its buffers.  Members must
 * outlive the batch and share one precision, one rounding mode and one stream, and each must keep
 * (18 ny + 17) nx bytes-per-value below 4 GiB (32-bit buffer offsets). */
typedef struct lbm_batch lbm_batch;  /* opaque; owned by the library */

/* Work distribution of a batched launch. */
typedef struct {
    int32_t rows_per_wave;   /* rows of one work item (>= 1)                          */
    int32_t waves_per_block; /* 1, 2 or 4                                              */
    int32_t queue;           /* 0: one wavefront per work item (grid sized to the work);
                                1: persistent grid of resident wavefronts taking work
                                items from per-XCD atomic tile queues                   */
    int32_t blocks;          /* queue mode: grid size; 0 = CUs x resident blocks per CU */
} lbm_batch_shape;

/* Device workspace of a batch of n members in this precision (descriptor table,
 * item offsets, queue counters, per-member step counters). */
int lbm_batch_workspace_bytes(int32_t n, int32_t precision, size_t* bytes);

/* Groups n >= 1 distinct device contexts.  workspace: device memory of at least
 * lbm_batch_workspace_bytes() bytes, 256-byte aligned.  Synchronises the stream
 * once (descriptor upload).  Default shape: grid mode with the single-lattice
 * default rows and waves of the precision (lbm_params.rows_per_wave).  On failure
 * *out is NULL and lbm_batch_last_error(NULL) explains. */
int lbm_batch_create(lbm_batch** out, lbm_ctx* const* members, int32_t n, void* workspace,
                     size_t workspace_bytes);

/* Sets / reads the launch shape (LBM_EINVAL for values outside the ranges above). */
int lbm_batch_set_shape(lbm_batch* b, const lbm_batch_shape* shape);
int lbm_batch_get_shape(const lbm_batch* b, lbm_batch_shape* shape);

/* Replays captured HIP graphs of steps_per_graph launches (even, >= 2) for the
 * bulk of lbm_batch_step; 0 launches every step directly.  The graph is captured
 * on the members' stream at the next step call and again after a shape change.
 * The stream must be a created stream (LBM_EINVAL for the null stream). */
int lbm_batch_set_graph(lbm_batch* b, int32_t steps_per_graph);

/* Advances every member n >= 0 time steps.  Asynchronous (a descriptor re-upload,
 * needed only after a member was stepped or reset alone, synchronises). */
int lbm_batch_step(lbm_batch* b, int64_t n);

/* Times every candidate shape (rows 2/4/8/16/32/64/128 x 1/2/4 waves per block x
 * grid and queue mode) over steps_per_candidate >= 1 steps after 2 warm-up steps,
 * and keeps the fastest.  The timed steps are real steps: every member advances
 * 42 x (steps_per_candidate + 2) steps, bitwise as it would under any fixed
 * shape.  Writes the chosen shape and its milliseconds per step (either pointer
 * may be NULL).  Synchronising. */
int lbm_batch_autotune(lbm_batch* b, int32_t steps_per_candidate, lbm_batch_shape* best,
                       double* ms_per_step);

/* Work items of one launch under the current shape, and total nodes. */
int lbm_batch_size(const lbm_batch* b, int64_t* items, int64_t* nodes);

/* Releases the batch (never the members or the workspace).  NULL is allowed. */
int lbm_batch_destroy(lbm_batch* b);

/* Message of the last failing call on b (or of the last failed create when b is
 * NULL). */
const char* lbm_batch_last_error(const lbm_batch* b);


/* Static description of a code; never NULL. */
const char* lbm_strerror(int code);

/* Message of the last failing call on ctx (or of the last failed lbm_init when
 * ctx is NULL); empty string when there is none.  Valid until the next call. */
const char* lbm_last_error(const lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
