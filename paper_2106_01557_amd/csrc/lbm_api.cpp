// C ABI of the liquid-vapour lattice Boltzmann library (declared in include/lbm.h).
#include "../../include/lbm.h"

#include <hip/hip_runtime.h>

#include <cerrno>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbm_ctx.hpp"
#include "thermo.hpp"

using lbm_dev::Consts;


namespace {

thread_local std::string g_init_error;

int fail(lbm_ctx* ctx, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_init_error = buf;
    return code;
}

int hip_fail(lbm_ctx* ctx, hipError_t e, const char* what) {
    return fail(ctx, LBM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

int check_lattice(const lbm_lattice* lat) {
    if (!lat) return fail(nullptr, LBM_EINVAL, "lattice is NULL");
    if (lat->nx < 1 || lat->ny < 1)
        return fail(nullptr, LBM_EINVAL, "nx and ny must be >= 1 (got %d x %d)", lat->nx, lat->ny);
    if ((int64_t)lat->nx * lat->ny > 0x7fffffffLL)
        return fail(nullptr, LBM_EINVAL, "nx * ny must be < 2^31 (got %lld)", (long long)lat->nx * lat->ny);
    if (!finite_pos(lat->dx)) return fail(nullptr, LBM_EINVAL, "dx must be finite and > 0");
    if (lat->bc_x != LBM_BC_PERIODIC && lat->bc_x != LBM_BC_HEATED_OUTFLOW)
        return fail(nullptr, LBM_EINVAL, "unknown bc_x %d", lat->bc_x);
    if (lat->bc_x == LBM_BC_HEATED_OUTFLOW &&
        (lat->nx < 4 || (int64_t)lat->nx * lat->ny > lbm_dev::kMaxBoundedNodes))
        return fail(nullptr, LBM_EINVAL, "bc_x = LBM_BC_HEATED_OUTFLOW needs nx >= 4 and nx * ny <= %d (got %d x %d)",
                    lbm_dev::kMaxBoundedNodes, lat->nx, lat->ny);
    return LBM_OK;
}

int check_params(const lbm_params* p) {
    if (!p) return fail(nullptr, LBM_EINVAL, "params is NULL");
    if (!(p->Tr0 > 0 && p->Tr0 < 1)) return fail(nullptr, LBM_EINVAL, "Tr0 must lie in (0, 1) (got %g)", p->Tr0);
    if (!finite_pos(p->K_int)) return fail(nullptr, LBM_EINVAL, "K_int must be > 0");
    if (!(p->varpi > 0 && p->varpi < 1.0 / 3.0))
        return fail(nullptr, LBM_EINVAL, "varpi must lie in (0, 1/3) (got %g)", p->varpi);
    if (!std::isfinite(p->gamma1) || !std::isfinite(p->gamma2))
        return fail(nullptr, LBM_EINVAL, "gamma1 and gamma2 must be finite");
    if (!finite_pos(p->tau_p)) return fail(nullptr, LBM_EINVAL, "tau_p must be > 0 (got %g)", p->tau_p);
    const double rates[5] = {p->s_eps, p->sigma_e, p->sigma_eps, p->sigma_q, p->sigma_p};
    const char* names[5] = {"s_eps", "sigma_e", "sigma_eps", "sigma_q", "sigma_p"};
    for (int i = 0; i < 5; ++i)
        if (!(rates[i] > 0 && rates[i] < 2))
            return fail(nullptr, LBM_EINVAL, "%s must lie in (0, 2) (got %g)", names[i], rates[i]);
    if (!finite_pos(p->tau_j_v)) return fail(nullptr, LBM_EINVAL, "tau_j_v must be > 0");
    if (!finite_pos(p->lambda_ratio)) return fail(nullptr, LBM_EINVAL, "lambda_ratio must be > 0");
    if (!std::isfinite(p->cv) || !std::isfinite(p->C_ref))
        return fail(nullptr, LBM_EINVAL, "cv and C_ref must be finite");
    if (p->cv <= 0 && !(finite_pos(p->ste) && finite_pos(p->dTr_ste)))
        return fail(nullptr, LBM_EINVAL, "cv <= 0 needs ste > 0 and dTr_ste > 0 to derive it");
    if (!std::isfinite(p->accel_x) || !std::isfinite(p->accel_y))
        return fail(nullptr, LBM_EINVAL, "acceleration must be finite");
    if (!std::isfinite(p->cs_override) || p->cs_override < 0)
        return fail(nullptr, LBM_EINVAL, "cs_override must be >= 0");
    if (!std::isfinite(p->rho_ref) || !std::isfinite(p->T_ref))
        return fail(nullptr, LBM_EINVAL, "rho_ref and T_ref must be finite");
    if (p->precision < LBM_F64 || p->precision > LBM_BF16)
        return fail(nullptr, LBM_EINVAL, "unknown precision %d", p->precision);
    if (p->scheme != LBM_SCHEME_AB && p->scheme != LBM_SCHEME_AA)
        return fail(nullptr, LBM_EINVAL, "unknown scheme %d", p->scheme);
    if (p->rows_per_wave < 0 || p->rows_per_wave > 65536)
        return fail(nullptr, LBM_EINVAL, "rows_per_wave must lie in [0, 65536]");
    const int w = p->waves_per_block;
    if (!(w == 0 || w == 1 || w == 2 || w == 4 || w == 8))
        return fail(nullptr, LBM_EINVAL, "waves_per_block must be 0, 1, 2, 4 or 8 (got %d)", w);
    if (p->columns_per_lane < 0 || p->columns_per_lane > 2)
        return fail(nullptr, LBM_EINVAL, "columns_per_lane must be 0, 1 or 2 (got %d)", p->columns_per_lane);
    if (p->rounding != LBM_ROUND_NEAREST && p->rounding != LBM_ROUND_STOCHASTIC)
        return fail(nullptr, LBM_EINVAL, "unknown rounding %d", p->rounding);
    if (p->check_every < 0) return fail(nullptr, LBM_EINVAL, "check_every must be >= 0 (got %d)", p->check_every);
    if (!std::isfinite(p->Tr_wall) || !std::isfinite(p->Tr_far) || !std::isfinite(p->p_out))
        return fail(nullptr, LBM_EINVAL, "Tr_wall, Tr_far and p_out must be finite");
    if (p->rounding == LBM_ROUND_STOCHASTIC &&
        ((p->precision != LBM_F16 && p->precision != LBM_BF16) || p->scheme != LBM_SCHEME_AB))
        return fail(nullptr, LBM_EINVAL, "stochastic rounding needs LBM_F16 or LBM_BF16 storage and LBM_SCHEME_AB");
    return LBM_OK;
}

int check_eos(const lbm_eos* e) {
    if (!e) return fail(nullptr, LBM_EINVAL, "eos is NULL");
    if (e->kind != LBM_EOS_CS && e->kind != LBM_EOS_VDW)
        return fail(nullptr, LBM_EINVAL, "unknown EOS kind %d", e->kind);
    if (!finite_pos(e->a_t) || !finite_pos(e->b_t) || !finite_pos(e->R) || !finite_pos(e->K_eos))
        return fail(nullptr, LBM_EINVAL, "EOS a_t, b_t, R and K_eos must be finite and > 0");
    return LBM_OK;
}

size_t state_buffer_bytes(const lbm_lattice* lat, const lbm_params* p) {
    return round256((size_t)18 * lat->nx * lat->ny * lbm_dev::storage_bytes(p->precision));
}

// Rest equilibria M^-1 m^eq and M^-1 n^eq (SM Eqs. (3a), (4a) with u = 0): the
// 16-bit storage formats keep deviations from these.
void rest_populations(const lbm_ctx* c, double rho, double T, double* f, double* g) {
    static const int M1[9] = {-4, -1, -1, -1, -1, 2, 2, 2, 2};
    static const int M2[9] = {4, -2, -2, -2, -2, 1, 1, 1, 1};
    const double cs2 = c->derived[6] * c->derived[6];
    lbm_host::Eos e{c->eos.kind, c->eos.a_t, c->eos.b_t, c->eos.R, c->eos.K_eos};
    const double pbe = (double)lbm_host::pressure(e, rho, T) + c->derived[10] * rho * rho;
    const double eta = pbe / cs2 - rho, beta = c->derived[14];
    const double m1 = -2 * rho + 2 * eta, m2 = rho + beta * eta;
    const double rek = rho * c->derived[12] * T, cref = c->derived[13];
    const double n1 = -4 * rek + (4 + c->p.gamma1) * cref * T, n2 = 4 * rek - (4 - c->p.gamma2) * cref * T;
    for (int i = 0; i < 9; ++i) {
        f[i] = rho / 9 + M1[i] * m1 / 36 + M2[i] * m2 / 36;
        g[i] = rek / 9 + M1[i] * n1 / 36 + M2[i] * n2 / 36;
    }
}

template <typename C>
void fill_consts(const lbm_ctx* c, Consts<C>* k) {
    const double* d = c->derived;
    const double dx = c->lat.dx;
    std::memset(k, 0, sizeof *k);
    k->nx = c->lat.nx;
    k->ny = c->lat.ny;
    k->eos_kind = c->eos.kind;
    const double G2 = d[9], cs = d[6], cc = d[7], dt = d[8];
    k->G2dx = (C)(G2 * dx);
    k->inv_dx = (C)(1.0 / dx);
    k->ax = (C)c->p.accel_x;
    k->ay = (C)c->p.accel_y;
    k->c = (C)cc;
    k->inv_c = (C)(1.0 / cc);
    k->c2 = (C)(cc * cc);
    k->dt = (C)dt;
    k->hdt = (C)(0.5 * dt);
    k->hdt_c = (C)(0.5 * dt / cc);
    k->cv = (C)d[12];
    k->inv_cv = (C)(1.0 / d[12]);
    k->C_ref = (C)d[13];
    k->KR = (C)(c->eos.K_eos * c->eos.R);
    k->Ka = (C)(c->eos.K_eos * c->eos.a_t);
    k->bq = (C)(c->eos.kind == LBM_EOS_CS ? 0.25 * c->eos.b_t : c->eos.b_t);
    k->a_diff = (C)(d[10] - c->eos.K_eos * c->eos.a_t);
    k->inv_cs2 = (C)(1.0 / (cs * cs));
    k->beta = (C)d[14];
    k->g1C = (C)((4 + c->p.gamma1) * d[13]);
    k->g2C = (C)((4 - c->p.gamma2) * d[13]);
    k->gamma1 = (C)c->p.gamma1;
    k->gamma2 = (C)c->p.gamma2;
    const double s_p = d[18], s_q = d[19], s_e = d[20], om_e = d[21], om_p = d[22];
    k->s_e = (C)s_e;
    k->s_eps = (C)c->p.s_eps;
    k->s_q = (C)s_q;
    k->s_p = (C)s_p;
    k->ks = (C)(d[15] * c->p.s_eps * om_e);
    k->hs = (C)(d[16] * s_q * om_e);
    k->bs = (C)(d[17] * s_q * om_p);
    k->sig_e = (C)c->p.sigma_e;
    k->sig_eps = (C)c->p.sigma_eps;
    k->sig_q = (C)c->p.sigma_q;
    k->sig_p = (C)c->p.sigma_p;
    k->rho_v = (C)d[3];
    k->inv_drho = (C)(1.0 / (d[4] - d[3]));
    k->tau_jv = (C)d[23];
    k->dtau_j = (C)(d[24] - d[23]);
    k->Qpre = (C)(G2 * dx * dx * dt * dt / 12.0);
    k->Ep_pre = (C)(-0.5 * G2 * dx * dx);
    if (c->p.precision == LBM_F16 || c->p.precision == LBM_BF16) {
        // default: the vapour coexistence state at T0.  Vapour populations are the small
        // ones, and T = rho e_k / (rho cv) divides by the small vapour density, so the fine
        // absolute resolution of small deviations belongs there
        const double rho_ref = c->p.rho_ref > 0 ? c->p.rho_ref : d[3];
        const double T_ref = c->p.T_ref > 0 ? c->p.T_ref : d[2];
        double f[9], g[9];
        rest_populations(c, rho_ref, T_ref, f, g);
        // at rest the populations depend only on the speed class (rest, axis, diagonal);
        // the references are made exactly class-uniform, so kernels may read the class
        // entry (0, 1 or 5) for every direction of the class
        for (int i = 0; i < 9; ++i) {
            const int cls = i == 0 ? 0 : (i < 5 ? 1 : 5);
            k->ref_f[i] = (C)f[cls];
            k->ref_g[i] = (C)g[cls];
        }
    }
}

int derive(lbm_ctx* c) {
    lbm_host::Eos e{c->eos.kind, c->eos.a_t, c->eos.b_t, c->eos.R, c->eos.K_eos};
    long double Tc, pc;
    lbm_host::critical(e, &Tc, &pc);
    const long double T0 = (long double)c->p.Tr0 * Tc;
    long double rv, rl, ps;
    std::string why;
    if (!lbm_host::coexistence(e, T0, &rv, &rl, &ps, &why))
        return fail(nullptr, LBM_EINVAL, "coexistence at Tr0 = %g: %s", c->p.Tr0, why.c_str());
    const long double dx = c->lat.dx;
    const long double Kint = c->p.K_int;
    const long double G2 = Kint * Kint * 2.0L * e.K * e.a / (dx * dx);           // Eq. (18)
    long double cs;
    if (c->p.cs_override > 0) {
        cs = c->p.cs_override;
    } else {
        const long double arg = lbm_host::pressure_slope(e, rl, T0) + 2.0L * e.K * e.a * rl;  // Eq. (19)
        if (!(arg > 0)) return fail(nullptr, LBM_EINVAL, "Eq. (19) gives a non-positive c_s^2");
        cs = Kint * std::sqrt(arg);
    }
    const long double cc = std::sqrt(3.0L) * cs, dt = dx / cc;
    const long double a_mf = G2 * dx * dx / 2, kappa = G2 * dx * dx * dx * dx / 4;  // Eq. (16)
    const long double h_lv = a_mf * (rl - rv) + ps * (1.0L / rv - 1.0L / rl);
    long double cv = c->p.cv;
    if (!(cv > 0)) cv = (long double)c->p.ste * rl * h_lv / (rv * Tc * (long double)c->p.dTr_ste);
    const long double Cref = c->p.C_ref > 0 ? (long double)c->p.C_ref : rv * cv;
    const long double w = c->p.varpi;
    const long double beta = -2.0L / (1 - w), k = 1 - w;
    const long double h = 6 * w * (1 - w) / (1 - 3 * w), bS = (1 - w) / (1 - 3 * w);
    const long double tau_p = c->p.tau_p;
    const long double tau_q = 1.0L / (12.0L * tau_p);          // tau_p tau_q = 1/12
    const long double tau_e = 1.0L / (12.0L * (k + 1) * tau_q); // (k+1) tau_e tau_q = 1/12
    const long double s_p = 1 / (tau_p + 0.5L), s_q = 1 / (tau_q + 0.5L), s_e = 1 / (tau_e + 0.5L);
    // heated-outflow walls: the boundary density is vapour at p_out and T_wall
    long double rho_wall = 0;
    if (c->lat.bc_x == LBM_BC_HEATED_OUTFLOW) {
        const long double T_wall = (long double)c->p.Tr_wall * Tc;
        const long double p_out = c->p.p_out > 0 ? (long double)c->p.p_out : ps;
        if (!lbm_host::vapour_root(e, T_wall, p_out, &rho_wall, &why))
            return fail(nullptr, LBM_EINVAL, "heated wall at Tr_wall = %g, p_out = %Lg: %s", c->p.Tr_wall, p_out,
                        why.c_str());
        const long double T_far = c->p.Tr_far > 0 ? (long double)c->p.Tr_far * Tc : T0;
        c->w64 = lbm_dev::Walls<double>{(double)rho_wall, (double)T_wall, (double)T_far};
        c->w32 = lbm_dev::Walls<float>{(float)rho_wall, (float)T_wall, (float)T_far};
    }
    const long double vals[27] = {Tc, pc, T0, rv, rl, ps, cs, cc, dt, G2, a_mf, kappa, cv, Cref,
                                  beta, k, h, bS, s_p, s_q, s_e, s_e / 2 - 1, s_p / 2 - 1,
                                  c->p.tau_j_v, c->p.tau_j_v * c->p.lambda_ratio, h_lv, rho_wall};
    for (int i = 0; i < 27; ++i) {
        c->derived[i] = (double)vals[i];
        if (!std::isfinite(c->derived[i])) return fail(nullptr, LBM_EINVAL, "derived constant %d is not finite", i);
    }
    return LBM_OK;
}

int need_device(lbm_ctx* c) {
    if (!c) return fail(nullptr, LBM_EINVAL, "context is NULL");
    if (c->host_only) return fail(c, LBM_ESTATE, "host-only context (created without a workspace)");
    return LBM_OK;
}

int need_fields(lbm_ctx* c) {
    int r = need_device(c);
    if (r) return r;
    if (!c->fields_set) return fail(c, LBM_ESTATE, "lbm_set_fields has not been called");
    return LBM_OK;
}

// Layout of the current state for the diagnostic kernels: the two-buffer scheme keeps
// post-collision populations at their source node (pull convention, 2); the AA
// scheme alternates between own-node (0) and shifted, swapped slots (1).
int aa_parity(const lbm_ctx* c) { return c->p.scheme == LBM_SCHEME_AA ? (int)(c->steps & 1) : 2; }

const void* current_state(const lbm_ctx* c) { return c->buf[c->p.scheme == LBM_SCHEME_AA ? 0 : c->cur]; }

// Density pass, the FP64 reductions of lbm_invariants and the state check, then a stream
// synchronisation; LBM_ENONFINITE (with the step count in the message) when any node fails.
int state_check(lbm_ctx* c, double* out) {
    hipError_t e;
    if (c->lat.bc_x == LBM_BC_HEATED_OUTFLOW) {
        e = lbm_dev::launch_invariants_bounded(c->p.precision, c->consts, c->walls, current_state(c), c->result,
                                               c->stream);
    } else {
        e = lbm_dev::launch_density(c->p.precision, c->consts, current_state(c), aa_parity(c), c->rho_scratch,
                                    c->stream);
        if (e == hipSuccess)
            e = lbm_dev::launch_invariants(c->p.precision, c->consts, current_state(c), aa_parity(c),
                                           c->rho_scratch, c->partials, c->result, c->stream);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(out, c->result, 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "state check");
    if (out[7] > 0)
        return fail(c, LBM_ENONFINITE, "state check failed at %.0f nodes after %lld steps", out[7],
                    (long long)c->steps);
    return LBM_OK;
}


// ---- checkpoint files -------------------------------------------------------------
// A 512-byte header, then the raw state of lbm_save_state.  Host byte order, which is
// little-endian on every host this library builds for.
constexpr char kFileMagic[8] = {'L', 'B', 'M', 'S', 'T', 'A', 'T', 'E'};
constexpr uint32_t kFileVersion = 1;
constexpr int kModelDoubles = 25;
const char* const kModelNames[kModelDoubles] = {
    "Tr0", "K_int", "varpi", "gamma1", "gamma2", "tau_p", "s_eps", "sigma_e", "sigma_eps", "sigma_q", "sigma_p",
    "tau_j_v", "lambda_ratio", "cv", "ste", "dTr_ste", "C_ref", "accel_x", "accel_y", "cs_override", "rho_ref",
    "T_ref", "Tr_wall", "Tr_far", "p_out"};

struct FileHeader {
    char magic[8];
    uint32_t version, header_bytes;
    int32_t nx, ny, precision, scheme, rounding, eos_kind, bc_x, pad_;
    int64_t steps;
    uint64_t state_bytes, checksum;
    double dx;
    double eos[4];               // a_t, b_t, R, K_eos
    double model[kModelDoubles];  // the double fields of lbm_params, in declaration order
    unsigned char reserved[512 - 8 - 8 - 32 - 8 - 16 - 8 - 32 - 8 * kModelDoubles];
};
static_assert(sizeof(FileHeader) == 512, "checkpoint header is 512 bytes");

void model_doubles(const lbm_params& p, double* m) {
    const double v[kModelDoubles] = {p.Tr0, p.K_int, p.varpi, p.gamma1, p.gamma2, p.tau_p, p.s_eps, p.sigma_e,
                                     p.sigma_eps, p.sigma_q, p.sigma_p, p.tau_j_v, p.lambda_ratio, p.cv, p.ste,
                                     p.dTr_ste, p.C_ref, p.accel_x, p.accel_y, p.cs_override, p.rho_ref, p.T_ref,
                                     p.Tr_wall, p.Tr_far, p.p_out};
    std::memcpy(m, v, sizeof v);
}

void fill_header(const lbm_ctx* c, FileHeader* h) {
    std::memset(h, 0, sizeof *h);
    std::memcpy(h->magic, kFileMagic, sizeof kFileMagic);
    h->version = kFileVersion;
    h->header_bytes = sizeof(FileHeader);
    h->nx = c->lat.nx;
    h->ny = c->lat.ny;
    h->precision = c->p.precision;
    h->scheme = c->p.scheme;
    h->rounding = c->p.rounding;
    h->eos_kind = c->eos.kind;
    h->bc_x = c->lat.bc_x;
    h->steps = c->steps;
    h->state_bytes = c->state_bytes;
    h->dx = c->lat.dx;
    h->eos[0] = c->eos.a_t;
    h->eos[1] = c->eos.b_t;
    h->eos[2] = c->eos.R;
    h->eos[3] = c->eos.K_eos;
    model_doubles(c->p, h->model);
}

// FNV-1a, 64-bit
uint64_t fnv1a(const unsigned char* p, size_t n) {
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

// First field in which the file's configuration differs from the context's, or nullptr.
const char* header_mismatch(const FileHeader& f, const FileHeader& want) {
    if (f.nx != want.nx || f.ny != want.ny) return "lattice size";
    if (f.bc_x != want.bc_x) return "boundary kind";
    if (std::memcmp(&f.dx, &want.dx, sizeof f.dx)) return "dx";
    if (f.precision != want.precision) return "precision";
    if (f.scheme != want.scheme) return "scheme";
    if (f.rounding != want.rounding) return "rounding";
    if (f.eos_kind != want.eos_kind || std::memcmp(f.eos, want.eos, sizeof f.eos)) return "equation of state";
    for (int i = 0; i < kModelDoubles; ++i)
        if (std::memcmp(&f.model[i], &want.model[i], sizeof(double))) return kModelNames[i];
    if (f.state_bytes != want.state_bytes) return "state size";
    return nullptr;
}

}  // namespace

extern "C" {

int lbm_interface_constants(const lbm_eos* eos, double Tr, double sigma, double W, double dx, double out[2]) {
    g_init_error.clear();
    if (!eos || !out) return fail(nullptr, LBM_EINVAL, "eos and out must not be NULL");
    lbm_eos unit = *eos;
    unit.K_eos = 1.0;
    int r = check_eos(&unit);
    if (r) return r;
    if (!(Tr > 0 && Tr < 1)) return fail(nullptr, LBM_EINVAL, "Tr must lie in (0, 1) (got %g)", Tr);
    if (!finite_pos(sigma) || !finite_pos(W) || !finite_pos(dx))
        return fail(nullptr, LBM_EINVAL, "sigma, W and dx must be finite and > 0");
    lbm_host::Eos e{unit.kind, unit.a_t, unit.b_t, unit.R, 1.0L};
    long double Tc, pc;
    lbm_host::critical(e, &Tc, &pc);
    // kappa at K_INT = K_EOS = 1: G^2 dx^4 / 4 with G^2 = 2 a~ / dx^2 (Eq. (18))
    const long double kappa1 = 0.5L * e.a * (long double)dx * dx;
    long double s1, w1;
    std::string why;
    if (!lbm_host::interface_sigma_width(e, (long double)Tr * Tc, kappa1, &s1, &w1, &why))
        return fail(nullptr, LBM_EINVAL, "interface at Tr = %g: %s", Tr, why.c_str());
    const long double Kint = (long double)W / w1;
    out[1] = (double)Kint;
    out[0] = (double)((long double)sigma / (Kint * s1));
    return LBM_OK;
}

int lbm_default_params(lbm_params* p) {
    if (!p) return LBM_EINVAL;
    std::memset(p, 0, sizeof *p);
    p->Tr0 = 0.8;
    p->K_int = 2.294922;
    p->varpi = 1.0 / 6.0;
    p->gamma1 = -2.0;
    p->gamma2 = 2.0;
    p->tau_p = 0.5;
    p->s_eps = 1.0;
    p->sigma_e = p->sigma_eps = p->sigma_q = p->sigma_p = 1.0;
    p->tau_j_v = 0.1;
    p->lambda_ratio = 10.0;
    p->cv = 0.0;
    p->ste = 0.005;
    p->dTr_ste = 0.05;
    p->C_ref = 0.0;
    p->precision = LBM_F64;
    p->scheme = LBM_SCHEME_AB;
    return LBM_OK;
}

int lbm_default_eos(lbm_eos* e) {
    if (!e) return LBM_EINVAL;
    e->kind = LBM_EOS_CS;
    e->a_t = 1.0;
    e->b_t = 4.0;
    e->R = 1.0;
    e->K_eos = 0.479820;
    return LBM_OK;
}

int lbm_workspace_bytes(const lbm_lattice* lat, const lbm_params* p, size_t* bytes) {
    int r = check_lattice(lat);
    if (r) return r;
    if ((r = check_params(p))) return r;
    if (!bytes) return fail(nullptr, LBM_EINVAL, "bytes is NULL");
    const size_t N = (size_t)lat->nx * lat->ny;
    const int nbuf = p->scheme == LBM_SCHEME_AA ? 1 : 2;
    *bytes = nbuf * state_buffer_bytes(lat, p) + round256(N * sizeof(double)) +
             round256(lbm_dev::kMaxPartialBlocks * 8 * sizeof(double)) + 256;
    return LBM_OK;
}

int lbm_init(lbm_ctx** out, const lbm_lattice* lat, const lbm_eos* eos, const lbm_params* p,
             void* workspace, size_t workspace_bytes, void* hip_stream) {
    g_init_error.clear();
    if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    int r;
    if ((r = check_lattice(lat)) || (r = check_eos(eos)) || (r = check_params(p))) return r;
    if (lat->bc_x == LBM_BC_HEATED_OUTFLOW) {
        if (p->scheme != LBM_SCHEME_AB || (p->precision != LBM_F64 && p->precision != LBM_F32))
            return fail(nullptr, LBM_EINVAL, "bc_x = LBM_BC_HEATED_OUTFLOW needs LBM_SCHEME_AB and LBM_F64 or LBM_F32");
        if (!(p->Tr_wall > 0)) return fail(nullptr, LBM_EINVAL, "Tr_wall must be > 0 (got %g)", p->Tr_wall);
    }
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(nullptr, LBM_EINVAL, "out of host memory");
    c->lat = *lat;
    c->eos = *eos;
    c->p = *p;
    if ((r = derive(c))) {
        delete c;
        return r;
    }
    fill_consts(c, &c->c64);
    fill_consts(c, &c->c32);
    c->consts = p->precision == LBM_F64 ? (const void*)&c->c64 : (const void*)&c->c32;
    c->walls = p->precision == LBM_F64 ? (const void*)&c->w64 : (const void*)&c->w32;
    // measured defaults (4096^2): short work items, so that vertically adjacent items run
    // at nearly the same time on one XCD and their shared halo rows come from its L2,
    // and each item spends a larger share of its life in the batched prologue with many
    // loads in flight; 16-bit storage is VALU-bound and prefers longer items
    c->shape.rows_per_wave = p->rows_per_wave > 0 ? p->rows_per_wave : lbm_dev::default_rows(p->precision);
    c->shape.waves_per_block = p->waves_per_block > 0 ? p->waves_per_block : lbm_dev::default_waves(p->precision);
    {
        // two columns per lane: 4- and 2-byte storage, even rows, two-buffer scheme
        const bool pair_ok = p->precision != LBM_F64 && lat->nx % 2 == 0;
        c->shape.columns_per_lane = (p->columns_per_lane == 1 || !pair_ok) ? 1 : 2;
    }
    c->host_only = workspace == nullptr;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (!c->host_only) {
        size_t need = 0;
        lbm_workspace_bytes(lat, p, &need);
        if (workspace_bytes < need) {
            fail(nullptr, LBM_ESPACE, "workspace has %zu bytes, %zu needed", workspace_bytes, need);
            delete c;
            return LBM_ESPACE;
        }
        if (reinterpret_cast<uintptr_t>(workspace) & 255) {
            fail(nullptr, LBM_EINVAL, "workspace must be 256-byte aligned");
            delete c;
            return LBM_EINVAL;
        }
        char* w = static_cast<char*>(workspace);
        const size_t sb = state_buffer_bytes(lat, p);
        const size_t N = (size_t)lat->nx * lat->ny;
        c->ws = workspace;
        c->ws_bytes = workspace_bytes;
        c->state_bytes = sb;
        c->buf[0] = w;
        w += sb;
        if (p->scheme == LBM_SCHEME_AB) {
            c->buf[1] = w;
            w += sb;
        } else {
            c->buf[1] = nullptr;
        }
        c->rho_scratch = reinterpret_cast<double*>(w);
        w += round256(N * sizeof(double));
        c->partials = reinterpret_cast<double*>(w);
        w += round256(lbm_dev::kMaxPartialBlocks * 8 * sizeof(double));
        c->result = reinterpret_cast<double*>(w);
    }
    *out = c;
    return LBM_OK;
}

int lbm_set_fields(lbm_ctx* c, const double* rho, const double* ux, const double* uy, const double* T) {
    int r = need_device(c);
    if (r) return r;
    if (!rho || !ux || !uy || !T) return fail(c, LBM_EINVAL, "field pointers must not be NULL");
    c->cur = 0;
    c->steps = 0;
    hipError_t e = lbm_dev::launch_init(c->p.precision, c->consts, c->buf[0], rho, ux, uy, T,
                                        c->p.scheme == LBM_SCHEME_AA ? 0 : 2, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "init launch");
    c->fields_set = true;
    return LBM_OK;
}

int lbm_step(lbm_ctx* c, int64_t n) {
    int r = need_fields(c);
    if (r) return r;
    if (n < 0) return fail(c, LBM_EINVAL, "n must be >= 0");
    if (c->lat.bc_x == LBM_BC_HEATED_OUTFLOW) {
        // many steps per launch (the whole small lattice is one workgroup), in chunks
        // that end at every state check
        const int64_t chunk = 2048;
        while (n > 0) {
            int64_t k = n < chunk ? n : chunk;
            if (c->p.check_every > 0) {
                const int64_t to_check = c->p.check_every - c->steps % c->p.check_every;
                if (to_check < k) k = to_check;
            }
            hipError_t e = lbm_dev::launch_step_bounded(c->p.precision, c->consts, c->walls, c->buf[0], c->buf[1],
                                                        c->cur, (int)k, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "bounded step launch");
            c->cur ^= (int)(k & 1);
            c->steps += k;
            n -= k;
            if (c->p.check_every > 0 && c->steps % c->p.check_every == 0) {
                double out[8];
                if ((r = state_check(c, out))) return r;
            }
        }
        return LBM_OK;
    }
    for (int64_t k = 0; k < n; ++k) {
        hipError_t e;
        if (c->p.scheme == LBM_SCHEME_AB) {
            // the step count seeds the stochastic-rounding stream (the constants are
            // copied into the launch's arguments, so they may change afterwards)
            c->c64.step = c->c32.step = (uint32_t)c->steps;
            e = lbm_dev::launch_step_ab(c->p.precision, c->consts, c->buf[c->cur], c->buf[c->cur ^ 1], c->shape,
                                        c->p.rounding == LBM_ROUND_STOCHASTIC, c->stream);
            if (e == hipSuccess) c->cur ^= 1;
        } else {
            e = lbm_dev::launch_step_aa(c->p.precision, c->consts, c->buf[0], c->rho_scratch, (int)(c->steps & 1),
                                        c->shape, c->stream);
        }
        if (e != hipSuccess) return hip_fail(c, e, "step launch");
        ++c->steps;
        if (c->p.check_every > 0 && c->steps % c->p.check_every == 0) {
            double out[8];
            if ((r = state_check(c, out))) return r;
        }
    }
    return LBM_OK;
}

int lbm_moments(lbm_ctx* c, double* rho, double* ux, double* uy, double* T) {
    int r = need_fields(c);
    if (r) return r;
    if (!rho) return fail(c, LBM_EINVAL, "rho must not be NULL");
    if (c->lat.bc_x == LBM_BC_HEATED_OUTFLOW) {
        hipError_t e = lbm_dev::launch_moments_bounded(c->p.precision, c->consts, c->walls, current_state(c), rho,
                                                       ux, uy, T, c->stream);
        return e == hipSuccess ? LBM_OK : hip_fail(c, e, "bounded moments launch");
    }
    hipError_t e = lbm_dev::launch_density(c->p.precision, c->consts, current_state(c), aa_parity(c), rho, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "density launch");
    if (ux || uy || T) {
        e = lbm_dev::launch_moments(c->p.precision, c->consts, current_state(c), aa_parity(c), rho, ux, uy, T,
                                    c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "moments launch");
    }
    return LBM_OK;
}

int lbm_invariants(lbm_ctx* c, double* out, int n_out) {
    int r = need_fields(c);
    if (r) return r;
    if (!out || n_out < 8) return fail(c, LBM_EINVAL, "out must hold at least 8 doubles");
    return state_check(c, out);
}

int lbm_derived(const lbm_ctx* c, double* out, int n) {
    if (!c || !out || n < 0) return LBM_EINVAL;
    for (int i = 0; i < n && i < 27; ++i) out[i] = c->derived[i];
    return LBM_OK;
}

int lbm_launch_shape(const lbm_ctx* c, int32_t* rows_per_wave, int32_t* waves_per_block, int32_t* columns_per_lane) {
    if (!c || !rows_per_wave || !waves_per_block) return LBM_EINVAL;
    if (columns_per_lane) *columns_per_lane = c->p.scheme == LBM_SCHEME_AB ? c->shape.columns_per_lane : 1;
    *rows_per_wave = c->shape.rows_per_wave;
    *waves_per_block = c->shape.waves_per_block;
    return LBM_OK;
}

int lbm_step_count(const lbm_ctx* c, int64_t* steps) {
    if (!c || !steps) return LBM_EINVAL;
    *steps = c->steps;
    return LBM_OK;
}

int lbm_state_bytes(const lbm_ctx* c, size_t* bytes) {
    if (!c || !bytes) return LBM_EINVAL;
    *bytes = state_buffer_bytes(&c->lat, &c->p);
    return LBM_OK;
}

int lbm_save_state(lbm_ctx* c, void* dst, int64_t* steps) {
    int r = need_fields(c);
    if (r) return r;
    if (!dst) return fail(c, LBM_EINVAL, "dst is NULL");
    hipError_t e = hipMemcpyAsync(dst, current_state(c), c->state_bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "save copy");
    if (steps) *steps = c->steps;
    return LBM_OK;
}

int lbm_load_state(lbm_ctx* c, const void* src, int64_t steps) {
    int r = need_device(c);
    if (r) return r;
    if (!src || steps < 0) return fail(c, LBM_EINVAL, "src is NULL or steps < 0");
    c->cur = 0;
    hipError_t e = hipMemcpyAsync(c->buf[0], src, c->state_bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "load copy");
    c->steps = steps;
    c->fields_set = true;
    return LBM_OK;
}

int lbm_save(lbm_ctx* c, const char* path) {
    int r = need_fields(c);
    if (r) return r;
    if (!path || !*path) return fail(c, LBM_EINVAL, "path is NULL or empty");
    std::vector<unsigned char> host;
    try {
        host.resize(c->state_bytes);
    } catch (const std::bad_alloc&) {
        return fail(c, LBM_EIO, "cannot allocate %zu bytes of host memory to stage the state", c->state_bytes);
    }
    hipError_t e = hipMemcpyAsync(host.data(), current_state(c), c->state_bytes, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "checkpoint copy to host");
    FileHeader h;
    fill_header(c, &h);
    h.checksum = fnv1a(host.data(), host.size());
    // written next to the target and renamed over it, so an interrupted save leaves any
    // previous checkpoint of that name intact
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(c, LBM_EIO, "cannot open %s for writing: %s", tmp.c_str(), std::strerror(errno));
    bool ok = std::fwrite(&h, sizeof h, 1, f) == 1 &&
              (host.empty() || std::fwrite(host.data(), host.size(), 1, f) == 1);
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(c, LBM_EIO, "cannot write checkpoint %s", path);
    }
    return LBM_OK;
}

int lbm_load(lbm_ctx* c, const char* path) {
    int r = need_device(c);
    if (r) return r;
    if (!path || !*path) return fail(c, LBM_EINVAL, "path is NULL or empty");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(c, LBM_EIO, "cannot open %s: %s", path, std::strerror(errno));
    FileHeader h;
    if (std::fread(&h, sizeof h, 1, f) != 1) {
        std::fclose(f);
        return fail(c, LBM_EIO, "%s: truncated header", path);
    }
    if (std::memcmp(h.magic, kFileMagic, sizeof kFileMagic) || h.version != kFileVersion ||
        h.header_bytes != sizeof(FileHeader)) {
        std::fclose(f);
        return fail(c, LBM_EIO, "%s: not a checkpoint of this format (magic, version %u or header size %u)", path,
                    h.version, h.header_bytes);
    }
    FileHeader want;
    fill_header(c, &want);
    if (const char* what = header_mismatch(h, want)) {
        std::fclose(f);
        return fail(c, LBM_EINVAL, "%s was written for a different %s", path, what);
    }
    if (h.steps < 0) {
        std::fclose(f);
        return fail(c, LBM_EIO, "%s: negative step count", path);
    }
    std::vector<unsigned char> host;
    try {
        host.resize(c->state_bytes);
    } catch (const std::bad_alloc&) {
        std::fclose(f);
        return fail(c, LBM_EIO, "cannot allocate %zu bytes of host memory to stage the state", c->state_bytes);
    }
    const bool got = host.empty() || std::fread(host.data(), host.size(), 1, f) == 1;
    std::fclose(f);
    if (!got) return fail(c, LBM_EIO, "%s: truncated state", path);
    if (fnv1a(host.data(), host.size()) != h.checksum) return fail(c, LBM_EIO, "%s: checksum mismatch", path);
    hipError_t e = hipMemcpyAsync(c->buf[0], host.data(), c->state_bytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "checkpoint copy to device");
    c->cur = 0;
    c->steps = h.steps;
    c->fields_set = true;
    return LBM_OK;
}

int lbm_destroy(lbm_ctx* c) {
    delete c;
    return LBM_OK;
}

const char* lbm_strerror(int code) {
    switch (code) {
        case LBM_OK: return "ok";
        case LBM_EINVAL: return "invalid argument";
        case LBM_ESPACE: return "workspace too small";
        case LBM_EHIP: return "HIP runtime error";
        case LBM_ENONFINITE: return "state check failed (non-finite or out-of-range values)";
        case LBM_ESTATE: return "call out of order";
        case LBM_EIO: return "checkpoint file error";
        default: return "unknown error";
    }
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

}  // extern "C"
