/* Drives the host-only paths of the library under AddressSanitizer and
 * UndefinedBehaviorSanitizer: parameter and shape validation (valid, invalid and
 * non-finite values), derived constants, the Maxwell construction for both equations of
 * state over the whole temperature range, error strings, batch and checkpoint calls on
 * host-only contexts, and NULL arguments.  Exits 0 when every call returned what the
 * header promises; any sanitizer report aborts the process. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "lbm.h"

static int failures = 0;
#define EXPECT(cond)                                                   \
    do {                                                               \
        if (!(cond)) {                                                 \
            fprintf(stderr, "line %d: %s\n", __LINE__, #cond);         \
            ++failures;                                                \
        }                                                              \
    } while (0)

static int init_host(lbm_ctx** c, int nx, int ny, const lbm_eos* e, const lbm_params* p) {
    lbm_lattice lat = {nx, ny, 1.0};
    return lbm_init(c, &lat, e, p, NULL, 0, NULL);
}

int main(void) {
    lbm_params p0, p;
    lbm_eos cs, vdw;
    EXPECT(lbm_default_params(&p0) == LBM_OK && lbm_default_eos(&cs) == LBM_OK);
    EXPECT(lbm_default_params(NULL) == LBM_EINVAL && lbm_default_eos(NULL) == LBM_EINVAL);
    vdw.kind = LBM_EOS_VDW; vdw.a_t = 9.0 / 49.0; vdw.b_t = 2.0 / 21.0; vdw.R = 1.0; vdw.K_eos = 1.0;

    /* Maxwell construction over the whole range and at its ends */
    for (int k = 1; k < 100; ++k) {
        double out[4];
        const double Tr = k / 100.0;
        int r1 = lbm_maxwell(&cs, Tr, out);
        EXPECT(r1 == LBM_OK || r1 == LBM_EINVAL);
        if (r1 == LBM_OK) EXPECT(out[0] > 0 && out[1] > out[0] && out[2] > 0 && out[3] > 0);
        int r2 = lbm_maxwell(&vdw, Tr, out);
        EXPECT(r2 == LBM_OK || r2 == LBM_EINVAL);
    }
    const double bad_tr[] = {0.0, 1.0, -1.0, 2.0, NAN, INFINITY};
    for (unsigned k = 0; k < sizeof bad_tr / sizeof *bad_tr; ++k) {
        double out[4];
        EXPECT(lbm_maxwell(&cs, bad_tr[k], out) == LBM_EINVAL);
    }
    EXPECT(lbm_maxwell(NULL, 0.8, NULL) == LBM_EINVAL);

    /* valid host-only contexts across temperatures, EOS kinds, precisions and schemes */
    for (int k = 60; k <= 95; k += 5) {
        for (int kind = 0; kind < 2; ++kind) {
            for (int prec = LBM_F64; prec <= LBM_BF16; ++prec) {
                p = p0;
                p.Tr0 = k / 100.0;
                p.precision = prec;
                p.scheme = (k / 5) % 2;
                if (kind) p.K_int = 1.0;
                lbm_ctx* c = NULL;
                EXPECT(init_host(&c, 37, 23, kind ? &vdw : &cs, &p) == LBM_OK && c != NULL);
                double d[26];
                EXPECT(lbm_derived(c, d, 26) == LBM_OK);
                for (int i = 0; i < 26; ++i) EXPECT(isfinite(d[i]));
                int32_t rows, waves, cols;
                EXPECT(lbm_launch_shape(c, &rows, &waves, &cols) == LBM_OK && rows > 0 && waves > 0);
                int64_t steps = -1;
                EXPECT(lbm_step_count(c, &steps) == LBM_OK && steps == 0);
                size_t sb = 0;
                EXPECT(lbm_state_bytes(c, &sb) == LBM_OK && sb >= (size_t)18 * 37 * 23 * 2);
                EXPECT(lbm_step(c, 1) == LBM_ESTATE && lbm_set_fields(c, NULL, NULL, NULL, NULL) == LBM_ESTATE);
                EXPECT(lbm_save(c, "/nonexistent/x.lbm") == LBM_ESTATE && lbm_load(c, "x.lbm") == LBM_ESTATE);
                double inv[8];
                EXPECT(lbm_invariants(c, inv, 8) == LBM_ESTATE);
                EXPECT(strlen(lbm_last_error(c)) > 0);
                lbm_lattice lat = {37, 23, 1.0};
                size_t ws = 0;
                EXPECT(lbm_workspace_bytes(&lat, &p, &ws) == LBM_OK && ws > sb);
                EXPECT(lbm_destroy(c) == LBM_OK);
            }
        }
    }

    /* every double of lbm_params set to a bad value in turn */
    const double bads[] = {NAN, INFINITY, -INFINITY, -1.0, 0.0, 1e300};
    double* fields[] = {&p.Tr0, &p.K_int, &p.varpi, &p.gamma1, &p.gamma2, &p.tau_p, &p.s_eps, &p.sigma_e,
                        &p.sigma_eps, &p.sigma_q, &p.sigma_p, &p.tau_j_v, &p.lambda_ratio, &p.cv, &p.ste,
                        &p.dTr_ste, &p.C_ref, &p.accel_x, &p.accel_y, &p.cs_override, &p.rho_ref, &p.T_ref,
                        &p.Tr_wall, &p.Tr_far, &p.p_out};
    for (unsigned f = 0; f < sizeof fields / sizeof *fields; ++f) {
        for (unsigned b = 0; b < sizeof bads / sizeof *bads; ++b) {
            p = p0;
            *fields[f] = bads[b];
            lbm_ctx* c = NULL;
            int r = init_host(&c, 16, 16, &cs, &p);
            EXPECT((r == LBM_OK) == (c != NULL));
            if (r != LBM_OK) EXPECT(strlen(lbm_last_error(NULL)) > 0);
            lbm_destroy(c);
        }
    }
    /* integer fields */
    const int ibad[] = {-1, 3, 7, 65537, -2147483647 - 1, 2147483647};
    int32_t* ifields[] = {&p.precision, &p.scheme, &p.rows_per_wave, &p.waves_per_block, &p.columns_per_lane,
                          &p.rounding, &p.check_every};
    for (unsigned f = 0; f < sizeof ifields / sizeof *ifields; ++f) {
        for (unsigned b = 0; b < sizeof ibad / sizeof *ibad; ++b) {
            p = p0;
            *ifields[f] = ibad[b];
            lbm_ctx* c = NULL;
            int r = init_host(&c, 16, 16, &cs, &p);
            EXPECT((r == LBM_OK) == (c != NULL));
            lbm_destroy(c);
        }
    }
    /* bounded lattices: valid and invalid shapes, schemes, precisions and wall states */
    {
        const int bshapes[][2] = {{1024, 4}, {4, 1}, {3, 4}, {8192, 1}, {8193, 1}, {100, 100}};
        for (unsigned k = 0; k < sizeof bshapes / sizeof *bshapes; ++k) {
            for (int prec = LBM_F64; prec <= LBM_BF16; ++prec) {
                for (int scheme = 0; scheme < 2; ++scheme) {
                    p = p0;
                    p.precision = prec;
                    p.scheme = scheme;
                    p.Tr_wall = 0.85;
                    lbm_lattice lat = {bshapes[k][0], bshapes[k][1], 1.0, LBM_BC_HEATED_OUTFLOW};
                    lbm_ctx* c = NULL;
                    int r = lbm_init(&c, &lat, &cs, &p, NULL, 0, NULL);
                    const int ok = lat.nx >= 4 && lat.nx * lat.ny <= 8192 && scheme == LBM_SCHEME_AB &&
                                   prec <= LBM_F32;
                    EXPECT((r == LBM_OK) == (ok != 0) && (r == LBM_OK) == (c != NULL));
                    if (c) {
                        double d[27];
                        EXPECT(lbm_derived(c, d, 27) == LBM_OK && d[26] > 0 && d[26] < d[3]);
                    }
                    lbm_destroy(c);
                }
            }
        }
        const double walls[][3] = {{0.0, 0, 0}, {-1, 0, 0}, {0.85, 0.8, 0}, {0.85, 0, 1.0}, {1.5, 0, 0},
                                   {0.85, 0, -1}, {NAN, 0, 0}, {0.85, INFINITY, 0}};
        for (unsigned k = 0; k < sizeof walls / sizeof *walls; ++k) {
            p = p0;
            p.Tr_wall = walls[k][0];
            p.Tr_far = walls[k][1];
            p.p_out = walls[k][2];
            lbm_lattice lat = {64, 4, 1.0, LBM_BC_HEATED_OUTFLOW};
            lbm_ctx* c = NULL;
            int r = lbm_init(&c, &lat, &cs, &p, NULL, 0, NULL);
            EXPECT((r == LBM_OK) == (c != NULL));
            lbm_destroy(c);
        }
        lbm_lattice bad = {64, 4, 1.0, 7};
        lbm_ctx* c = NULL;
        EXPECT(lbm_init(&c, &bad, &cs, &p0, NULL, 0, NULL) == LBM_EINVAL && c == NULL);
    }

    /* shapes and EOS */
    const int shapes[][2] = {{0, 1}, {1, 0}, {-5, 5}, {65536, 65536}, {1, 1}, {1, 2147483647}};
    for (unsigned k = 0; k < sizeof shapes / sizeof *shapes; ++k) {
        lbm_ctx* c = NULL;
        int r = init_host(&c, shapes[k][0], shapes[k][1], &cs, &p0);
        EXPECT((r == LBM_OK) == (c != NULL));
        lbm_destroy(c);
    }
    lbm_eos e = cs;
    e.kind = 9;
    lbm_ctx* c = NULL;
    EXPECT(init_host(&c, 8, 8, &e, &p0) == LBM_EINVAL && c == NULL);
    e = cs;
    e.b_t = NAN;
    EXPECT(init_host(&c, 8, 8, &e, &p0) == LBM_EINVAL && c == NULL);
    EXPECT(lbm_init(&c, NULL, &cs, &p0, NULL, 0, NULL) == LBM_EINVAL);
    EXPECT(lbm_init(&c, NULL, NULL, NULL, NULL, 0, NULL) == LBM_EINVAL);

    /* interface constants (sigma, W -> K_EOS, K_INT) over the temperature range */
    for (int k = 55; k <= 97; k += 6) {
        double kk[2];
        EXPECT(lbm_interface_constants(&cs, k / 100.0, 0.01, 10.0, 1.0, kk) == LBM_OK && kk[0] > 0 && kk[1] > 0);
        EXPECT(lbm_interface_constants(&vdw, k / 100.0, 0.02, 8.0, 0.5, kk) == LBM_OK && kk[0] > 0 && kk[1] > 0);
    }
    {
        double kk[2];
        EXPECT(lbm_interface_constants(&cs, 1.0, 0.01, 10.0, 1.0, kk) == LBM_EINVAL);
        EXPECT(lbm_interface_constants(&cs, 0.8, NAN, 10.0, 1.0, kk) == LBM_EINVAL);
        EXPECT(lbm_interface_constants(NULL, 0.8, 0.01, 10.0, 1.0, kk) == LBM_EINVAL);
        EXPECT(lbm_interface_constants(&cs, 0.8, 0.01, 10.0, 1.0, NULL) == LBM_EINVAL);
    }

    /* error strings */
    for (int code = -10; code <= 1; ++code) EXPECT(lbm_strerror(code) != NULL);

    /* batch calls on host-only members and bad arguments */
    size_t bytes = 0;
    EXPECT(lbm_batch_workspace_bytes(64, LBM_F32, &bytes) == LBM_OK && bytes > 0);
    EXPECT(lbm_batch_workspace_bytes(0, LBM_F32, &bytes) == LBM_EINVAL);
    EXPECT(lbm_batch_workspace_bytes(4, 11, &bytes) == LBM_EINVAL);
    EXPECT(init_host(&c, 16, 16, &cs, &p0) == LBM_OK);
    lbm_batch* b = NULL;
    lbm_ctx* members[2] = {c, NULL};
    EXPECT(lbm_batch_create(&b, members, 1, (void*)(size_t)4096, 1 << 20) == LBM_ESTATE && b == NULL);
    int rb = lbm_batch_create(&b, members, 2, (void*)(size_t)4096, 1 << 20);
    EXPECT((rb == LBM_EINVAL || rb == LBM_ESTATE) && b == NULL);
    EXPECT(lbm_batch_create(&b, members, 0, (void*)(size_t)4096, 1 << 20) == LBM_EINVAL && b == NULL);
    EXPECT(strlen(lbm_batch_last_error(NULL)) > 0);
    EXPECT(lbm_batch_destroy(NULL) == LBM_OK);
    EXPECT(lbm_destroy(c) == LBM_OK && lbm_destroy(NULL) == LBM_OK);

    if (failures) {
        fprintf(stderr, "%d expectation(s) failed\n", failures);
        return 1;
    }
    printf("host paths ok\n");
    return 0;
}
