/*
 * sanitize_driver.c -- exercises every path of the CPU oracle (both
 * closures, 1D and 2D, open and periodic boundaries, the axisymmetric
 * geometry, slices, every observable, the unit entry points) in a host
 * build with AddressSanitizer and UndefinedBehaviorSanitizer. TEST
 * INFRASTRUCTURE: tests/test_oracle_sanitize.py compiles and runs it.
 * Exit status 0 and no sanitizer report mean no out-of-bounds access,
 * use after free, leak or undefined arithmetic on these paths.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "lbw_oracle.h"

static int run_case(int dims, int nz, int nx, int closure, double dvel, int bcz, int bcx, int geom,
                    int nslices, double alpha, int steps)
{
    orc_params p = {0};
    p.dims = dims; p.nz = nz; p.nx = nx;
    p.delta = 2.0 * M_PI / 32.0; p.dt = 0.1 * p.delta;
    p.tau_tilde = dims == 1 ? 0.52 : 0.53;
    p.closure = closure; p.dvel = dvel; p.bc_z = bcz; p.bc_x = bcx; p.mu = 0.03;
    p.alpha = alpha; p.sigma_z = 0.8; p.sigma_x = 0.6; p.z0 = 4.0; p.x0 = 0.0;
    p.geom = geom;
    double w[5] = {0.6, 1.2, 0.9, 1.4, 0.7};
    if (nslices) { p.nslices = nslices; p.slice_w = w; p.slice_zmin = -2.0; p.slice_zmax = 2.0; }
    orc_state *s = orc_create(&p);
    if (!s) { fprintf(stderr, "create failed\n"); return 1; }
    const int nc = nz * nx;
    double *n = malloc(sizeof(double) * nc), *uz = malloc(sizeof(double) * nc), *ux = malloc(sizeof(double) * nc);
    for (int c = 0; c < nc; ++c) {
        n[c] = 1.0 + 0.01 * sin(0.37 * c);
        uz[c] = 0.02 * cos(0.21 * c);
        ux[c] = dims == 2 ? 0.015 * sin(0.13 * c) : 0.0;
    }
    if (orc_init(s, n, uz, dims == 2 ? ux : NULL, alpha != 0.0) != 0) return 1;
    if (orc_step(s, steps) != 0) return 1;
    double *out = malloc(sizeof(double) * nc), diag[8];
    for (int q = 0; q < ORC_NOBS; ++q) {
        if (orc_get(s, q, out) != 0) continue;  /* observables the closure does not have */
        for (int c = 0; c < nc; ++c)
            if (!isfinite(out[c])) { fprintf(stderr, "non-finite observable %d\n", q); return 1; }
    }
    orc_diagnostics(s, diag);
    /* arbitrary scalars, the Yee arrays, more steps */
    const int K = orc_num_scalars(s);
    double *A = malloc(sizeof(double) * K * nc);
    for (int k = 0; k < K; ++k)
        for (int c = 0; c < nc; ++c) A[k * nc + c] = (k == 0 ? 1.0 : 0.01) * (1.0 + 0.001 * k);
    orc_init_moments(s, A, uz, dims == 2 ? ux : NULL);
    for (int f = 0; f < (dims == 2 ? 3 : 1); ++f) orc_set_yee(s, f, out);
    orc_step(s, 3);
    orc_diagnostics(s, diag);
    (void)orc_bunch(s, 1.0, 0.2, 0.5);
    orc_destroy(s);
    free(n); free(uz); free(ux); free(out); free(A);
    return 0;
}

int main(void)
{
    int bad = 0;
    for (int cl = 0; cl < 2; ++cl) {
        bad |= run_case(1, 67, 1, cl, 1.0, ORC_BC_OPEN, ORC_BC_OPEN, ORC_GEOM_SLAB, 0, 0.4, 20);
        bad |= run_case(1, 40, 1, cl, 3.0, ORC_BC_PERIODIC, ORC_BC_OPEN, ORC_GEOM_SLAB, 0, 0.0, 20);
        bad |= run_case(2, 37, 11, cl, 3.0, ORC_BC_OPEN, ORC_BC_OPEN, ORC_GEOM_SLAB, 5, 0.5, 12);
        bad |= run_case(2, 24, 9, cl, 3.0, ORC_BC_PERIODIC, ORC_BC_PERIODIC, ORC_GEOM_SLAB, 0, 0.0, 12);
        bad |= run_case(2, 30, 10, cl, 3.0, ORC_BC_OPEN, ORC_BC_OPEN, ORC_GEOM_AXI, 0, 0.5, 12);
    }
    /* unit entry points */
    double f[9], o[12], Aw[8] = {1.0, 1.05, 0.01, 0.02, 0.03, 0.03, 0.031, 0.001};
    orc_feq(2, 1.0, 0.1, -0.05, 10.0, f);
    orc_feq(1, 1.0, 0.1, 0.0, 10.0, f);
    orc_lec_recover(1.1, 0.3, -0.2, 3.0, 0.05, o);
    orc_lec_recover(1.1, 0.0, 0.0, 1.0, 0.05, o);
    orc_warmc_recover(2, Aw, o);
    orc_warmc_recover(1, Aw, o);
    (void)orc_ppar(0.03, 0.03, 0.031, 0.001, 0.02, 0.01);
    (void)orc_lambda0(0.04, 3.0);
    double Ain[64 * 8], Aout[64 * 8];
    for (int c = 0; c < 64 * 8; ++c) Ain[c] = exp(-0.01 * (c % 64 - 32) * (c % 64 - 32));
    orc_ade_run(2, 64, 8, 1.0, 0.1, 0.8, ORC_BC_PERIODIC, 0.3, 0.1, Ain, 30, Aout);
    orc_ade_run(1, 64, 1, 1.0, 0.1, 0.8, ORC_BC_OPEN, 0.3, 0.0, Ain, 30, Aout);
    if (!bad) printf("sanitize driver ok\n");
    return bad;
}
