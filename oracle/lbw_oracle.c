/*
 * lbw_oracle.c -- plain FP64 CPU oracle of the moment-matching lattice
 * Boltzmann (LB) scheme for warm relativistic plasma wakes of Simeoni et al.,
 * "Lattice Boltzmann method for warm fluid simulations of plasma wakefield
 * acceleration" (arXiv 2309.04872).
 *
 * TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
 * baseline of the benchmark load it. It shares no code with the GPU library.
 *
 * Every loop runs over whole arrays in the order of one time step:
 *   S1 moments A_k = sum_i f_{k,i}                       (Sec. 2.2, eq. disc-moments-ade)
 *   S2 closure recovery (LEC fixed point, Sec. 3.1; WARMC algebra, Sec. 4.1 + App. A)
 *   S3 E^n and B^n = B^{n-1/2} - dt/2 curl E^n at the nodes (Yee FDTD, Sec. 5)
 *   S4 rigid driver density (Sec. 5, eq. bunch-density)
 *   S5 forcing F_k (eq. lb-ade-lec-comps-F, eq. lb-ade-warmc-comps-F, App. A)
 *   S6 BGK collision toward the moment-matching equilibrium plus S_i = w_i F
 *      (Sec. 2.1 eq. lbe/lsource, Sec. 2.2 eq. ade-feq, S_i = w_i F)
 *   S7 streaming with open (copy) or periodic boundaries (Sec. 2.2 eq. open-bc)
 *   S8 recovery of n^{n+1}, u^{n+1}
 *   S9 Yee update with the plasma current J^{n+1} and the driver current
 *   S10 store the lagged values for the explicit time derivatives (warm closure)
 *
 * Readings of points the paper leaves open are listed in the design notes;
 * the ones that change arithmetic are repeated at the place they apply.
 */
#include "lbw_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------- */
/* Velocity stencils. The paper's 19-velocity 3D stencil (Sec. 2.1, Fig. 1)
 * projected on one axis gives D1Q3 (2/3, 1/6, 1/6) and on a plane gives
 * D2Q9 (4/9, 1/9, 1/36): summing the 3D weights over the dropped components. */
static const int D1_ez[3] = {0, 1, -1};
static const double D1_w[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};

static const int D2_ez[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
static const int D2_ex[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
static const double D2_w[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                               1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                               1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* Scalar (advected quantity) indices. */
/* LEC (eq. lb-ade-lec-comps-A): n, and the momentum-like vector
 * [1 + (1 + D/2) mu (n/(gamma n_i))^{2/D}] n p. */
enum { L_N = 0, L_AZ = 1, L_AX = 2 };
/* WARMC (eq. lb-ade-warmc-comps-A, App. A with r -> x, phi -> y):
 * n, n lambda, n lambda u_z, n lambda u_x, lambda theta^{zz}, ^{xx}, ^{yy}, ^{xz}.
 * In 1D only n, n lambda, n lambda u_z, lambda theta^{zz} are advected. */
enum { W_N = 0, W_NL = 1, W_NLUZ = 2, W_NLUX = 3, W_THZZ = 4, W_THXX = 5,
       W_THYY = 6, W_THXZ = 7 };
enum { W1_N = 0, W1_NL = 1, W1_NLUZ = 2, W1_THZZ = 3 };

/* Recovered per-node quantities. */
enum {
    R_N = 0, R_UZ, R_UX, R_GAM, R_N0, R_PHI, R_LAM, R_THZZ, R_THXX, R_THYY,
    R_THXZ, R_TH0Z, R_TH0X, R_TH00, R_LUZ, R_LUX, R_ITER, NR
};
/* Lagged quantities for the explicit time derivatives of the warm closure. */
enum { G_TH00 = 0, G_TH0Z, G_TH0X, G_LUZ, G_LUX, NG };

struct orc_state {
    orc_params p;
    double *slice_w;
    int mirror_x[9];  /* direction with e_x reversed (2D) */
    int Q, K, nz, nx, ncell;
    const int *ez, *ex;
    const double *w;
    double *f, *fs;          /* populations [K][Q][ncell]; post-collision */
    double *Ez, *Ex, *By;    /* Yee arrays (E^n, B^{n-1/2}) */
    double *Bh;              /* B^n on the Yee grid (temporary) */
    double *En_z, *En_x, *Bn_y; /* node fields */
    double *A;               /* [K][ncell] */
    double *R, *R1;          /* [NR][ncell]: step n and step n+1 */
    double *F;               /* [K][ncell] */
    double *lag;             /* [NG][ncell] */
    double *nb;              /* driver density at nodes */
    int have_lag;
    long step;
    long fallbacks;
};

/* ---------------------------------------------------------------------- */
/* Index helpers: open boundaries copy the nearest bulk node (eq. open-bc),
 * periodic boundaries wrap. The same rule serves streaming sources, the
 * central differences and the Yee ghosts. */
static int fixidx(int i, int n, int bc)
{
    if (bc == ORC_BC_PERIODIC) {
        i %= n;
        if (i < 0) i += n;
        return i;
    }
    if (i < 0) return 0;
    if (i >= n) return n - 1;
    return i;
}

static int cell(const orc_state *s, int j, int i)
{
    return fixidx(j, s->nx, s->p.bc_x) * s->nz + fixidx(i, s->nz, s->p.bc_z);
}

/* Yee arrays: along a staggered direction with open boundaries the n - 1
 * half-integer positions between the n nodes are real and the last slot is a
 * copy ghost, so both ends of the domain see the same copy rule; periodic
 * boundaries have n real positions. sz / sx: staggered along z / x. */
static int fixstag(int i, int n, int bc)
{
    if (bc == ORC_BC_PERIODIC) return fixidx(i, n, bc);
    return fixidx(i, n - 1, bc);
}

static int ycell(const orc_state *s, int j, int i, int sz, int sx)
{
    int jj = sx ? fixstag(j, s->nx, s->p.bc_x) : fixidx(j, s->nx, s->p.bc_x);
    int ii = sz ? fixstag(i, s->nz, s->p.bc_z) : fixidx(i, s->nz, s->p.bc_z);
    return jj * s->nz + ii;
}
#define EZ_AT(j, i) s->Ez[ycell(s, (j), (i), 1, 0)]
#define EX_AT(j, i) s->Ex[ycell(s, (j), (i), 0, 1)]
#define BY_AT(arr, j, i) (arr)[ycell(s, (j), (i), 1, 1)]

static double node_z(const orc_state *s, double i) { return i * s->p.delta; }
static double node_x(const orc_state *s, double j)
{
    if (s->p.geom == ORC_GEOM_AXI) return (j + 0.5) * s->p.delta; /* r_j */
    return (j - 0.5 * (s->nx - 1)) * s->p.delta;
}

/* ---------------------------------------------------------------------- */
/* Rigid bi-Gaussian driver moving at c along +z (Sec. 5, eq. bunch-density),
 * read with rms widths: exp(-zeta^2 / (2 sigma_z^2)) exp(-x^2 / (2 sigma_x^2)),
 * zeta = z - z0 - t. Optional piecewise-constant slice weights over
 * [slice_zmin, slice_zmax) in zeta; outside that span the bunch is empty. */
static double slice_weight(const orc_state *s, double zeta)
{
    if (s->p.nslices <= 0) return 1.0;
    double a = s->p.slice_zmin, b = s->p.slice_zmax;
    if (!(zeta >= a && zeta < b)) return 0.0;
    int k = (int)floor((zeta - a) / (b - a) * s->p.nslices);
    if (k < 0) k = 0;
    if (k >= s->p.nslices) k = s->p.nslices - 1;
    return s->slice_w[k];
}

double orc_bunch(const orc_state *s, double z, double x, double t)
{
    if (s->p.alpha == 0.0) return 0.0;
    double zeta = z - s->p.z0 - t;
    double g = s->p.alpha * slice_weight(s, zeta) *
               exp(-zeta * zeta / (2.0 * s->p.sigma_z * s->p.sigma_z));
    if (s->p.dims == 2) {
        double dx = x - s->p.x0;
        g *= exp(-dx * dx / (2.0 * s->p.sigma_x * s->p.sigma_x));
    }
    return g;
}

/* Integral of the longitudinal profile from zeta to +infinity. */
static double bunch_tail_integral(const orc_state *s, double zeta)
{
    double sz = s->p.sigma_z, c = sz * sqrt(M_PI / 2.0), r2s = sqrt(2.0) * sz;
    if (s->p.nslices <= 0) return c * erfc(zeta / r2s);
    double a = s->p.slice_zmin, b = s->p.slice_zmax, h = (b - a) / s->p.nslices;
    double acc = 0.0;
    for (int k = 0; k < s->p.nslices; ++k) {
        double lo = a + k * h, hi = a + (k + 1) * h;
        if (zeta >= hi) continue;
        if (zeta > lo) lo = zeta;
        acc += s->slice_w[k] * c * (erf(hi / r2s) - erf(lo / r2s));
    }
    return acc;
}

/* ---------------------------------------------------------------------- */
/* Moment-matching equilibrium (Sec. 2.2, eq. ade-feq) with xi_i = Lambda e_i,
 * nu^2 = Lambda^2 / 3 and the quadratic term carrying the factor 1/2 of the
 * standard second-order form (the printed equation drops it; without it
 * sum_i f_eq != A). */
static double feq(double w, double A, double uxi, double uu, double nu2)
{
    return w * A * (1.0 + uxi / nu2 + (uxi * uxi) / (2.0 * nu2 * nu2) -
                    uu / (2.0 * nu2));
}

void orc_feq(int dims, double A, double uz, double ux, double lattice_speed,
             double *out)
{
    double nu2 = lattice_speed * lattice_speed / 3.0;
    double uu = uz * uz + ux * ux;
    if (dims == 1) {
        for (int q = 0; q < 3; ++q)
            out[q] = feq(D1_w[q], A, uz * lattice_speed * D1_ez[q], uz * uz, nu2);
    } else {
        for (int q = 0; q < 9; ++q) {
            double uxi = lattice_speed * (uz * D2_ez[q] + ux * D2_ex[q]);
            out[q] = feq(D2_w[q], A, uxi, uu, nu2);
        }
    }
}

/* ---------------------------------------------------------------------- */
/* LEC transport-velocity recovery (Sec. 3.1): start from p^(0) = A_1 / n and
 * iterate u^(k) = p^(k) / sqrt(1 + |p^(k)|^2), gamma^(k) = 1 / sqrt(1 - u^(k)^2),
 * p^(k+1) = p^(0) / [1 + (1 + D/2) mu (n / gamma^(k))^{2/D}] until
 * |p^(k+1) - p^(k)| <= 1e-15 (1 + |p^(k+1)|), at most 64 times. If that does
 * not settle, bisect p (1 + (1 + D/2) mu (n / sqrt(1 + p^2))^{2/D}) = |p^(0)|
 * on [0, |p^(0)|]. Returns the iteration count (negative: fallback used). */
static double lec_h(double n, double g, double D, double mu)
{
    return 1.0 + (1.0 + 0.5 * D) * mu * pow(n / g, 2.0 / D);
}

int orc_lec_recover(double n, double A1z, double A1x, double D, double mu,
                    double *out)
{
    double p0z = A1z / n, p0x = A1x / n;
    double pz = p0z, px = p0x;
    int it, done = 0;
    for (it = 1; it <= 64; ++it) {
        double pm = sqrt(pz * pz + px * px);
        double uz = pz / sqrt(1.0 + pm * pm), ux = px / sqrt(1.0 + pm * pm);
        double g = 1.0 / sqrt(1.0 - (uz * uz + ux * ux));
        double h = lec_h(n, g, D, mu);
        double qz = p0z / h, qx = p0x / h;
        double dz = qz - pz, dx = qx - px;
        double qm = sqrt(qz * qz + qx * qx);
        pz = qz;
        px = qx;
        if (sqrt(dz * dz + dx * dx) <= 1e-15 * (1.0 + qm)) {
            done = 1;
            break;
        }
    }
    int iters = it;
    if (!done) {
        double P = sqrt(p0z * p0z + p0x * p0x), lo = 0.0, hi = P;
        for (int k = 0; k < 200 && hi - lo > 1e-17 * (1.0 + hi); ++k) {
            double mid = 0.5 * (lo + hi);
            double r = mid * lec_h(n, sqrt(1.0 + mid * mid), D, mu) - P;
            if (r > 0.0) hi = mid; else lo = mid;
        }
        double pm = 0.5 * (lo + hi);
        pz = P > 0.0 ? p0z * (pm / P) : 0.0;
        px = P > 0.0 ? p0x * (pm / P) : 0.0;
        iters = -iters;
    }
    double pm = sqrt(pz * pz + px * px);
    out[0] = pz / sqrt(1.0 + pm * pm);
    out[1] = px / sqrt(1.0 + pm * pm);
    out[2] = 1.0 / sqrt(1.0 - (out[0] * out[0] + out[1] * out[1]));
    out[3] = iters;
    return iters;
}

/* ---------------------------------------------------------------------- */
/* WARMC recovery (Sec. 4.1; App. A): lambda = n/h from the n lambda scalar,
 * u from n lambda u, theta^{ij} from lambda theta^{ij}; the time-like
 * components follow from U_nu theta^{mu nu} = 0 (eq. traces4, App. A):
 * theta^{0i} = u_j theta^{ij}, theta^{00} = u_i theta^{0i}. */
void orc_warmc_recover(int dims, const double *A, double *out)
{
    double n = A[0], nl = A[1];
    double lam = nl / n;
    double uz, ux, thzz, thxx, thyy, thxz, lamuz, lamux;
    if (dims == 1) {
        uz = A[W1_NLUZ] / nl;
        ux = 0.0;
        thzz = A[W1_THZZ] / lam;
        thxx = thyy = thxz = 0.0;
        lamuz = A[W1_NLUZ] / n;
        lamux = 0.0;
    } else {
        uz = A[W_NLUZ] / nl;
        ux = A[W_NLUX] / nl;
        thzz = A[W_THZZ] / lam;
        thxx = A[W_THXX] / lam;
        thyy = A[W_THYY] / lam;
        thxz = A[W_THXZ] / lam;
        lamuz = A[W_NLUZ] / n;
        lamux = A[W_NLUX] / n;
    }
    double th0z = ux * thxz + uz * thzz;
    double th0x = ux * thxx + uz * thxz;
    double th00 = ux * th0x + uz * th0z;
    out[0] = lam; out[1] = uz; out[2] = ux;
    out[3] = thzz; out[4] = thxx; out[5] = thyy; out[6] = thxz;
    out[7] = th0z; out[8] = th0x; out[9] = th00;
    out[10] = lamuz; out[11] = lamux;
}

/* Rest-frame longitudinal pressure (App. A, item 3, with r -> x, phi -> y). */
double orc_ppar(double thxx, double thyy, double thzz, double th00, double ux,
                double uz)
{
    double uu = ux * ux + uz * uz;
    return -(-(thxx + thzz) + th00 * uu + thyy * (1.0 + ux * ux)) / (1.0 + uz * uz);
}

/* lambda at rest from the trace condition (eq. traces3) with theta^{00} = 0
 * and D diagonal entries n mu: lambda - 1/lambda = D mu. */
double orc_lambda0(double mu, double D)
{
    return 0.5 * (D * mu + sqrt(D * D * mu * mu + 4.0));
}

/* ---------------------------------------------------------------------- */
static void recover_all(orc_state *s, const double *f, double *R)
{
    const int K = s->K, Q = s->Q, nc = s->ncell;
    const double D = s->p.dvel, mu = s->p.mu;
    long fb = 0;
#pragma omp parallel for reduction(+ : fb)
    for (int c = 0; c < nc; ++c) {
        double A[8];
        for (int k = 0; k < K; ++k) {         /* S1: A_k = sum_i f_{k,i} */
            double acc = 0.0;
            for (int q = 0; q < Q; ++q) acc += f[(k * Q + q) * nc + c];
            A[k] = acc;
        }
        double n = A[0];
        R[R_N * nc + c] = n;
        if (s->p.closure == ORC_LEC) {
            double o[4];
            double a1x = s->p.dims == 2 ? A[L_AX] : 0.0;
            orc_lec_recover(n, A[L_AZ], a1x, D, mu, o);
            if (o[3] < 0) fb++;
            double g = o[2], n0 = n / g;
            R[R_UZ * nc + c] = o[0];
            R[R_UX * nc + c] = o[1];
            R[R_GAM * nc + c] = g;
            R[R_N0 * nc + c] = n0;
            R[R_PHI * nc + c] = pow(n0, 1.0 + 2.0 / D); /* P0 / mu (Sec. 3) */
            R[R_ITER * nc + c] = o[3];
        } else {
            double o[12];
            orc_warmc_recover(s->p.dims, A, o);
            double uu = o[1] * o[1] + o[2] * o[2];
            double g = 1.0 / sqrt(1.0 - uu);
            R[R_UZ * nc + c] = o[1];
            R[R_UX * nc + c] = o[2];
            R[R_GAM * nc + c] = g;
            R[R_N0 * nc + c] = n / g;
            R[R_LAM * nc + c] = o[0];
            R[R_THZZ * nc + c] = o[3];
            R[R_THXX * nc + c] = o[4];
            R[R_THYY * nc + c] = o[5];
            R[R_THXZ * nc + c] = o[6];
            R[R_TH0Z * nc + c] = o[7];
            R[R_TH0X * nc + c] = o[8];
            R[R_TH00 * nc + c] = o[9];
            R[R_LUZ * nc + c] = o[10];
            R[R_LUX * nc + c] = o[11];
            R[R_PHI * nc + c] = 0.0;
            R[R_ITER * nc + c] = 0.0;
        }
    }
    s->fallbacks += fb;
}

/* S3: fields at the nodes at time level n. 2D: B^n = B^{n-1/2} - dt/2 curl E^n
 * on the Yee grid, then E averaged over 2 and B over 4 neighbours. */
static double curl_e(const orc_state *s, int j, int i)
{
    return ((EX_AT(j, i + 1) - EX_AT(j, i)) - (EZ_AT(j + 1, i) - EZ_AT(j, i))) / s->p.delta;
}

static void node_fields(orc_state *s)
{
    const int nz = s->nz, nx = s->nx;
    if (s->p.dims == 1) {
        for (int i = 0; i < nz; ++i) {
            s->En_z[i] = s->Ez[i];
            s->En_x[i] = 0.0;
            s->Bn_y[i] = 0.0;
        }
        return;
    }
    const double hd = 0.5 * s->p.dt;
#pragma omp parallel for
    for (int j = 0; j < nx; ++j)
        for (int i = 0; i < nz; ++i)
            s->Bh[j * nz + i] = s->By[j * nz + i] - hd * curl_e(s, j, i);
#pragma omp parallel for
    for (int j = 0; j < nx; ++j)
        for (int i = 0; i < nz; ++i) {
            int c = j * nz + i;
            s->En_z[c] = 0.5 * (EZ_AT(j, i - 1) + EZ_AT(j, i));
            if (s->p.geom == ORC_GEOM_AXI && j == 0) {
                /* E_r and B_phi are odd in r: zero on the axis (r_{-1/2} = 0) */
                s->En_x[c] = 0.5 * EX_AT(j, i);
                s->Bn_y[c] = 0.25 * (BY_AT(s->Bh, j, i) + BY_AT(s->Bh, j, i - 1));
            } else {
                s->En_x[c] = 0.5 * (EX_AT(j - 1, i) + EX_AT(j, i));
                s->Bn_y[c] = 0.25 * (BY_AT(s->Bh, j, i) + BY_AT(s->Bh, j, i - 1) +
                                     BY_AT(s->Bh, j - 1, i) + BY_AT(s->Bh, j - 1, i - 1));
            }
        }
}

/* Second-order central differences with the boundary rule of fixidx. */
static double ddz(const orc_state *s, const double *X, int j, int i)
{
    return (X[cell(s, j, i + 1)] - X[cell(s, j, i - 1)]) / (2.0 * s->p.delta);
}
static double ddx(const orc_state *s, const double *X, int j, int i)
{
    if (s->p.dims == 1) return 0.0;
    return (X[cell(s, j + 1, i)] - X[cell(s, j - 1, i)]) / (2.0 * s->p.delta);
}
/* Radial derivative of a quantity that changes sign under r -> -r: in the
 * axisymmetric geometry the row below the axis holds -X of row 0. */
static double ddx_odd(const orc_state *s, const double *X, int j, int i)
{
    if (s->p.geom == ORC_GEOM_AXI && j == 0)
        return (X[cell(s, 1, i)] + X[cell(s, 0, i)]) / (2.0 * s->p.delta);
    return ddx(s, X, j, i);
}

/* S5: forcing terms. */
static void forces(orc_state *s)
{
    const int nz = s->nz, nx = s->nx, nc = s->ncell, K = s->K;
    const double *R = s->R, mu = s->p.mu, dt = s->p.dt;
    double *F = s->F;
#define RR(q) (R + (q) * nc)
#pragma omp parallel for
    for (int j = 0; j < nx; ++j)
        for (int i = 0; i < nz; ++i) {
            int c = j * nz + i;
            double n = RR(R_N)[c], uz = RR(R_UZ)[c], ux = RR(R_UX)[c];
            double Ez = s->En_z[c], Ex = s->En_x[c], By = s->Bn_y[c];
            for (int k = 0; k < K; ++k) F[k * nc + c] = 0.0;
            if (s->p.closure == ORC_LEC) {
                /* eq. lb-ade-lec-comps-F with q = -1, n_i = 1:
                 * F = -mu grad (n/gamma)^{1+2/D} - n (E + u x B);
                 * (u x B)_z = u_x B_y, (u x B)_x = -u_z B_y (App. A, LEC). */
                F[L_AZ * nc + c] = -mu * ddz(s, RR(R_PHI), j, i) - n * (Ez + ux * By);
                if (s->p.dims == 2)
                    F[L_AX * nc + c] = -mu * ddx(s, RR(R_PHI), j, i) - n * (Ex - uz * By);
                if (s->p.geom == ORC_GEOM_AXI) {
                    /* App. A: the cylindrical part of the divergence, -u_r A / r,
                     * as a source of every advected scalar (x is r here) */
                    double ir = 1.0 / node_x(s, j);
                    double An = n, Az = 0.0, Ar = 0.0;
                    for (int q = 0; q < s->Q; ++q) {
                        Az += s->f[(L_AZ * s->Q + q) * nc + c];
                        Ar += s->f[(L_AX * s->Q + q) * nc + c];
                    }
                    F[0 * nc + c] -= ux * An * ir;
                    F[L_AZ * nc + c] -= ux * Az * ir;
                    F[L_AX * nc + c] -= ux * Ar * ir;
                }
            } else {
                /* eq. lb-ade-warmc-comps-F written out in App. A; Cartesian
                 * slab: the 1/r terms vanish, r -> x, phi -> y, c = e = 1.
                 * Time derivatives: backward difference against the lagged
                 * values (zero on the first step). */
                const double *G = s->lag;
                double th00 = RR(R_TH00)[c], th0z = RR(R_TH0Z)[c], th0x = RR(R_TH0X)[c];
                double thzz = RR(R_THZZ)[c], thxx = RR(R_THXX)[c], thxz = RR(R_THXZ)[c];
                double luz = RR(R_LUZ)[c], lux = RR(R_LUX)[c];
                double dt_th00 = (th00 - G[G_TH00 * nc + c]) / dt;
                double dt_th0z = (th0z - G[G_TH0Z * nc + c]) / dt;
                double dt_th0x = (th0x - G[G_TH0X * nc + c]) / dt;
                double dt_luz = (luz - G[G_LUZ * nc + c]) / dt;
                double dt_lux = (lux - G[G_LUX * nc + c]) / dt;
                /* theta^{0x}, theta^{xz} and lambda u_x are odd in x (r) */
                double dz_th0z = ddz(s, RR(R_TH0Z), j, i), dx_th0x = ddx_odd(s, RR(R_TH0X), j, i);
                double dz_thzz = ddz(s, RR(R_THZZ), j, i), dx_thxz = ddx_odd(s, RR(R_THXZ), j, i);
                double dz_thxz = ddz(s, RR(R_THXZ), j, i), dx_thxx = ddx(s, RR(R_THXX), j, i);
                double dz_luz = ddz(s, RR(R_LUZ), j, i), dx_luz = ddx(s, RR(R_LUZ), j, i);
                double dz_lux = ddz(s, RR(R_LUX), j, i), dx_lux = ddx_odd(s, RR(R_LUX), j, i);
                if (s->p.dims == 1) {
                    F[W1_NL * nc + c] = -dt_th00 - dz_th0z - n * (Ez * uz);
                    F[W1_NLUZ * nc + c] = -dt_th0z - dz_thzz - n * Ez;
                    F[W1_THZZ * nc + c] = -2.0 * th0z * dt_luz - 2.0 * thzz * dz_luz -
                                          2.0 * (Ez * th0z);
                } else {
                    F[W_NL * nc + c] = -dt_th00 - dx_th0x - dz_th0z - n * (Ex * ux + Ez * uz);
                    F[W_NLUX * nc + c] = -dt_th0x - dx_thxx - dz_thxz - n * (Ex - uz * By);
                    F[W_NLUZ * nc + c] = -dt_th0z - dx_thxz - dz_thzz - n * (Ez + ux * By);
                    F[W_THXX * nc + c] = -2.0 * th0x * dt_lux - 2.0 * thxx * dx_lux -
                                         2.0 * thxz * dz_lux - 2.0 * (Ex * th0x - By * thxz);
                    F[W_THYY * nc + c] = 0.0;
                    F[W_THZZ * nc + c] = -2.0 * th0z * dt_luz - 2.0 * thxz * dx_luz -
                                         2.0 * thzz * dz_luz - 2.0 * (Ez * th0z + By * thxz);
                    F[W_THXZ * nc + c] = -th0z * dt_lux - th0x * dt_luz - thxz * dx_lux -
                                         thxx * dx_luz - thzz * dz_lux - thxz * dz_luz -
                                         (Ex * th0z + Ez * th0x + By * (thxx - thzz));
                    if (s->p.geom == ORC_GEOM_AXI) {
                        /* App. A, WARMC: -u_r A / r for every advected scalar,
                         * the cylindrical parts of the divergences of theta^{0j}
                         * and theta^{ij} (-theta^{0r}/r, -(theta^{rr} -
                         * theta^{phiphi})/r, -theta^{rz}/r), and a total of
                         * -3 lambda theta^{phiphi} u_r / r for theta^{phiphi} */
                        double ir = 1.0 / node_x(s, j), A[8];
                        for (int k = 0; k < 8; ++k) {
                            A[k] = 0.0;
                            for (int q = 0; q < s->Q; ++q) A[k] += s->f[(k * s->Q + q) * nc + c];
                        }
                        double thyy = RR(R_THYY)[c];
                        F[W_N * nc + c] -= ux * A[W_N] * ir;
                        F[W_NL * nc + c] -= ux * A[W_NL] * ir + th0x * ir;
                        F[W_NLUZ * nc + c] -= ux * A[W_NLUZ] * ir + thxz * ir;
                        F[W_NLUX * nc + c] -= ux * A[W_NLUX] * ir + (thxx - thyy) * ir;
                        F[W_THZZ * nc + c] -= ux * A[W_THZZ] * ir;
                        F[W_THXX * nc + c] -= ux * A[W_THXX] * ir;
                        F[W_THYY * nc + c] -= 3.0 * ux * A[W_THYY] * ir;
                        F[W_THXZ * nc + c] -= ux * A[W_THXZ] * ir;
                    }
                }
            }
        }
#undef RR
}

/* S6 + S7: collide into fs, then stream (pull) into f. */
static void collide_stream(orc_state *s)
{
    const int K = s->K, Q = s->Q, nc = s->ncell, nz = s->nz, nx = s->nx;
    const double Lam = s->p.delta / s->p.dt, nu2 = Lam * Lam / 3.0;
    const double omega = 1.0 / s->p.tau_tilde, dt = s->p.dt;
    double *f = s->f, *fs = s->fs;
    const double *R = s->R, *F = s->F;
#pragma omp parallel for
    for (int c = 0; c < nc; ++c) {
        double uz = R[R_UZ * nc + c], ux = R[R_UX * nc + c];
        double uu = uz * uz + ux * ux;
        for (int k = 0; k < K; ++k) {
            double A = 0.0;
            for (int q = 0; q < Q; ++q) A += f[(k * Q + q) * nc + c];
            for (int q = 0; q < Q; ++q) {
                double uxi = Lam * (uz * s->ez[q] + (s->ex ? ux * s->ex[q] : 0.0));
                double fi = f[(k * Q + q) * nc + c];
                double fe = feq(s->w[q], A, uxi, uu, nu2);
                /* eq. lbe: f + dt (Omega + S), Omega = -(f - f_eq)/tau, S = w F */
                fs[(k * Q + q) * nc + c] = fi - omega * (fi - fe) + dt * s->w[q] * F[k * nc + c];
            }
        }
    }
    /* Streaming: f_i(x + xi_i dt) = f*_i(x), read as a pull from x - e_i.
     * Axisymmetric geometry: the axis lies midway between row 0 and the
     * ghost row -1, and the ghost holds the mirror image of row 0: the
     * populations of the mirrored direction (eq. reflective-bc), with the
     * sign reversed for the scalars that are odd under r -> -r (the radial
     * momentum A_r; n lambda u_r and lambda theta^{rz}). This is our reading of the axis rule of Sec. 2.2 for
     * this node layout: a plain copy (eq. open-bc) for the even scalars
     * would let mass cross the axis, which the cylindrical divergence of
     * App. A does not allow. */
    const int axi = s->p.geom == ORC_GEOM_AXI;
#pragma omp parallel for
    for (int j = 0; j < nx; ++j)
        for (int i = 0; i < nz; ++i) {
            int c = j * nz + i;
            for (int q = 0; q < Q; ++q) {
                int sj = j - (s->ex ? s->ex[q] : 0);
                int src = cell(s, sj, i - s->ez[q]);
                for (int k = 0; k < K; ++k) {
                    int qs = q;
                    double sg = 1.0;
                    if (axi && sj < 0) {
                        qs = s->mirror_x[q];
                        if (s->p.closure == ORC_LEC ? k == L_AX : (k == W_NLUX || k == W_THXZ)) sg = -1.0;
                    }
                    f[(k * Q + q) * nc + c] = sg * fs[(k * Q + qs) * nc + src];
                }
            }
        }
}

/* S9: Yee update with J^{n+1} = -n^{n+1} u^{n+1} (edge averages) and the
 * driver current -n_b z^ at t^{n+1/2}. */
static void maxwell(orc_state *s)
{
    const int nz = s->nz, nx = s->nx, nc = s->ncell;
    const double dt = s->p.dt, d = s->p.delta;
    const double th = (s->step + 0.5) * dt;
    const double *R1 = s->R1;
    if (s->p.dims == 1) {
        for (int i = 0; i < nz; ++i) {
            double jz = -R1[R_N * nc + i] * R1[R_UZ * nc + i];
            double jb = -orc_bunch(s, node_z(s, i), 0.0, th);
            s->Ez[i] = s->Ez[i] + dt * (-jz - jb);
        }
        return;
    }
    /* B^{n+1/2} = B^n - dt/2 curl E^n (B^n was formed in S3 from B^{n-1/2}). */
#pragma omp parallel for
    for (int j = 0; j < nx; ++j)
        for (int i = 0; i < nz; ++i)
            s->By[j * nz + i] = s->Bh[j * nz + i] - 0.5 * dt * curl_e(s, j, i);
    /* E^{n+1} = E^n + dt (curl B^{n+1/2} - J - J_b). */
#pragma omp parallel for
    for (int j = 0; j < nx; ++j)
        for (int i = 0; i < nz; ++i) {
            int c = j * nz + i;
            int cx = cell(s, j + 1, i), cz = cell(s, j, i + 1);
            double jx = 0.5 * (-R1[R_N * nc + c] * R1[R_UX * nc + c] -
                               R1[R_N * nc + cx] * R1[R_UX * nc + cx]);
            double jz = 0.5 * (-R1[R_N * nc + c] * R1[R_UZ * nc + c] -
                               R1[R_N * nc + cz] * R1[R_UZ * nc + cz]);
            double jb = -orc_bunch(s, node_z(s, i + 0.5), node_x(s, j), th);
            double curl_x = -(BY_AT(s->By, j, i) - BY_AT(s->By, j, i - 1)) / d;
            double curl_z = (BY_AT(s->By, j, i) - BY_AT(s->By, j - 1, i)) / d;
            if (s->p.geom == ORC_GEOM_AXI) {
                /* (1/r) d_r (r B_phi) at r_j = (j + 1/2) d from B_phi at
                 * r = (j + 1) d and j d (the latter on the axis for j = 0) */
                double bm = j > 0 ? BY_AT(s->By, j - 1, i) : 0.0;
                curl_z = ((j + 1.0) * BY_AT(s->By, j, i) - j * bm) / ((j + 0.5) * d);
            }
            s->Ex[c] = s->Ex[c] + dt * (curl_x - jx);
            s->Ez[c] = s->Ez[c] + dt * (curl_z - jz - jb);
        }
}

static void store_lag(orc_state *s, const double *R)
{
    const int nc = s->ncell;
    for (int c = 0; c < nc; ++c) {
        s->lag[G_TH00 * nc + c] = R[R_TH00 * nc + c];
        s->lag[G_TH0Z * nc + c] = R[R_TH0Z * nc + c];
        s->lag[G_TH0X * nc + c] = R[R_TH0X * nc + c];
        s->lag[G_LUZ * nc + c] = R[R_LUZ * nc + c];
        s->lag[G_LUX * nc + c] = R[R_LUX * nc + c];
    }
}

static void step_once(orc_state *s)
{
    recover_all(s, s->f, s->R);                    /* S1, S2 */
    if (s->p.closure == ORC_WARMC && !s->have_lag) { /* d/dt = 0 on step 0 */
        store_lag(s, s->R);
        s->have_lag = 1;
    }
    node_fields(s);                                /* S3 */
    forces(s);                                     /* S4, S5 */
    collide_stream(s);                             /* S6, S7 */
    recover_all(s, s->f, s->R1);                   /* S8 */
    maxwell(s);                                    /* S9 */
    if (s->p.closure == ORC_WARMC) store_lag(s, s->R); /* S10 */
    s->step++;
}

/* ---------------------------------------------------------------------- */
orc_state *orc_create(const orc_params *p)
{
    if (!p || (p->dims != 1 && p->dims != 2) || p->nz < 2 || p->nx < 1) return NULL;
    if (p->dims == 2 && p->nx < 2) return NULL;
    if (p->dims == 1 && p->nx != 1) return NULL;
    if (!(p->tau_tilde > 0.5) || !(p->dt > 0) || !(p->delta > 0)) return NULL;
    if (p->geom != ORC_GEOM_SLAB && p->geom != ORC_GEOM_AXI) return NULL;
    if (p->geom == ORC_GEOM_AXI &&
        (p->dims != 2 || p->bc_x != ORC_BC_OPEN || p->x0 != 0.0))
        return NULL;
    orc_state *s = (orc_state *)calloc(1, sizeof(orc_state));
    s->p = *p;
    if (p->nslices > 0) {
        s->slice_w = (double *)malloc(sizeof(double) * p->nslices);
        memcpy(s->slice_w, p->slice_w, sizeof(double) * p->nslices);
    }
    s->p.slice_w = s->slice_w;
    s->nz = p->nz;
    s->nx = p->nx;
    s->ncell = p->nz * p->nx;
    if (p->dims == 1) {
        s->Q = 3; s->ez = D1_ez; s->ex = NULL; s->w = D1_w;
        s->K = p->closure == ORC_LEC ? 2 : 4;
    } else {
        s->Q = 9; s->ez = D2_ez; s->ex = D2_ex; s->w = D2_w;
        for (int q = 0; q < 9; ++q)
            for (int m = 0; m < 9; ++m)
                if (D2_ez[m] == D2_ez[q] && D2_ex[m] == -D2_ex[q]) s->mirror_x[q] = m;
        s->K = p->closure == ORC_LEC ? 3 : 8;
    }
    size_t nc = (size_t)s->ncell;
    s->f = (double *)calloc(nc * s->K * s->Q, sizeof(double));
    s->fs = (double *)calloc(nc * s->K * s->Q, sizeof(double));
    s->Ez = (double *)calloc(nc, sizeof(double));
    s->Ex = (double *)calloc(nc, sizeof(double));
    s->By = (double *)calloc(nc, sizeof(double));
    s->Bh = (double *)calloc(nc, sizeof(double));
    s->En_z = (double *)calloc(nc, sizeof(double));
    s->En_x = (double *)calloc(nc, sizeof(double));
    s->Bn_y = (double *)calloc(nc, sizeof(double));
    s->A = (double *)calloc(nc * s->K, sizeof(double));
    s->R = (double *)calloc(nc * NR, sizeof(double));
    s->R1 = (double *)calloc(nc * NR, sizeof(double));
    s->F = (double *)calloc(nc * s->K, sizeof(double));
    s->lag = (double *)calloc(nc * NG, sizeof(double));
    s->nb = (double *)calloc(nc, sizeof(double));
    return s;
}

void orc_destroy(orc_state *s)
{
    if (!s) return;
    free(s->slice_w); free(s->f); free(s->fs); free(s->Ez); free(s->Ex);
    free(s->By); free(s->Bh); free(s->En_z); free(s->En_x); free(s->Bn_y);
    free(s->A); free(s->R); free(s->R1); free(s->F); free(s->lag); free(s->nb);
    free(s);
}

/* Initial state: equilibrium populations of the initial fluid (plasma at rest
 * unless a velocity field is given) and, when asked, the field of the bunch
 * alone. 1D: E_z(z) = integral of n_b from z to +infinity (causal, satisfies
 * Gauss's law). 2D: the vacuum solution travelling at c, E_z = 0,
 * E_x = -g(zeta) int_0^x exp(-x'^2/2 sigma_x^2) dx', B_y = E_x, with B_y taken
 * at t = -dt/2 (Sec. 5: fields initialised from the bunch alone). */
int orc_init(orc_state *s, const double *n_init, const double *uz_init,
             const double *ux_init, int fields_from_driver)
{
    const int nc = s->ncell, Q = s->Q, K = s->K, nz = s->nz, nx = s->nx;
    const double Lam = s->p.delta / s->p.dt, nu2 = Lam * Lam / 3.0;
    const double D = s->p.dvel, mu = s->p.mu;
    for (int c = 0; c < nc; ++c) {
        double n = n_init ? n_init[c] : 1.0;
        double uz = uz_init ? uz_init[c] : 0.0;
        double ux = (ux_init && s->p.dims == 2) ? ux_init[c] : 0.0;
        double uu = uz * uz + ux * ux;
        double A[8] = {0};
        A[0] = n;
        if (s->p.closure == ORC_LEC) {
            double g = 1.0 / sqrt(1.0 - uu);
            double h = lec_h(n, g, D, mu);
            A[L_AZ] = h * n * g * uz;
            if (s->p.dims == 2) A[L_AX] = h * n * g * ux;
        } else {
            /* Moving warm fluid: the rest state (theta_0 = diag(0, P, P, P) over
             * the D populated directions, P = n0 mu, lambda_0 from eq. traces3)
             * boosted to the lab (eq. double-boost): lambda = gamma lambda_0
             * since h is invariant and n = gamma n0. */
            double g = 1.0 / sqrt(1.0 - uu);
            double n0 = n / g, P = n0 * mu;
            double lam = g * orc_lambda0(mu, D);
            double v[3] = {ux, 0.0, uz};                 /* (x, y, z) */
            double p0[3] = {D >= 3.0 ? P : 0.0, D >= 3.0 ? P : 0.0, P};
            double L[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    L[a][b] = (a == b ? 1.0 : 0.0) + (uu > 0.0 ? (g - 1.0) * v[a] * v[b] / uu : 0.0);
            double th[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double acc = 0.0;
                    for (int m = 0; m < 3; ++m) acc += L[a][m] * L[b][m] * p0[m];
                    th[a][b] = acc;
                }
            if (s->p.dims == 1) {
                A[W1_NL] = n * lam;
                A[W1_NLUZ] = n * lam * uz;
                A[W1_THZZ] = lam * th[2][2];
            } else {
                A[W_NL] = n * lam;
                A[W_NLUZ] = n * lam * uz;
                A[W_NLUX] = n * lam * ux;
                A[W_THZZ] = lam * th[2][2];
                A[W_THXX] = lam * th[0][0];
                A[W_THYY] = lam * th[1][1];
                A[W_THXZ] = lam * th[0][2];
            }
        }
        for (int k = 0; k < K; ++k)
            for (int q = 0; q < Q; ++q) {
                double uxi = Lam * (uz * s->ez[q] + (s->ex ? ux * s->ex[q] : 0.0));
                s->f[(k * Q + q) * nc + c] = feq(s->w[q], A[k], uxi, uu, nu2);
            }
    }
    memset(s->Ez, 0, sizeof(double) * nc);
    memset(s->Ex, 0, sizeof(double) * nc);
    memset(s->By, 0, sizeof(double) * nc);
    memset(s->lag, 0, sizeof(double) * nc * NG);
    if (fields_from_driver && s->p.alpha != 0.0) {
        if (s->p.dims == 1) {
            for (int i = 0; i < nz; ++i)
                s->Ez[i] = s->p.alpha * bunch_tail_integral(s, node_z(s, i) - s->p.z0);
        } else {
            const double sx = s->p.sigma_x, sz = s->p.sigma_z;
            for (int j = 0; j < nx; ++j)
                for (int i = 0; i < nz; ++i) {
                    double xh = node_x(s, j + 0.5) - s->p.x0;
                    double tr = -sx * sqrt(M_PI / 2.0) * erf(xh / (sqrt(2.0) * sx));
                    if (s->p.geom == ORC_GEOM_AXI) /* Gauss in r: (1/r) d_r (r E_r) = -n_b */
                        tr = -sx * sx * (1.0 - exp(-xh * xh / (2.0 * sx * sx))) / xh;
                    double ze = node_z(s, i) - s->p.z0;
                    double zb = node_z(s, i + 0.5) - s->p.z0 + 0.5 * s->p.dt;
                    s->Ex[j * nz + i] = s->p.alpha * slice_weight(s, ze) *
                                        exp(-ze * ze / (2.0 * sz * sz)) * tr;
                    s->By[j * nz + i] = s->p.alpha * slice_weight(s, zb) *
                                        exp(-zb * zb / (2.0 * sz * sz)) * tr;
                }
        }
    }
    s->have_lag = 0;
    s->step = 0;
    s->fallbacks = 0;
    return 0;
}

int orc_init_moments(orc_state *s, const double *A, const double *uz,
                     const double *ux)
{
    const int nc = s->ncell, Q = s->Q, K = s->K;
    const double Lam = s->p.delta / s->p.dt, nu2 = Lam * Lam / 3.0;
    for (int c = 0; c < nc; ++c) {
        double vz = uz ? uz[c] : 0.0, vx = (ux && s->p.dims == 2) ? ux[c] : 0.0;
        double uu = vz * vz + vx * vx;
        for (int k = 0; k < K; ++k)
            for (int q = 0; q < Q; ++q) {
                double uxi = Lam * (vz * s->ez[q] + (s->ex ? vx * s->ex[q] : 0.0));
                s->f[(k * Q + q) * nc + c] = feq(s->w[q], A[k * nc + c], uxi, uu, nu2);
            }
    }
    memset(s->Ez, 0, sizeof(double) * nc);
    memset(s->Ex, 0, sizeof(double) * nc);
    memset(s->By, 0, sizeof(double) * nc);
    memset(s->lag, 0, sizeof(double) * nc * NG);
    s->have_lag = 0;
    s->step = 0;
    s->fallbacks = 0;
    return 0;
}

int orc_set_yee(orc_state *s, int which, const double *v)
{
    double *dst = which == 0 ? s->Ez : which == 1 ? s->Ex : which == 2 ? s->By : NULL;
    if (!dst) return -1;
    memcpy(dst, v, sizeof(double) * s->ncell);
    return 0;
}

int orc_num_scalars(const orc_state *s) { return s->K; }

int orc_ade_run(int dims, int nz, int nx, double delta, double dt, double tau_tilde,
                int bc, double uz, double ux, const double *A_in, int nsteps,
                double *A_out)
{
    orc_params p;
    memset(&p, 0, sizeof(p));
    p.dims = dims; p.nz = nz; p.nx = nx; p.delta = delta; p.dt = dt;
    p.tau_tilde = tau_tilde; p.closure = ORC_LEC; p.dvel = 1.0;
    p.bc_z = bc; p.bc_x = bc;
    orc_state *s = orc_create(&p);
    if (!s) return -1;
    /* one advected scalar: reuse the first population set only */
    s->K = 1;
    const int nc = s->ncell;
    double *uzv = (double *)malloc(sizeof(double) * nc);
    double *uxv = (double *)malloc(sizeof(double) * nc);
    for (int c = 0; c < nc; ++c) { uzv[c] = uz; uxv[c] = ux; }
    orc_init_moments(s, A_in, uzv, uxv);
    for (int t = 0; t < nsteps; ++t) {
        for (int c = 0; c < nc; ++c) {
            s->R[R_UZ * nc + c] = uz;
            s->R[R_UX * nc + c] = dims == 2 ? ux : 0.0;
            s->F[c] = 0.0;
        }
        collide_stream(s);
    }
    for (int c = 0; c < nc; ++c) {
        double acc = 0.0;
        for (int q = 0; q < s->Q; ++q) acc += s->f[q * nc + c];
        A_out[c] = acc;
    }
    free(uzv); free(uxv);
    orc_destroy(s);
    return 0;
}

int orc_step(orc_state *s, int nsteps)
{
    for (int t = 0; t < nsteps; ++t) step_once(s);
    return 0;
}

long orc_step_count(const orc_state *s) { return s->step; }

int orc_get(orc_state *s, int which, double *out)
{
    const int nc = s->ncell;
    if (which < 0 || which >= ORC_NOBS) return -1;
    if (which == ORC_EZ_YEE || which == ORC_EX_YEE || which == ORC_BY_YEE) {
        if (s->p.dims == 1) {
            memcpy(out, which == ORC_EZ_YEE ? s->Ez : which == ORC_EX_YEE ? s->Ex : s->By,
                   sizeof(double) * nc);
            return 0;
        }
        /* ghost slots of the open boundaries are reported as the copies they stand for */
        for (int j = 0; j < s->nx; ++j)
            for (int i = 0; i < s->nz; ++i)
                out[j * s->nz + i] = which == ORC_EZ_YEE ? EZ_AT(j, i)
                                   : which == ORC_EX_YEE ? EX_AT(j, i)
                                                         : BY_AT(s->By, j, i);
        return 0;
    }
    if (which == ORC_EZ || which == ORC_EX || which == ORC_BY) {
        node_fields(s);
        const double *src = which == ORC_EZ ? s->En_z : which == ORC_EX ? s->En_x : s->Bn_y;
        memcpy(out, src, sizeof(double) * nc);
        return 0;
    }
    long fb = s->fallbacks;
    recover_all(s, s->f, s->R1);
    s->fallbacks = fb;
    const double *R = s->R1;
    for (int c = 0; c < nc; ++c) {
        double v = 0.0;
        switch (which) {
        case ORC_N: v = R[R_N * nc + c]; break;
        case ORC_UZ: v = R[R_UZ * nc + c]; break;
        case ORC_UX: v = R[R_UX * nc + c]; break;
        case ORC_GAMMA: v = R[R_GAM * nc + c]; break;
        case ORC_N0: v = R[R_N0 * nc + c]; break;
        case ORC_P0:
            v = s->p.closure == ORC_LEC ? s->p.mu * R[R_PHI * nc + c] : R[R_THYY * nc + c];
            break;
        case ORC_LAMBDA: v = R[R_LAM * nc + c]; break;
        case ORC_THZZ: v = R[R_THZZ * nc + c]; break;
        case ORC_THXX: v = R[R_THXX * nc + c]; break;
        case ORC_THYY: v = R[R_THYY * nc + c]; break;
        case ORC_THXZ: v = R[R_THXZ * nc + c]; break;
        case ORC_PPAR:
            v = s->p.closure == ORC_LEC
                    ? s->p.mu * R[R_PHI * nc + c]
                    : orc_ppar(R[R_THXX * nc + c], R[R_THYY * nc + c], R[R_THZZ * nc + c],
                               R[R_TH00 * nc + c], R[R_UX * nc + c], R[R_UZ * nc + c]);
            break;
        case ORC_MZ: v = R[R_N * nc + c] * R[R_GAM * nc + c] * R[R_UZ * nc + c]; break;
        case ORC_MX: v = R[R_N * nc + c] * R[R_GAM * nc + c] * R[R_UX * nc + c]; break;
        default: v = 0.0;
        }
        out[c] = v;
    }
    return 0;
}

int orc_diagnostics(orc_state *s, double *out)
{
    const int nc = s->ncell, nz = s->nz, nx = s->nx;
    const double dV0 = s->p.dims == 1 ? s->p.delta : s->p.delta * s->p.delta;
    const int axi = s->p.geom == ORC_GEOM_AXI;
    const double Lam = s->p.delta / s->p.dt, t = s->step * s->p.dt, d = s->p.delta;
    long fb = s->fallbacks;
    recover_all(s, s->f, s->R1);
    s->fallbacks = fb;
    const double *R = s->R1;
    double sn = 0, fe = 0, ke = 0, g2 = 0, umax = 0, bad = 0;
    for (int j = 0; j < nx; ++j)
        for (int i = 0; i < nz; ++i) {
            int c = j * nz + i;
            double n = R[R_N * nc + c], uz = R[R_UZ * nc + c], ux = R[R_UX * nc + c];
            double g = R[R_GAM * nc + c];
            /* axisymmetric: volume 2 pi r per unit cell area, nodes at r_j,
             * E_r and B_phi at r_{j+1/2} */
            const double dV = axi ? 2.0 * M_PI * node_x(s, j) * dV0 : dV0;
            const double dVh = axi ? 2.0 * M_PI * node_x(s, j + 0.5) * dV0 : dV0;
            sn += n * dV;
            if (s->p.dims == 1) {
                fe += 0.5 * s->Ez[c] * s->Ez[c] * dV;
            } else {
                /* energy of the real Yee slots only */
                int rz = s->p.bc_z == ORC_BC_PERIODIC || i < nz - 1;
                int rx = s->p.bc_x == ORC_BC_PERIODIC || j < nx - 1;
                if (rz) fe += 0.5 * s->Ez[c] * s->Ez[c] * dV;
                if (rx) fe += 0.5 * s->Ex[c] * s->Ex[c] * dVh;
                if (rz && rx) fe += 0.5 * s->By[c] * s->By[c] * dVh;
            }
            ke += n * (g - 1.0) * dV;
            double um = sqrt(uz * uz + ux * ux) / Lam;
            if (um > umax) umax = um;
            double div;
            if (s->p.dims == 1) {
                div = (s->Ez[cell(s, j, i + 1)] - s->Ez[cell(s, j, i - 1)]) / (2.0 * d);
            } else {
                div = (EZ_AT(j, i) - EZ_AT(j, i - 1)) / d + (EX_AT(j, i) - EX_AT(j - 1, i)) / d;
                if (axi) {
                    double em = j > 0 ? EX_AT(j - 1, i) : 0.0;
                    div = (EZ_AT(j, i) - EZ_AT(j, i - 1)) / d +
                          ((j + 1.0) * EX_AT(j, i) - j * em) / ((j + 0.5) * d);
                }
            }
            double rho = 1.0 - n - orc_bunch(s, node_z(s, i), node_x(s, j), t);
            g2 += (div - rho) * (div - rho);
            if (!isfinite(n) || !isfinite(uz) || !isfinite(ux) || !isfinite(s->Ez[c]) ||
                !isfinite(s->Ex[c]) || !isfinite(s->By[c]))
                bad += 1;
        }
    out[0] = sn; out[1] = fe; out[2] = ke; out[3] = sqrt(g2 / nc);
    out[4] = umax; out[5] = bad; out[6] = (double)s->fallbacks; out[7] = (double)s->step;
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
