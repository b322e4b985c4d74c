/*
 * lbw_oracle.h -- plain FP64 CPU oracle of the moment-matching lattice
 * Boltzmann scheme for warm relativistic plasma wakes (Simeoni et al.,
 * arXiv 2309.04872).
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. It shares no code,
 * header, table or helper with the GPU library.
 *
 * Units: plasma units, c = m_e = e = 1, ion density n_i = 1, electrons carry
 * charge -1; time in 1/omega_p, length in 1/k_p, fields in m_e c omega_p / e.
 *
 * Grid: node (j, i) sits at z_i = i*delta, x_j = (j - (nx-1)/2)*delta
 * (axisymmetric geometry: r_j = (j + 1/2)*delta);
 * arrays are [nx][nz] with z fastest. In 2D the Yee arrays hold
 *   Ez[j][i] at (z_{i+1/2}, x_j), Ex[j][i] at (z_i, x_{j+1/2}),
 *   By[j][i] at (z_{i+1/2}, x_{j+1/2}).
 * In 1D, Ez[i] sits on the node.
 *
 * Canonical state after n steps: post-streaming populations f^n, E^n,
 * B^{n-1/2}, and (warm closure) the lagged values of step n-1.
 */
#ifndef LBW_ORACLE_H
#define LBW_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_LEC = 0, ORC_WARMC = 1 };
enum { ORC_BC_OPEN = 0, ORC_BC_PERIODIC = 1 };

/* Observables returned by orc_get (one value per node, [nx][nz]). */
enum {
    ORC_N = 0,      /* lab-frame electron density n */
    ORC_UZ = 1,     /* transport velocity u_z */
    ORC_UX = 2,     /* transport velocity u_x (0 in 1D) */
    ORC_GAMMA = 3,  /* Lorentz factor of u */
    ORC_N0 = 4,     /* rest-frame density n / gamma */
    ORC_P0 = 5,     /* LEC rest-frame pressure mu n0^{1+2/D}; WARMC: P_perp */
    ORC_LAMBDA = 6, /* WARMC lambda = n / h */
    ORC_THZZ = 7, ORC_THXX = 8, ORC_THYY = 9, ORC_THXZ = 10,
    ORC_PPAR = 11,  /* WARMC rest-frame longitudinal pressure */
    ORC_EZ = 12, ORC_EX = 13, ORC_BY = 14,  /* node-averaged E^n, B^n */
    ORC_EZ_YEE = 15, ORC_EX_YEE = 16, ORC_BY_YEE = 17, /* raw E^n, B^{n-1/2} */
    ORC_MZ = 18,    /* momentum density n*gamma*u_z */
    ORC_MX = 19,
    ORC_NOBS = 20
};

typedef struct {
    int dims;          /* 1 or 2 */
    int nz, nx;        /* nodes along z and x (nx = 1 in 1D) */
    double delta;      /* cell size */
    double dt;         /* time step */
    double tau_tilde;  /* relaxation time over dt, > 1/2 */
    int closure;       /* ORC_LEC or ORC_WARMC */
    double dvel;       /* D, dimension of kinetic momentum space (1 or 3) */
    int bc_z, bc_x;    /* ORC_BC_OPEN or ORC_BC_PERIODIC */
    double mu;         /* initial temperature k_B T_i / (m c^2) */
    /* rigid driver bunch moving at c along +z */
    double alpha, sigma_z, sigma_x, z0, x0;
    int nslices;           /* 0: plain Gaussian; else piecewise-constant slices */
    double slice_zmin, slice_zmax; /* slice span in zeta = z - z0 - t */
    const double *slice_w; /* nslices weights (copied) */
    /* ORC_GEOM_SLAB: Cartesian (z, x). ORC_GEOM_AXI: axisymmetric (z, r), the
     * 3D3V geometry of Sec. 2.2 and App. A (2D, either closure, bc_x open at
     * the outer radius; x0 must be 0; x, y read as r, phi). Node j sits at
     * r_j = (j + 1/2) delta; the ghost row j = -1 mirrors the axis. */
    int geom;
} orc_params;

enum { ORC_GEOM_SLAB = 0, ORC_GEOM_AXI = 1 };

typedef struct orc_state orc_state;

orc_state *orc_create(const orc_params *p);
void orc_destroy(orc_state *s);
/* n_init, uz_init, ux_init: nullable [nx][nz] arrays (default 1, 0, 0).
 * fields_from_driver: 1 = analytic bunch field at t = 0, 0 = zero fields. */
int orc_init(orc_state *s, const double *n_init, const double *uz_init,
             const double *ux_init, int fields_from_driver);
/* Initial populations f = f_eq(A_k, u) from arbitrary scalars A [K][nx][nz]
 * and velocity (nullable: 0); zero fields, no lag. */
int orc_init_moments(orc_state *s, const double *A, const double *uz,
                     const double *ux);
/* Overwrite a raw Yee array: 0 = E_z, 1 = E_x, 2 = B_y (B at t^{n-1/2}). */
int orc_set_yee(orc_state *s, int which, const double *v);
int orc_step(orc_state *s, int nsteps);
long orc_step_count(const orc_state *s);
int orc_get(orc_state *s, int which, double *out);
/* out[0..7]: sum n dV, field energy, kinetic energy sum n(gamma-1) dV,
 * rms Gauss residual, max |u| / (delta/dt), non-finite count,
 * recovery-fallback count, step. */
int orc_diagnostics(orc_state *s, double *out);
int orc_num_threads(void);
void orc_set_threads(int n);

/* Unit-level entry points (pins). */
void orc_feq(int dims, double A, double uz, double ux, double lattice_speed,
             double *out);
int orc_lec_recover(double n, double A1z, double A1x, double D, double mu,
                    double *out /* uz, ux, gamma, iterations */);
void orc_warmc_recover(int dims, const double *A, double *out
                       /* lambda, uz, ux, thzz, thxx, thyy, thxz,
                          th0z, th0x, th00, lam_uz, lam_ux */);
double orc_ppar(double thxx, double thyy, double thzz, double th00,
                double ux, double uz);
double orc_lambda0(double mu, double D);
double orc_bunch(const orc_state *s, double z, double x, double t);
/* Bare moment-matching advection-diffusion run for one scalar with constant
 * transport velocity and no forcing: A [nx][nz] in, A after nsteps out. */
int orc_ade_run(int dims, int nz, int nx, double delta, double dt, double tau_tilde,
                int bc, double uz, double ux, const double *A_in, int nsteps,
                double *A_out);
int orc_num_scalars(const orc_state *s);

#ifdef __cplusplus
}
#endif
#endif
