/*
 * lbwake.h -- C ABI of the MI355X library for the moment-matching lattice
 * Boltzmann (LB) scheme for warm relativistic plasma wakes of Simeoni et al.,
 * "Lattice Boltzmann method for warm fluid simulations of plasma wakefield
 * acceleration" (arXiv 2309.04872).
 *
 * The calls follow the paper's statement of the problem (Sec. 5): a plasma of
 * ion density n_i = 1 at initial temperature mu, a rigid bi-Gaussian driver
 * bunch moving at c (eq. bunch-density), a domain and resolution; initialise
 * the plasma and the driver, advance N time steps, read moments and fields.
 *
 * Units: plasma units, c = m_e = e = 1, n_i = 1, electrons carry charge -1;
 * time in 1/omega_p, length in 1/k_p, E in m_e c omega_p / e, B in E / c.
 *
 * Grid: node (j, i) sits at z_i = i*delta, x_j = (j - (nx-1)/2)*delta. Every
 * host array is [nx][nz] doubles with z fastest (nx = 1 in 1D). In 2D the
 * fields live on a Yee grid: E_z at (z_{i+1/2}, x_j), E_x at (z_i, x_{j+1/2}),
 * B_y at (z_{i+1/2}, x_{j+1/2}); with open boundaries the last half-integer
 * slot along a staggered direction is a copy ghost.
 *
 * One time step (Sec. 2.1 eq. lbe, Sec. 2.2, Sec. 3.1 / 4.1, Sec. 5):
 *   zeroth moments A_k = sum_i f_{k,i}; closure recovery of n, u (and theta);
 *   forcing F_k from gradients of the recovered fields and the Lorentz force
 *   of E^n, B^n; BGK relaxation toward the moment-matching equilibrium plus
 *   S_i = w_i F_k; streaming (open copy or periodic boundaries); Yee update of
 *   E, B with the plasma current -n u and the driver current -n_b z^.
 *
 * Ownership: the caller owns the device workspace (e.g. a torch tensor of
 * lbw_workspace_bytes() bytes) and the HIP stream, and keeps both alive for
 * the lifetime of the lbw_sim; the library never allocates device memory.
 * Host buffers passed in are read during the call only.
 *
 * Errors: every call returns an lbw_status; the message of the last failure
 * is available from lbw_last_error(). Calls on one lbw_sim are not
 * thread-safe; different lbw_sim objects on different streams are
 * independent.
 */
#ifndef LBWAKE_H
#define LBWAKE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The library is built with hidden visibility; the declarations below are
 * its exported interface. */
#pragma GCC visibility push(default)

typedef enum {
    LBW_OK = 0,
    LBW_ERR_ARG = -1,        /* invalid argument or size mismatch */
    LBW_ERR_WORKSPACE = -2,  /* workspace missing, too small or misaligned */
    LBW_ERR_HIP = -3,        /* a HIP call failed */
    LBW_ERR_UNSTABLE = -4,   /* tau~ <= 1/2 or Courant number too large */
    LBW_ERR_NONFINITE = -5,  /* NaN or Inf found in the state */
    LBW_ERR_STATE = -6,      /* call out of order (e.g. step before init) */
    LBW_ERR_UNSUPPORTED = -7 /* valid request the library does not implement */
} lbw_status;

typedef enum { LBW_LEC = 0, LBW_WARMC = 1 } lbw_closure;
/* Population storage: FP64; FP32 or FP16 deviations g = f - w_i A_ref from
 * the uniform rest state A_ref, with FP32 collision arithmetic and FP64
 * moment sums promoted from FP32 and FP64 closure recovery. */
typedef enum { LBW_FP64 = 0, LBW_FP32 = 1, LBW_FP16DEV = 2 } lbw_storage;
typedef enum { LBW_BC_OPEN = 0, LBW_BC_PERIODIC = 1 } lbw_bc;

/* Transverse geometry of a 2D grid. SLAB: Cartesian (z, x), node row j at
 * x_j = (j - (nx-1)/2) delta. AXI: the axisymmetric (z, r) geometry of
 * Sec. 2.2 and App. A (both closures, open outer radius): node row j at
 * r_j = (j + 1/2) delta, the cylindrical parts of the divergences as sources
 * (-u_r A / r for every advected scalar; for the warm closure also
 * -theta^{0r}/r, -(theta^{rr} - theta^{phiphi})/r, -theta^{rz}/r and the
 * theta^{phiphi} term of App. A), the E_z update with (1/r) d_r (r B_phi),
 * E_r and B_phi zero on the axis; below the axis the populations are the
 * mirror image of row 0 (mirrored directions, eq. reflective-bc, with the
 * scalars odd in r negated: A_r; n lambda u_r and lambda theta^{rz}). The x
 * arrays then run over r, the y components over phi. */
typedef enum { LBW_GEOM_SLAB = 0, LBW_GEOM_AXI = 1 } lbw_geom;

/* Fluid observables for lbw_read_moment (one value per node). */
typedef enum {
    LBW_N = 0,      /* lab-frame electron density n */
    LBW_UZ = 1,     /* transport velocity u_z */
    LBW_UX = 2,     /* transport velocity u_x (0 in 1D) */
    LBW_GAMMA = 3,  /* Lorentz factor of u */
    LBW_N0 = 4,     /* rest-frame density n / gamma */
    LBW_P0 = 5,     /* LEC: mu n0^{1+2/D}; WARMC: P_perp = theta^{yy} */
    LBW_LAMBDA = 6, /* WARMC lambda = n / h */
    LBW_THZZ = 7, LBW_THXX = 8, LBW_THYY = 9, LBW_THXZ = 10, /* WARMC theta */
    LBW_PPAR = 11,  /* rest-frame longitudinal pressure (LEC: = P0) */
    LBW_MZ = 12,    /* momentum density n gamma u_z */
    LBW_MX = 13,
    LBW_NMOMENTS = 14
} lbw_moment;

/* Fields for lbw_read_field. */
typedef enum {
    LBW_EZ = 0, LBW_EX = 1, LBW_BY = 2,
    LBW_WAKE_X = 3, /* transverse wakefield E_x - B_y (nodes only) */
    LBW_NFIELDS = 4
} lbw_field;

typedef struct {
    int dims;          /* 1 (D1Q3 stencil) or 2 (D2Q9 stencil, Yee TM fields) */
    int nz, nx;        /* nodes along z and x; nx = 1 in 1D */
    double delta;      /* cell size */
    double dt;         /* time step */
    double tau_tilde;  /* BGK relaxation time over dt, must exceed 1/2 */
    int closure;       /* lbw_closure */
    double dvel;       /* D, dimension of the kinetic momentum space: 1 or 3 */
    int storage;       /* lbw_storage */
    int bc_z, bc_x;    /* lbw_bc */
    int geom;          /* lbw_geom (2D; SLAB in 1D). Zero-initialise the
                          descriptor: 0 is the Cartesian slab */
} lbw_grid_desc;

typedef struct {
    double mu;             /* k_B T_i / (m c^2) */
    const double *n_init;  /* nullable [nx][nz] initial density (default 1) */
    const double *uz_init; /* nullable initial velocity u_z (default 0) */
    const double *ux_init; /* nullable initial velocity u_x (default 0) */
} lbw_plasma_desc;

typedef struct {
    double alpha;      /* peak bunch density n_b / n_i */
    double sigma_z;    /* rms length */
    double sigma_x;    /* rms width (ignored in 1D) */
    double z0, x0;     /* initial centre */
    int nslices;       /* 0: Gaussian; else piecewise-constant slice weights */
    const double *slice_w;         /* nslices weights (copied) */
    double slice_zmin, slice_zmax; /* slice span in zeta = z - z0 - t */
} lbw_driver_desc;

typedef struct lbw_sim lbw_sim;

/* Bytes of device workspace a simulation of this grid needs (0 if the
 * descriptor is invalid or unsupported, which includes grids of more than
 * 2e9 / 72 nodes: population offsets are 32-bit). The workspace must be
 * 256-byte aligned. */
size_t lbw_workspace_bytes(const lbw_grid_desc *grid);

/* Validate the grid (tau~ > 1/2, Courant dt <= delta / sqrt(dims)) and bind
 * the caller's workspace and stream (hipStream_t, NULL = default stream). */
lbw_status lbw_create(const lbw_grid_desc *grid, void *device_workspace,
                      size_t workspace_bytes, void *hip_stream, lbw_sim **out);

/* Plasma at equilibrium (Sec. 2: f_i = f_eq_i(A_k, u) of the initial fluid;
 * the warm closure starts from the boosted rest state, eq. traces3 and
 * eq. double-boost). Resets fields to zero, the driver to none and the step
 * counter to 0. Host arrays are [nx][nz]. */
lbw_status lbw_init_plasma(lbw_sim *sim, const lbw_plasma_desc *plasma);

/* Equilibrium populations of arbitrary advected scalars A[K][nx][nz]
 * (K = 2/4 in 1D, 3/8 in 2D for LEC/WARMC, in the order of the paper's
 * advected vectors) moving at u; fields zero; mu as given (>= 0, else
 * LBW_ERR_ARG). */
lbw_status lbw_init_moments(lbw_sim *sim, double mu, const double *A,
                            const double *uz, const double *ux);

/* Rigid driver (eq. bunch-density with rms widths). init_fields = 1 also sets
 * E, B to the field of the bunch alone at t = 0 (Sec. 5): 1D the causal
 * Gauss-consistent E_z, 2D the vacuum solution travelling at c (in the
 * axisymmetric geometry from the cylindrical Gauss law; there the bunch sits
 * on the axis, x0 = 0, else LBW_ERR_ARG). Setting the fields needs a
 * canonical state (LBW_ERR_STATE otherwise); a rejected call changes
 * nothing. */
lbw_status lbw_init_driver(lbw_sim *sim, const lbw_driver_desc *driver,
                           int init_fields);

/* Overwrite a raw Yee array (LBW_EZ, LBW_EX: E^n; LBW_BY: B^{n-1/2}). */
lbw_status lbw_set_field(lbw_sim *sim, int which, const double *host, size_t count);

/* Advance nsteps time steps (asynchronous on the stream unless the
 * non-finite check below is on). One step is the LB time step of Sec. 2.1
 * (eq. lbe: collision toward the moment-matching equilibrium of Sec. 2.2,
 * eq. ade-feq, with the source S_i = w_i F of eq. lsource; streaming with
 * eq. open-bc or periodic wrap) for every advected scalar of the closure
 * (Sec. 3.1 eq. lb-ade-lec-comps-A/F, Sec. 4.1 eq. lb-ade-warmc-comps-A/F,
 * App. A), with the forcing from the Lorentz force of the Yee fields and the
 * gradients of the recovered fluid variables, then the Yee update with the
 * plasma current -n u and the driver current -n_b z^ (Sec. 5). The call ends
 * on the canonical state (post-streaming populations f^n, E^n, B^{n-1/2}); a
 * series of calls equals one call of the summed length bit for bit. */
lbw_status lbw_step(lbw_sim *sim, int nsteps);

/* Optional non-finite check (0 = off, the default). With every = M > 0,
 * lbw_step runs in chunks that end on multiples of M steps (counted from
 * lbw_init_plasma); at the end of each such chunk the kernels that bring the
 * state to canonical form also test every node's advected scalars, velocity
 * and fields, and lbw_step returns LBW_ERR_NONFINITE (the state is then the
 * canonical state of that step, lbw_step_count tells which) as soon as one is
 * not finite. The check costs no extra pass over the state, but lbw_step
 * then synchronises the stream after each checked chunk. Results are the
 * same bits as without the check. The paper's only stability statement is
 * tau~ > 1/2 (Sec. 2.2, eq. diff-coeff); the check catches the rest. */
lbw_status lbw_set_nonfinite_check(lbw_sim *sim, int every);

/* Diagnostics every M steps (the reductions of lbw_diagnostics: FP64
 * wavefront and workgroup sums, Sec. 2.2 moments and the Sec. 5 fields):
 * with every = M > 0, lbw_step also ends its chunks on multiples of M steps
 * (counted from lbw_init_plasma) and after each writes the 8 values of
 * lbw_diagnostics for that step into the next row of device_series
 * (caller-owned device memory, capacity rows of 8 doubles), asynchronously
 * on the simulation's stream, without copies to the host or
 * synchronisation. Rows beyond capacity are counted but not written;
 * lbw_diagnostics_rows tells how many rows were due since the call.
 * every = 0 turns recording off (the default). Results of the steps are the
 * same bits as without recording. The buffer must stay valid while
 * recording is on. LBW_ERR_ARG for negative arguments or for every > 0
 * without a buffer of at least one row. */
lbw_status lbw_set_diagnostics_every(lbw_sim *sim, int every, double *device_series, long capacity);
long lbw_diagnostics_rows(const lbw_sim *sim);

/* Recover one fluid observable at every node into host_out (count =
 * nx*nz doubles); synchronises the stream. The observables come from the
 * zeroth moments of the canonical populations (eq. disc-moments-ade) by the
 * closure's recovery: LEC, the fixed point of Sec. 3.1 for |p| with
 * n0 = n / gamma and P0 = mu n0^{1+2/D} (eq. temp-scaling); WARMC, the
 * algebra of Sec. 4.1 and App. A (lambda = n / h, theta^{0i}, theta^{00}
 * from eq. traces4, P_par by the double boost of eq. double-boost). */
lbw_status lbw_read_moment(lbw_sim *sim, int which, double *host_out, size_t count);

/* Same into a device buffer of nx*nz doubles, asynchronous on the stream. */
lbw_status lbw_read_moment_device(lbw_sim *sim, int which, double *device_out);

/* Fields of the Yee FDTD update (Sec. 5): at_nodes = 1 gives node averages
 * of E^n and B^n = B^{n-1/2} - dt/2 curl E^n (E over 2, B over 4 slots) and
 * the transverse wakefield E_x - B_y of the paper's wake plots; at_nodes = 0
 * the raw Yee arrays E^n, B^{n-1/2} (ghost slots reported as their copies).
 * count = nx*nz doubles; synchronises the stream. */
lbw_status lbw_read_field(lbw_sim *sim, int which, int at_nodes, double *host_out,
                          size_t count);

/* out[8]: sum n dV; field energy; kinetic energy sum n (gamma - 1) dV; rms
 * Gauss residual div E - (1 - n - n_b); max |u| / (delta / dt); number of
 * non-finite nodes; LEC recovery fallbacks so far; step count. Reductions in
 * FP64. Returns LBW_ERR_NONFINITE when out[5] > 0. */
lbw_status lbw_diagnostics(lbw_sim *sim, double *out);

/* For callers that cannot allocate device memory or synchronise (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * lbw_diagnostics with its scratch (the per-workgroup partial sums and
 * totals of the reduction) in a static device array of the library instead
 * of the simulation's workspace, 1 MiB per GPU, held until the process ends.
 * Writes the same 8 values to device_out (caller-owned device memory, 8
 * doubles), asynchronously on the simulation's stream, and neither
 * allocates, copies to the host nor synchronises; out[5] > 0 reports
 * non-finite nodes (no LBW_ERR_NONFINITE here). Grids of more than
 * 5 586 944 nodes return LBW_ERR_UNSUPPORTED. All calls on one GPU share its
 * array: calls that overlap on one GPU (different streams or threads) race;
 * calls in one stream's order do not. Nothing in the array needs clearing
 * between calls. */
lbw_status lbw_diagnostics_static(lbw_sim *sim, double *device_out);

long lbw_step_count(const lbw_sim *sim);

/* Kernel timing: while enabled, lbw_step brackets its back-to-back fused
 * step launches (not the closing canonicalisation) with a pair of HIP events
 * on the simulation's stream; lbw_get_timing returns the summed time (ms) of
 * those batches and the number of fused launches since the last enable (it
 * synchronises the stream). Off by default. */
lbw_status lbw_set_timing(lbw_sim *sim, int enable);
lbw_status lbw_get_timing(lbw_sim *sim, double *kernel_ms, long *launches);

/* Checkpoint: populations, fields, lagged values, step counter. The host
 * format starts with the tag "LBWSTAT2" (populations in the grouped layout of
 * this library version); lbw_load_state refuses a buffer with another tag,
 * a different grid, closure or storage, or fewer than lbw_state_bytes bytes
 * (LBW_ERR_ARG). */
size_t lbw_state_bytes(const lbw_sim *sim);
lbw_status lbw_save_state(lbw_sim *sim, void *host, size_t bytes);
/* The same checkpoint without waiting: the header is written at once, the
 * device parts are copied on the simulation's stream, after the work queued
 * there and before the work queued later (steps may be queued at once). The
 * caller synchronises the stream (or an event recorded on it) before reading
 * the buffer, which must stay valid until then; pinned host memory
 * (hipHostMalloc, torch pin_memory) lets the copies overlap the steps. */
lbw_status lbw_save_state_async(lbw_sim *sim, void *host, size_t bytes);
lbw_status lbw_load_state(lbw_sim *sim, const void *host, size_t bytes);

/* ---------------------------------------------------------------------------
 * Device-side checkpoints of the canonical state (f^n, E^n, B^{n-1/2} and the
 * warm closure's lagged values) for checkpoint-and-recompute. The buffer is
 * caller-owned device memory, 256-byte aligned, of lbw_state_device_bytes();
 * layout: the populations (storage type), then E_z, E_x, B_y (FP64), then the
 * lagged values, each part starting on a 256-byte boundary. The populations
 * are those of the library's buffers: over nc = nz nx nodes (node j nz + z),
 * the K scalars in groups of G, the largest power of two that neither
 * exceeds K nor makes a group longer than 16 bytes (FP64 2; FP32 4, or 2 for
 * K = 3; FP16 8 for K = 8, 4 for K = 4, 2 for K = 2 or 3), population (k, q) of
 * node c at element ((k / G) Q + q) nc G + c G + k % G for k < K - K % G,
 * and a leftover scalar (k >= K - K % G) at (K - K % G) Q nc
 * + ((k - K + K % G) Q + q) nc + c. Both calls are
 * asynchronous on the simulation's stream. lbw_load_state_device restores a
 * state saved from a simulation with the same descriptor and plasma (it
 * keeps the current mu, storage reference and driver) and sets the step
 * counter to step. */
size_t lbw_state_device_bytes(const lbw_sim *sim);
lbw_status lbw_save_state_device(lbw_sim *sim, void *device_dst);
lbw_status lbw_load_state_device(lbw_sim *sim, const void *device_src, long step);

/* Advance nsteps steps one at a time and record the canonical state after
 * each: the state after step m (m = 1 .. nsteps of this call) goes to
 * device_states + (m - 1) * stride, in the layout above (caller-owned device
 * memory; stride a multiple of 256 and at least lbw_state_device_bytes()).
 * The records and the simulation's final state equal those of nsteps calls of
 * lbw_step(sim, 1), each followed by lbw_save_state_device, bit for bit: each
 * step's closing canonicalisation (streaming and field completion, Sec. 2.1
 * and Sec. 5) writes its record directly and the next step reads it, so no
 * state is copied. For checkpoint-and-recompute. Asynchronous on the stream;
 * not included in lbw_set_timing's kernel timing, and without the optional
 * non-finite checks and diagnostics records of lbw_step. */
lbw_status lbw_step_record(lbw_sim *sim, int nsteps, void *device_states, size_t stride);

/* The same steps as lbw_step(sim, nsteps) from a canonical state at step n0,
 * recording each fused launch's own output instead of a canonical state:
 * record m (m = 0 .. nsteps - 1, at device_states + m * stride, same layout
 * and stride rules) holds the post-collision populations f*^{n0+m} of step
 * n0 + m (Sec. 2.2, before the streaming of Sec. 2.1) and the fields
 * E^{n0+m}, B^{n0+m-1/2} of state n0 + m (its lagged-value part is not
 * written). Each launch reads the previous record, and only the last is
 * canonicalised, into the simulation, whose final state equals that of
 * lbw_step(sim, nsteps) bit for bit. For the recompute of
 * lbw_adjoint_step_post; asynchronous on the stream, without lbw_step's
 * optional non-finite checks, diagnostics records and kernel timing. */
lbw_status lbw_step_record_post(lbw_sim *sim, int nsteps, void *device_states, size_t stride);

/* ---------------------------------------------------------------------------
 * Discrete adjoint of the 2D local-equilibrium step (Sec. 2.2, Sec. 3.1,
 * Sec. 5): the transposed Jacobian of one step of lbw_step, and the
 * derivatives of the driver's slice weights (per-slice current profile) in
 * the bunch current and in the initial fields. 2D slab, LBW_LEC, any storage
 * (the adjoint itself is FP64), any slice count lbw_init_driver accepts; LBW_ERR_UNSUPPORTED
 * otherwise, LBW_ERR_STATE when the driver has no slices.
 *
 * adj (device, FP64, caller-owned, 16-byte aligned) holds the adjoint of a
 * canonical state: its K*Q*nx*nz populations in the layout of the FP64
 * population buffers (the device checkpoints above), then E_z, E_x, B_y, each
 * nx*nz values; lbw_adjoint_bytes() bytes. scratch: lbw_adjoint_workspace_bytes()
 * bytes of device memory, 256-byte aligned. grad: nslices FP64 values on the
 * device, accumulated into (the caller zeroes it).
 *
 * lbw_adjoint_step: given the saved states at steps n and n+1
 * (lbw_save_state_device) and the adjoint of state n+1 in adj, overwrite adj
 * with the adjoint of state n and add the step's slice derivatives to grad.
 * lbw_adjoint_init_fields: with adj the adjoint of state 0, add the slice
 * derivatives of the initial fields (lbw_init_driver with init_fields).
 * Both are asynchronous on the simulation's stream. */
size_t lbw_adjoint_bytes(const lbw_sim *sim);
size_t lbw_adjoint_workspace_bytes(const lbw_sim *sim);
lbw_status lbw_adjoint_step(lbw_sim *sim, const void *state_n, const void *state_n1, long n, double *adj,
                            double *grad, void *scratch);
/* lbw_adjoint_step for records of lbw_step_record_post: rec_n is the record
 * of step n (post-collision f*^n, whose streaming gives state n+1's
 * populations, and state n's fields); pops_n holds state n's populations,
 * canonical (pops_n_post = 0, e.g. the checkpoint the records start from)
 * or as the record of step n - 1 (pops_n_post = 1). The kernels stream
 * those populations themselves while summing their moments; the result is
 * bit for bit that of lbw_adjoint_step on the canonical states. */
lbw_status lbw_adjoint_step_post(lbw_sim *sim, const void *pops_n, int pops_n_post, const void *rec_n, long n,
                                 double *adj, double *grad, void *scratch);
lbw_status lbw_adjoint_init_fields(lbw_sim *sim, const double *adj, double *grad, void *scratch);

/* ---------------------------------------------------------------------------
 * Batched 1D parameter scans (one launch for many independent 1D runs).
 *
 * A batch holds ninst independent 1D simulations ("instances") of their own
 * length, closure, temperature, time step and driver, all with FP64
 * populations on the D1Q3 stencil. Each instance follows exactly the 1D step
 * of lbw_step (Sec. 2.1-2.2 streaming and collision, Sec. 3.1 / Sec. 4.1
 * recoveries and forces, Sec. 5 field update and driver); the instances only
 * share the launch. lbw_batch_step runs all requested steps of every
 * instance inside one persistent kernel launch: by default one workgroup
 * owns one instance for the whole launch and advances it in passes separated
 * by workgroup barriers (after the first step, passes of 16 steps and then
 * pairs of steps, the state read and written once per pass), so no instance
 * ever waits on another and the launch needs no co-residency; the split
 * schedule (lbw_batch_set_schedule) shares long instances among several
 * co-resident workgroups. Workgroups take instances longest first.
 *
 * The workspace is caller-owned device memory (256-byte aligned) of at least
 * lbw_batch_workspace_bytes(); the library allocates no device memory. It
 * holds, per instance, two population buffers (K x 3 planes of the padded
 * length, K = 2 for LEC and 4 for WARMC), two E_z buffers, two sets of the
 * warm closure's three lagged values, a snapshot of the state used by the
 * autotuner, and the instance's parameters, step counter and non-finite
 * count.
 * ------------------------------------------------------------------------- */
typedef struct {
    int nz;            /* nodes, >= 4 */
    int closure;       /* lbw_closure */
    double dvel;       /* D: velocity dimensions of the closure (eq. temp-scaling, eq. traces3) */
    double mu;         /* k_B T / (m c^2) of the uniform plasma, >= 0 */
    double delta;      /* grid spacing in units of c / omega_p */
    double dt;         /* time step, 0 < dt <= delta */
    double tau_tilde;  /* dimensionless relaxation time, > 1/2 */
    int bc;            /* lbw_bc along z */
    double alpha;      /* driver peak density n_b / n_0 (0: no driver) */
    double sigma_z;    /* driver rms length, > 0 when alpha != 0 */
    double z0;         /* driver centre at t = 0 */
} lbw_instance_desc;

/* E_z (on the nodes, as lbw_read_field gives it in 1D) for lbw_batch_read. */
#define LBW_BATCH_EZ 100

typedef struct lbw_batch lbw_batch;

/* Workspace bytes for this set of instances; 0 if a descriptor is invalid. */
size_t lbw_batch_workspace_bytes(const lbw_instance_desc *inst, int ninst);
/* Validates the descriptors (as lbw_create), copies them to the device and
 * returns a handle. Returns LBW_ERR_ARG for an invalid descriptor or
 * ninst outside [1, 65536], LBW_ERR_UNSTABLE for tau_tilde <= 1/2 or
 * dt > delta, LBW_ERR_WORKSPACE for a short or misaligned workspace. */
lbw_status lbw_batch_create(const lbw_instance_desc *inst, int ninst, void *device_workspace,
                            size_t workspace_bytes, void *hip_stream, lbw_batch **out);
/* Every instance to the uniform plasma at rest at its temperature with the
 * causal field of its driver (as lbw_init_plasma + lbw_init_driver with
 * init_fields = 1). n_init (host, nullable): the densities of all instances
 * concatenated in instance order (sum of nz values), positive and finite.
 * Synchronises the stream. */
lbw_status lbw_batch_init(lbw_batch *b, const double *n_init);
/* Advance every instance by nsteps steps in one persistent kernel launch,
 * ending on the canonical state (f^n, E^n). use_graph = 1 launches it from a
 * HIP graph captured on first use for this (nsteps, configuration). Returns
 * without synchronising. */
lbw_status lbw_batch_step(lbw_batch *b, int nsteps, int use_graph);
/* Launch configuration of the persistent kernel with one workgroup per
 * instance: threads per workgroup and nodes per thread per pass, one of
 * (256, 1), (256, 2), (512, 1), (512, 2), (1024, 1); the default is
 * (1024, 1). LBW_ERR_ARG for any other pair. get_config reports the shape of
 * the current configuration, whatever its schedule. */
lbw_status lbw_batch_set_config(lbw_batch *b, int threads, int nodes_per_thread);
lbw_status lbw_batch_get_config(const lbw_batch *b, int *threads, int *nodes_per_thread);
/* Schedule of the launch. split = 0: one workgroup per instance (as
 * lbw_batch_set_config), so the launch is bound by the longest instance.
 * split = 1, for the shapes (256, 2), (512, 1), (512, 2), (1024, 1): as many
 * workgroups as the occupancy query proves co-resident (a cooperative
 * launch); instance i gets ceil(tiles_i / L) of them for the smallest L that
 * fits (tiles_i: tiles of its deep passes), they take contiguous runs of
 * every sweep's tiles and meet at a barrier of their own after each sweep
 * (the only waits between workgroups, safe because all are resident).
 * Results are the same bits under every schedule. LBW_ERR_UNSUPPORTED when
 * fewer workgroups than instances can be resident or the device has no
 * cooperative launch. get_schedule also returns the workgroups a launch
 * uses. */
lbw_status lbw_batch_set_schedule(lbw_batch *b, int threads, int nodes_per_thread, int split);
lbw_status lbw_batch_get_schedule(const lbw_batch *b, int *threads, int *nodes_per_thread, int *split,
                                  int *workgroups);
/* Autotuner: runs probe_steps steps under every configuration (shape and
 * schedule) the device can launch, from the same state (snapshot and
 * restore inside the workspace), keeps the fastest and returns its shape
 * (lbw_batch_get_schedule tells its schedule). The state afterwards is
 * bit-for-bit the state before. Synchronises the stream. */
lbw_status lbw_batch_autotune(lbw_batch *b, int probe_steps, int *threads, int *nodes_per_thread);
/* One observable of instance inst into host_out (count = that instance's
 * nz): an lbw_moment, or LBW_BATCH_EZ. Synchronises the stream. */
lbw_status lbw_batch_read(lbw_batch *b, int inst, int which, double *host_out, size_t count);
/* Per instance, the number of nodes whose density, velocity or E_z was not
 * finite at the end of the last lbw_batch_step (ninst ints, host).
 * Synchronises the stream. */
lbw_status lbw_batch_nonfinite(lbw_batch *b, int *counts);
/* Steps taken since lbw_batch_init (the same for every instance). */
long lbw_batch_step_count(const lbw_batch *b);
/* Duration in ms of the last lbw_batch_step launch (HIP events on the
 * batch's stream around it). Synchronises on the end event. */
lbw_status lbw_batch_get_timing(lbw_batch *b, double *ms_last_step);
const char *lbw_batch_last_error(const lbw_batch *b);
void lbw_batch_destroy(lbw_batch *b);

const char *lbw_last_error(const lbw_sim *sim);
const char *lbw_version(void);

/* Measurement aid, not a step of the method: copies bytes bytes from src to
 * dst (device pointers, 16-byte aligned, not overlapping; bytes a multiple
 * of 16) on stream (a hipStream_t; NULL: the null stream) with a plain
 * streaming kernel, one 16-byte non-temporal load and store per thread in
 * 256-thread workgroups. Read plus write bytes over its duration is the HBM
 * rate that a simple kernel sustains on the device, the practical ceiling
 * beside the nominal peak. Asynchronous. LBW_ERR_ARG for a NULL pointer,
 * misalignment, overlap or a size not a multiple of 16 (checked on the host,
 * before any launch), LBW_ERR_HIP if the launch fails. */
lbw_status lbw_stream_copy(void *dst, const void *src, size_t bytes, void *stream);

/* Releases the handle; the workspace and stream stay the caller's. */
void lbw_destroy(lbw_sim *sim);

#pragma GCC visibility pop

#ifdef __cplusplus
}
#endif
#endif
