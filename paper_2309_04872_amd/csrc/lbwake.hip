// lbwake.hip -- host side of the C ABI declared in include/lbwake.h: workspace
// layout, argument checks, launch sequencing on the caller's stream. The hot
// path is the fused step kernel of lbw_kernels.hpp; everything here is
// bookkeeping around it.
#include "../../include/lbwake.h"
#include "lbw_kernels.hpp"
#include "lbw_adjoint.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

using namespace lbw;

namespace {

// Tile shapes (nodes along z x x per workgroup) and nodes per thread of the 2D
// step, per closure and storage; the build may override them for sweeps.
#ifndef LBW_TZ2
#define LBW_TZ2 64
#endif
#ifndef LBW_TX2
#define LBW_TX2 16
#endif
#ifndef LBW_CPT2
#define LBW_CPT2 1
#endif
#ifndef LBW_TZ2_F64
#define LBW_TZ2_F64 64
#endif
#ifndef LBW_TX2_F64
#define LBW_TX2_F64 4
#endif
#ifndef LBW_TZ2_W
#define LBW_TZ2_W 64
#endif
#ifndef LBW_TX2_W
#define LBW_TX2_W 4
#endif
#ifndef LBW_TZ2_WF64
#define LBW_TZ2_WF64 64
#endif
#ifndef LBW_TX2_WF64
#define LBW_TX2_WF64 4
#endif
#ifndef LBW_STRIP_WF64
#define LBW_STRIP_WF64 6
#endif
#ifndef LBW_TZ2_S
#define LBW_TZ2_S 64
#endif
#ifndef LBW_TX2_S
#define LBW_TX2_S 8
#endif
#ifndef LBW_TZ1
#define LBW_TZ1 256
#endif
template <int CL, class ST> struct Tile2 {  // local-equilibrium, FP32 / FP16 storage
    static constexpr int TZ = LBW_TZ2, TX = LBW_TX2, CPT = LBW_CPT2, STRIP = 1;
};
// Local equilibrium, FP32 / FP16 storage, second shape: 512-thread workgroups,
// two per compute unit, so that one workgroup's loads overlap the other's
// recovery, field update and collision. The 1024-thread 64 x 16 tile has the
// smaller recovery ring (16 % of the tile instead of 29 %) and wins while the
// populations sit largely in the 256 MB last-level cache; once the grid
// streams from HBM the overlap wins (3000 x 600: 151 -> 143 us FP32,
// 108 -> 97 us FP16; 4096 x 1024: 321 -> 298 us, 248 -> 228 us), and for FP16
// it wins at 2048 x 512 too (52.1 -> 46.8 us; FP32 66.8 -> 69.5 us there).
struct Tile2Stream {
    static constexpr int TZ = LBW_TZ2_S, TX = LBW_TX2_S, CPT = 1, STRIP = 1;
};
constexpr size_t MALL_BYTES = size_t(256) << 20;
template <> struct Tile2<LEC, double> {
    static constexpr int TZ = LBW_TZ2_F64, TX = LBW_TX2_F64, CPT = 1, STRIP = 1;
};
// Warm closure, FP32 / FP16-deviation storage: 64 x 4 tiles in strips of 3
// tile-rows (4096 x 1024: FP32 684.5 -> 669.6 and 686.1 -> 670.9 us, FP16
// 492.6 -> 484.7 and 493.3 -> 485.4 us on two boxes; axisymmetric 3000 x 600
// FP32 357.4 -> 352.8 us; strips of 4, 6, 12 measured equal or slower).
template <class ST> struct Tile2<WARMC, ST> {
    static constexpr int TZ = LBW_TZ2_W, TX = LBW_TX2_W, CPT = 1, STRIP = 3;
};
// Warm closure, FP64, slab: 64 x 4 tiles in strips of 6 tile-rows. Swept on
// 4096 x 1024 (us per step): 32 x 8 in strips of 1, 2, 3, 4, 5, 6, 8, 12, 16:
// 1310, 1255, 1222, 1255, 1243, 1231, 1333, 1309, 1272; 64 x 4 in strips of 4 to
// 14, 20, 24, 32: 1258, 1204 (5), 1190 (6), 1242 (7), 1234-1241 (8), 1294 (9),
// 1214 (10), 1209 (11), 1193-1199 (12), 1246 (13), 1212 (14), 1238, 1276, 1245;
// 128 x 2 in strips of 8 or 16: 1324. The fused kernel streams its 72 planes at
// the rate a plain multi-plane copy reaches, so the order that keeps a tile's
// ring rows and columns in L2 is what is left, and it does not vary smoothly
// with the strip height.
template <> struct Tile2<WARMC, double> {
    static constexpr int TZ = LBW_TZ2_WF64, TX = LBW_TX2_WF64, CPT = 1, STRIP = LBW_STRIP_WF64;
};
// Warm closure, FP64, axisymmetric geometry: 64 x 4 (the paper's 3000 x 600
// grid: 573 us per step against 605 us with 32 x 8; both 256 threads and two
// waves per SIMD, the slab 4096 x 1024 grid the other way round, 1355 / 1305).
struct Tile2WarmAxi64 {
    static constexpr int TZ = LBW_TZ2_W, TX = LBW_TX2_W, CPT = 1, STRIP = 1;
};
constexpr int TZ1 = LBW_TZ1;  // 1D tile, one launch per step
constexpr int TZP_SMALL = 192, TZP_LARGE = 256;  // 1D tiles of the persistent kernel
constexpr int MAX_SLICES = 4096;
constexpr size_t ALIGN = 256;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

int nscalars(int dims, int closure) { return closure == LBW_LEC ? 1 + dims : (dims == 1 ? 4 : 8); }
int nlag(int dims, int closure) { return closure == LBW_WARMC ? (dims == 1 ? NLAG1 : NLAG2) : 0; }
size_t storage_size(int storage) { return storage == LBW_FP64 ? 8 : (storage == LBW_FP32 ? 4 : 2); }

struct Layout {
    size_t pop[2], fld[2][3], lag, lag_alt, stage, part, aref, slice, fallbacks, nonfinite, diag, total;
    int K, Q, nblk_diag;
};

bool grid_valid(const lbw_grid_desc *g, std::string *why)
{
    auto bad = [&](const char *m) { if (why) *why = m; return false; };
    if (!g) return bad("grid descriptor is NULL");
    if (g->dims != 1 && g->dims != 2) return bad("dims must be 1 or 2");
    if (g->nz < 4) return bad("nz must be >= 4");
    if (g->dims == 1 && g->nx != 1) return bad("nx must be 1 in 1D");
    if (g->dims == 2 && g->nx < 4) return bad("nx must be >= 4 in 2D");
    if ((double)g->nz * g->nx > 2.0e9 / 72) return bad("grid too large for 32-bit plane offsets");
    if (!(g->delta > 0) || !(g->dt > 0)) return bad("delta and dt must be positive");
    if (g->closure != LBW_LEC && g->closure != LBW_WARMC) return bad("unknown closure");
    if (g->storage != LBW_FP64 && g->storage != LBW_FP32 && g->storage != LBW_FP16DEV)
        return bad("unknown storage");
    if (g->bc_z != LBW_BC_OPEN && g->bc_z != LBW_BC_PERIODIC) return bad("unknown bc_z");
    if (g->bc_x != LBW_BC_OPEN && g->bc_x != LBW_BC_PERIODIC) return bad("unknown bc_x");
    if (!(g->dvel > 0)) return bad("dvel must be positive");
    if (g->geom != LBW_GEOM_SLAB && g->geom != LBW_GEOM_AXI) return bad("unknown geometry");
    if (g->geom == LBW_GEOM_AXI && (g->dims != 2 || g->bc_x != LBW_BC_OPEN))
        return bad("the axisymmetric geometry is 2D with an open outer radius");
    return true;
}

// Valid descriptors the library does not implement (none at present).
bool grid_supported(const lbw_grid_desc *) { return true; }

Layout make_layout(const lbw_grid_desc *g)
{
    Layout L{};
    const size_t nc = (size_t)g->nz * g->nx;
    L.K = nscalars(g->dims, g->closure);
    L.Q = g->dims == 1 ? 3 : 9;
    size_t off = 0;
    const size_t popb = align_up(nc * L.K * L.Q * storage_size(g->storage));
    L.pop[0] = off; off += popb;
    L.pop[1] = off; off += popb;
    for (int b = 0; b < 2; ++b)
        for (int f = 0; f < 3; ++f) { L.fld[b][f] = off; off += align_up(nc * 8); }
    L.lag = off; off += align_up(nc * 8 * (size_t)nlag(g->dims, g->closure));
    // 1D warm closure: a second buffer, which the multi-step passes of the
    // persistent kernel write while their ring slots still read the first
    L.lag_alt = L.lag;
    if (g->dims == 1 && g->closure == LBW_WARMC) { L.lag_alt = off; off += align_up(nc * 8 * (size_t)NLAG1); }
    const int ks = L.K > 3 ? L.K : 3;
    L.stage = off; off += align_up(nc * 8 * (size_t)ks);
    L.nblk_diag = (int)((nc + DIAG_THREADS - 1) / DIAG_THREADS);
    L.part = off; off += align_up((size_t)L.nblk_diag * NDIAG * 8);
    L.aref = off; off += align_up(8 * 8);
    L.slice = off; off += align_up(MAX_SLICES * 8);
    L.fallbacks = off; off += align_up(8);
    L.nonfinite = off; off += align_up(8);
    L.diag = off; off += align_up(NDIAG * 8);
    L.total = off;
    return L;
}

}  // namespace

struct lbw_sim {
    lbw_grid_desc g;
    Layout L;
    char *ws;
    hipStream_t stream;
    int pcur, fcur;
    bool initialized, canonical, lag_valid;
    long step;
    double mu;
    double aref_host[8];
    Driver drv;
    std::string err;
    // kernel timing (event pairs around each fused launch)
    bool timing;
    std::vector<hipEvent_t> ev;
    int ev_used;
    double kernel_ms;
    long launches, pending_launches;
    int persist;  // 1D: workgroups of the persistent kernel (-1: not queried yet, 0: unavailable)
    int lcur;     // 1D warm closure: the lagged values are in L.lag_alt (1) or L.lag (0)
    int check_every;  // non-finite check after every this many steps (0: off)
    int diag_every;   // diagnostics recorded after every this many steps (0: off)
    double *diag_series;  // caller's device rows of 8 values
    long diag_capacity, diag_rows;  // rows the buffer holds, rows due so far
};

static char *lag_cur(lbw_sim *s) { return s->ws + (s->lcur ? s->L.lag_alt : s->L.lag); }

static lbw_status fail(lbw_sim *s, lbw_status code, const std::string &m)
{
    if (s) s->err = m;
    return code;
}

#define HIPCHK(sim, call)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((sim), LBW_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// Kernel dispatch over (dims, closure, storage).
namespace {

StepArgs base_args(lbw_sim *s)
{
    StepArgs a{};
    const lbw_grid_desc &g = s->g;
    a.nz = g.nz;
    a.nx = g.nx;
    a.ncell = g.nz * g.nx;
    a.bcz = g.bc_z;
    a.bcx = g.bc_x;
    a.delta = g.delta;
    a.dt = g.dt;
    a.inv2d = 1.0 / (2.0 * g.delta);
    a.omega = 1.0 / g.tau_tilde;
    a.lam = g.delta / g.dt;
    a.mu = s->mu;
    a.a_lec = (1.0 + 0.5 * g.dvel) * s->mu;
    a.two_over_d = 2.0 / g.dvel;
    a.dcode = g.dvel == 1.0 ? 1 : (g.dvel == 3.0 ? 3 : 0);
    a.axi = g.geom == LBW_GEOM_AXI;
    a.aref = (const double *)(s->ws + s->L.aref);
    a.fallbacks = (unsigned int *)(s->ws + s->L.fallbacks);
    a.lag = g.closure == LBW_WARMC ? (double *)lag_cur(s) : nullptr;
    a.lag_alt = g.closure == LBW_WARMC ? (double *)(s->ws + (s->lcur ? s->L.lag : s->L.lag_alt)) : nullptr;
    a.step = s->step;
    a.drv = s->drv;
    return a;
}

void set_io(lbw_sim *s, StepArgs &a)
{
    a.src = s->ws + s->L.pop[s->pcur];
    a.dst = s->ws + s->L.pop[1 - s->pcur];
    a.ez_in = (const double *)(s->ws + s->L.fld[s->fcur][0]);
    a.ex_in = (const double *)(s->ws + s->L.fld[s->fcur][1]);
    a.by_in = (const double *)(s->ws + s->L.fld[s->fcur][2]);
    a.ez_out = (double *)(s->ws + s->L.fld[1 - s->fcur][0]);
    a.ex_out = (double *)(s->ws + s->L.fld[1 - s->fcur][1]);
    a.by_out = (double *)(s->ws + s->L.fld[1 - s->fcur][2]);
}

// Non-temporal population stores in the 2D fused step (and, for the warm
// closure, field and lagged-value stores), whenever the two population
// buffers exceed the 256 MB last-level cache: below it the hint would send to
// HBM what the next kernel reads from that cache (1024 x 256 FP32 local
// equilibrium: the canonicalisation after a step 15.6 -> 21.8 us). Above it
// they measured faster in every case on the grouped population layout
// (4096 x 1024 warm FP64 1198 -> 1166 us, FP32 726 -> 693, FP16 513 -> 493
// before the layout; after it, 2048 x 512 local equilibrium FP64
// 121.4 -> 107.2 us, the axisymmetric 3000 x 600 local equilibrium FP64
// 217.5 -> 210.0, warm FP64 542.8 -> 508.4, FP32 297.1 -> 280.9, FP16
// 213.9 -> 208.5 us). With one population per access some cases had measured
// slower (warm FP64 on 32 x 8 tiles 1254 -> 1350 us, axisymmetric warm FP32
// 371 -> 377 and FP16 284 -> 305 us).

template <int DIM, int CL, class ST, bool AXI = false> struct Impl {
    template <class T> static void launch2d(const StepArgs &a, hipStream_t st)
    {
        // one-dimensional grid: the kernel maps blocks to tiles XCD by XCD
        dim3 grid(((a.nz + T::TZ - 1) / T::TZ) * ((a.nx + T::TX - 1) / T::TX));
        constexpr int K = NScal<2, CL>::K;
        const size_t pop_bytes = (size_t)a.ncell * 2 * K * 9 * sizeof(ST);
        if (pop_bytes > MALL_BYTES) {
            hipLaunchKernelGGL((k_step2d<CL, ST, T::TZ, T::TX, T::CPT, AXI, T::STRIP, true>), grid,
                               dim3(T::TZ * T::TX / T::CPT), 0, st, a);
            return;
        }
        hipLaunchKernelGGL((k_step2d<CL, ST, T::TZ, T::TX, T::CPT, AXI, T::STRIP, false>), grid,
                           dim3(T::TZ * T::TX / T::CPT), 0, st, a);
    }
    static void step(const StepArgs &a, hipStream_t st)
    {
        if constexpr (DIM == 2) {
            if constexpr (CL == LEC && !std::is_same<ST, double>::value) {
                const size_t pop_bytes = (size_t)a.ncell * 2 * 27 * sizeof(ST);
                if (std::is_same<ST, __half>::value || pop_bytes > MALL_BYTES) {
                    launch2d<Tile2Stream>(a, st);
                    return;
                }
            }
            if constexpr (AXI && CL == WARMC && std::is_same<ST, double>::value) {
                launch2d<Tile2WarmAxi64>(a, st);
                return;
            }
            launch2d<Tile2<CL, ST>>(a, st);
        } else {
            dim3 grid((a.nz + TZ1 - 1) / TZ1);
            hipLaunchKernelGGL((k_step1d<CL, ST, TZ1>), grid, dim3(TZ1), 0, st, a);
        }
    }
    // Tile of the persistent 1D kernel. With passes of 24 steps per grid
    // barrier the latency of a pass's own steps dominates, and it grows with
    // the waves a workgroup runs per SIMD: small tiles on many compute units
    // win although their rings redo more work. Measured per step (local
    // equilibrium / warm closure) at 4096 nodes: 1.97 / 1.32 us with 512-node
    // tiles, 1.79 / 1.04 with 256, 1.73 / 1.03 with 192, 1.73 / 1.36 with 128;
    // at 16384 nodes: 2.57 / 2.07 with 1024, 1.99 / 1.43 with 512, 1.85 / 1.45
    // with 256. (With one step per pass the barrier dominated and large tiles
    // won: 4096 nodes 5.6 / 5.2 / 5.5 us with 256 / 512 / 1024.)
    static bool persist_large(int nz) { return nz > 8192; }
    template <int TZ> static int persist_grid_t(int nz)
    {
        int dev = 0, coop = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 0;
        if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_step1d_persist<CL, ST, TZ>, TZ, 0) != hipSuccess)
            return 0;
        // passes of S steps run on tiles of TZ - 4S + 2 nodes
        const int t1 = (nz + TZ - 1) / TZ, t2 = (nz + multi_width<TZ, 2>() - 1) / multi_width<TZ, 2>();
        const int td = (nz + multi_width<TZ, PERSIST_DEPTH>() - 1) / multi_width<TZ, PERSIST_DEPTH>();
        const int ntiles = std::max(t1, std::max(t2, td));
        const int maxg = per * cus;
        return ntiles < maxg ? ntiles : maxg;
    }
    template <int TZ> static hipError_t step_persist_t(const StepArgs &a, int nsteps, int grid, hipStream_t st)
    {
        StepArgs aa = a;
        int ns = nsteps;
        void *args[] = {&aa, &ns};
        return hipLaunchCooperativeKernel((const void *)k_step1d_persist<CL, ST, TZ>, dim3(grid), dim3(TZ), args, 0,
                                          st);
    }
    // Workgroups of the persistent 1D kernel that can all be resident at once
    // (0: no cooperative launch on this device).
    static int persist_grid(int nz)
    {
        if constexpr (DIM == 1) {
            return persist_large(nz) ? persist_grid_t<TZP_LARGE>(nz) : persist_grid_t<TZP_SMALL>(nz);
        } else {
            return 0;
        }
    }
    static hipError_t step_persist(const StepArgs &a, int nsteps, int grid, hipStream_t st)
    {
        if constexpr (DIM == 1) {
            return persist_large(a.nz) ? step_persist_t<TZP_LARGE>(a, nsteps, grid, st)
                                       : step_persist_t<TZP_SMALL>(a, nsteps, grid, st);
        } else {
            return hipErrorInvalidValue;
        }
    }
    static void finish(const StepArgs &a, double *jz, double *jx, hipStream_t st)
    {
        const int nb = (a.ncell + 255) / 256;
        // non-temporal population stores when the buffers exceed the last-level
        // cache, as in the fused step
        constexpr int K = NScal<DIM, CL>::K;
        if ((size_t)a.ncell * 2 * K * Lattice<DIM>::Q * sizeof(ST) > MALL_BYTES)
            hipLaunchKernelGGL((k_finish_pull<DIM, CL, ST, true>), dim3(nb), dim3(256), 0, st, a, jz, jx);
        else
            hipLaunchKernelGGL((k_finish_pull<DIM, CL, ST, false>), dim3(nb), dim3(256), 0, st, a, jz, jx);
        if constexpr (DIM == 2) {
            hipLaunchKernelGGL(k_finish_b2d, dim3(nb), dim3(256), 0, st, a);
            hipLaunchKernelGGL(k_finish_e2d, dim3(nb), dim3(256), 0, st, a, (const double *)jz,
                               (const double *)jx);
        }
    }
    static void init_pops(void *dst, const double *A, const double *uz, const double *ux,
                          const double *aref, int ncell, double lam, hipStream_t st)
    {
        const int nb = (ncell + 255) / 256;
        hipLaunchKernelGGL((k_init_pops<DIM, CL, ST>), dim3(nb), dim3(256), 0, st, dst, A, uz, ux,
                           aref, ncell, lam);
    }
    static void read_moment(const StepArgs &a, int which, double *out, hipStream_t st)
    {
        const int nb = (a.ncell + 255) / 256;
        hipLaunchKernelGGL((k_read_moment<DIM, CL, ST>), dim3(nb), dim3(256), 0, st, a, which, out);
    }
    static void diag(const StepArgs &a, double *part, int nblk, double *out, hipStream_t st)
    {
        hipLaunchKernelGGL((k_diag_partial<DIM, CL, ST>), dim3(nblk), dim3(DIAG_THREADS), 0, st, a, part);
        hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(DIAG_THREADS), 0, st, (const double *)part, nblk, out);
    }
};

struct Ops {
    void (*step)(const StepArgs &, hipStream_t);
    int (*persist_grid)(int);
    hipError_t (*step_persist)(const StepArgs &, int, int, hipStream_t);
    void (*finish)(const StepArgs &, double *, double *, hipStream_t);
    void (*init_pops)(void *, const double *, const double *, const double *, const double *, int,
                      double, hipStream_t);
    void (*read_moment)(const StepArgs &, int, double *, hipStream_t);
    void (*diag)(const StepArgs &, double *, int, double *, hipStream_t);
};

template <int DIM, int CL, class ST, bool AXI = false> Ops ops_of()
{
    using I = Impl<DIM, CL, ST, AXI>;
    return Ops{&I::step, &I::persist_grid, &I::step_persist, &I::finish, &I::init_pops, &I::read_moment, &I::diag};
}

template <int DIM, int CL> Ops ops_st(int storage)
{
    if (storage == LBW_FP64) return ops_of<DIM, CL, double>();
    if (storage == LBW_FP32) return ops_of<DIM, CL, float>();
    return ops_of<DIM, CL, __half>();
}

Ops ops_for(const lbw_grid_desc &g)
{
    if (g.geom == LBW_GEOM_AXI) {  // 2D (grid_valid)
        if (g.closure == LBW_LEC) {
            if (g.storage == LBW_FP64) return ops_of<2, LEC, double, true>();
            if (g.storage == LBW_FP32) return ops_of<2, LEC, float, true>();
            return ops_of<2, LEC, __half, true>();
        }
        if (g.storage == LBW_FP64) return ops_of<2, WARMC, double, true>();
        if (g.storage == LBW_FP32) return ops_of<2, WARMC, float, true>();
        return ops_of<2, WARMC, __half, true>();
    }
    if (g.dims == 1) return g.closure == LBW_LEC ? ops_st<1, LEC>(g.storage) : ops_st<1, WARMC>(g.storage);
    return g.closure == LBW_LEC ? ops_st<2, LEC>(g.storage) : ops_st<2, WARMC>(g.storage);
}

double lambda_rest(double mu, double D) { return 0.5 * (D * mu + std::sqrt(D * D * mu * mu + 4.0)); }

// Storage reference A_ref per scalar: zero for FP64 storage; for FP32 and
// FP16 storage the uniform rest state (n = 1, lambda_0, lambda_0 mu on the
// populated pressure diagonal, zero momenta), so that a quiet region stores
// values near zero and its rounding does not add up coherently over steps.
void fill_aref(lbw_sim *s)
{
    const lbw_grid_desc &g = s->g;
    for (int k = 0; k < 8; ++k) s->aref_host[k] = 0.0;
    if (g.storage == LBW_FP64) return;
    s->aref_host[0] = 1.0;
    if (g.closure == LBW_WARMC) {
        const double l0 = lambda_rest(s->mu, g.dvel);
        s->aref_host[1] = l0;
        if (g.dims == 1) {
            s->aref_host[3] = l0 * s->mu;
        } else {
            s->aref_host[4] = l0 * s->mu;
            if (g.dvel >= 3.0) { s->aref_host[5] = l0 * s->mu; s->aref_host[6] = l0 * s->mu; }
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Static scratch of lbw_diagnostics_static: the per-workgroup partial sums of
// the diagnostics reduction (NDIAG values per workgroup of DIAG_THREADS
// nodes) and its NDIAG totals, 1 MiB in all, which bounds that call to grids
// of at most STATIC_DIAG_MAX_NODES nodes. Each GPU the library runs on holds
// its own copy until the process ends. In host code `scratch` only names the
// symbol: kernels get the device address from hipGetSymbolAddress, taken once
// per device with that device current and kept in g_scratch_ptr.
namespace {
constexpr int STATIC_DIAG_MAX_BLOCKS = 21824;
constexpr size_t STATIC_DIAG_MAX_NODES = (size_t)STATIC_DIAG_MAX_BLOCKS * DIAG_THREADS;
constexpr int STATIC_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[STATIC_DEVICES] = {};
}  // namespace
static __device__ __align__(256) double scratch[NDIAG * STATIC_DIAG_MAX_BLOCKS + 64];

// The public layout of lbw_diagnostics from the reduction's raw totals
// (sums of n dV, field energy, kinetic energy, Gauss residual^2, non-finite
// nodes; max |u| / Lambda).
static __global__ void k_diag_publish(const double *raw, const unsigned int *fallbacks, double nodes, long step,
                                      double *out)
{
    if (threadIdx.x != 0) return;
    out[0] = raw[0];
    out[1] = raw[1];
    out[2] = raw[2];
    out[3] = sqrt(raw[3] / nodes);
    out[4] = raw[5];
    out[5] = raw[4];
    out[6] = (double)*fallbacks;
    out[7] = (double)step;
}

// ---------------------------------------------------------------------------
// Streaming-copy reference: one 16-byte non-temporal load and store per thread.
// (A sweep of 1, 2, 4 and 8 accesses per thread and 256- to 1024-thread
// workgroups, with and without the non-temporal hint, found this form the
// fastest on gfx950.)
typedef unsigned int lbw_v4u __attribute__((ext_vector_type(4)));
static __global__ __launch_bounds__(256) void k_stream_copy(const lbw_v4u *__restrict__ src,
                                                            lbw_v4u *__restrict__ dst, size_t n16)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

extern "C" {

size_t lbw_workspace_bytes(const lbw_grid_desc *grid)
{
    if (!grid_valid(grid, nullptr) || !grid_supported(grid)) return 0;
    return make_layout(grid).total;
}

const char *lbw_version(void) { return "lbwake 0.2 (gfx950)"; }

lbw_status lbw_stream_copy(void *dst, const void *src, size_t bytes, void *stream)
{
    if (!dst || !src) return LBW_ERR_ARG;
    const uintptr_t d = (uintptr_t)dst, sp = (uintptr_t)src;
    if ((d | sp | bytes) & 15) return LBW_ERR_ARG;
    if (d < sp + bytes && sp < d + bytes) return LBW_ERR_ARG;
    const size_t n16 = bytes / 16;
    if (n16 == 0) return LBW_OK;
    const size_t blocks = (n16 + 255) / 256;
    if (blocks > 0xFFFFFFFFull) return LBW_ERR_ARG;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (const lbw_v4u *)src, (lbw_v4u *)dst, n16);
    return hipGetLastError() == hipSuccess ? LBW_OK : LBW_ERR_HIP;
}

lbw_status lbw_create(const lbw_grid_desc *grid, void *ws, size_t ws_bytes, void *stream,
                      lbw_sim **out)
{
    if (!out) return LBW_ERR_ARG;
    *out = nullptr;
    std::string why;
    if (!grid_valid(grid, &why)) return LBW_ERR_ARG;
    if (!grid_supported(grid)) return LBW_ERR_UNSUPPORTED;
    if (!(grid->tau_tilde > 0.5)) return LBW_ERR_UNSTABLE;
    if (grid->dt > grid->delta / std::sqrt((double)grid->dims) * (1.0 + 1e-12)) return LBW_ERR_UNSTABLE;
    const Layout L = make_layout(grid);
    if (!ws || ws_bytes < L.total || ((uintptr_t)ws % ALIGN) != 0) return LBW_ERR_WORKSPACE;
    lbw_sim *s = new lbw_sim();
    s->g = *grid;
    s->L = L;
    s->ws = (char *)ws;
    s->stream = (hipStream_t)stream;
    s->pcur = s->fcur = 0;
    s->initialized = s->canonical = s->lag_valid = false;
    s->step = 0;
    s->mu = 0.0;
    s->drv = Driver{};
    s->timing = false;
    s->ev_used = 0;
    s->kernel_ms = 0.0;
    s->launches = 0;
    s->pending_launches = 0;
    s->persist = -1;
    s->lcur = 0;
    s->check_every = 0;
    s->diag_every = 0;
    s->diag_series = nullptr;
    s->diag_capacity = s->diag_rows = 0;
    *out = s;
    return LBW_OK;
}

void lbw_destroy(lbw_sim *s)
{
    if (!s) return;
    for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
    delete s;
}

static lbw_status drain_timing(lbw_sim *s)
{
    if (s->ev_used == 0) return LBW_OK;
    HIPCHK(s, hipEventSynchronize(s->ev[s->ev_used - 1]));
    for (int i = 0; i + 1 < s->ev_used; i += 2) {
        float ms = 0.0f;
        HIPCHK(s, hipEventElapsedTime(&ms, s->ev[i], s->ev[i + 1]));
        s->kernel_ms += ms;
    }
    s->launches += s->pending_launches;
    s->pending_launches = 0;
    s->ev_used = 0;
    return LBW_OK;
}

lbw_status lbw_set_timing(lbw_sim *s, int enable)
{
    if (!s) return LBW_ERR_ARG;
    lbw_status st = drain_timing(s);
    if (st != LBW_OK) return st;
    if (enable && s->ev.empty()) {
        s->ev.resize(256);
        for (auto &e : s->ev) HIPCHK(s, hipEventCreate(&e));
    }
    if (!enable && !s->ev.empty()) {
        // a simulation without timing holds no HIP objects
        for (hipEvent_t e : s->ev) HIPCHK(s, hipEventDestroy(e));
        s->ev.clear();
    }
    s->timing = enable != 0;
    s->kernel_ms = 0.0;
    s->launches = 0;
    return LBW_OK;
}

lbw_status lbw_get_timing(lbw_sim *s, double *kernel_ms, long *launches)
{
    if (!s || !kernel_ms || !launches) return LBW_ERR_ARG;
    lbw_status st = drain_timing(s);
    if (st != LBW_OK) return st;
    *kernel_ms = s->kernel_ms;
    *launches = s->launches;
    return LBW_OK;
}

const char *lbw_last_error(const lbw_sim *s) { return s ? s->err.c_str() : "NULL simulation"; }

long lbw_step_count(const lbw_sim *s) { return s ? s->step : -1; }

static lbw_status reset_common(lbw_sim *s, double mu)
{
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    s->mu = mu;
    fill_aref(s);
    HIPCHK(s, hipMemcpyAsync(s->ws + s->L.aref, s->aref_host, 8 * sizeof(double),
                             hipMemcpyHostToDevice, s->stream));
    for (int b = 0; b < 2; ++b)
        for (int f = 0; f < 3; ++f)
            HIPCHK(s, hipMemsetAsync(s->ws + s->L.fld[b][f], 0, nc * 8, s->stream));
    if (s->L.lag != s->L.stage)
        HIPCHK(s, hipMemsetAsync(s->ws + s->L.lag, 0, s->L.stage - s->L.lag, s->stream));
    HIPCHK(s, hipMemsetAsync(s->ws + s->L.fallbacks, 0, 8, s->stream));
    HIPCHK(s, hipMemsetAsync(s->ws + s->L.nonfinite, 0, 8, s->stream));
    s->pcur = s->fcur = 0;
    s->lcur = 0;
    s->canonical = true;
    s->lag_valid = false;
    s->step = 0;
    s->drv = Driver{};
    s->initialized = true;
    return LBW_OK;
}

static lbw_status upload_and_init(lbw_sim *s, const std::vector<double> &A, const std::vector<double> &uz,
                                  const std::vector<double> &ux)
{
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    const int K = s->L.K;
    double *stage = (double *)(s->ws + s->L.stage);
    // stage holds A [K][nc]; the velocities go to the other population buffer
    // (free until the first step) as scratch
    double *uzd = (double *)(s->ws + s->L.pop[1]);
    double *uxd = uzd + nc;
    if (s->L.pop[1] - s->L.pop[0] < 2 * nc * 8) {
        // populations smaller than two FP64 planes (FP16 1D): use the field buffers
        uzd = (double *)(s->ws + s->L.fld[1][0]);
        uxd = (double *)(s->ws + s->L.fld[1][1]);
    }
    HIPCHK(s, hipMemcpyAsync(stage, A.data(), (size_t)K * nc * 8, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(uzd, uz.data(), nc * 8, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(uxd, ux.data(), nc * 8, hipMemcpyHostToDevice, s->stream));
    ops_for(s->g).init_pops(s->ws + s->L.pop[0], stage, uzd, uxd, (const double *)(s->ws + s->L.aref),
                            (int)nc, s->g.delta / s->g.dt, s->stream);
    HIPCHK(s, hipGetLastError());
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (int f = 0; f < 3; ++f)
        HIPCHK(s, hipMemsetAsync(s->ws + s->L.fld[1][f], 0, nc * 8, s->stream));
    return LBW_OK;
}

lbw_status lbw_init_plasma(lbw_sim *s, const lbw_plasma_desc *p)
{
    if (!s || !p) return fail(s, LBW_ERR_ARG, "NULL argument");
    if (!(p->mu >= 0.0)) return fail(s, LBW_ERR_ARG, "mu must be >= 0");
    lbw_status st = reset_common(s, p->mu);
    if (st != LBW_OK) return st;
    const lbw_grid_desc &g = s->g;
    const size_t nc = (size_t)g.nz * g.nx;
    const int K = s->L.K;
    const double D = g.dvel, mu = p->mu;
    std::vector<double> A((size_t)K * nc, 0.0), uz(nc, 0.0), ux(nc, 0.0);
    for (size_t c = 0; c < nc; ++c) {
        const double n = p->n_init ? p->n_init[c] : 1.0;
        const double vz = p->uz_init ? p->uz_init[c] : 0.0;
        const double vx = (p->ux_init && g.dims == 2) ? p->ux_init[c] : 0.0;
        const double uu = vz * vz + vx * vx;
        if (!(n > 0.0) || !(uu < 1.0) || !std::isfinite(n) || !std::isfinite(uu))
            return fail(s, LBW_ERR_NONFINITE, "initial density must be positive and |u| < 1");
        const double gam = 1.0 / std::sqrt(1.0 - uu);
        uz[c] = vz;
        ux[c] = vx;
        A[c] = n;
        if (g.closure == LBW_LEC) {
            // A_1 = [1 + (1 + D/2) mu (n/gamma)^{2/D}] n gamma u (eq. lb-ade-lec-comps-A)
            const double h = 1.0 + (1.0 + 0.5 * D) * mu * std::pow(n / gam, 2.0 / D);
            A[1 * nc + c] = h * n * gam * vz;
            if (g.dims == 2) A[2 * nc + c] = h * n * gam * vx;
        } else {
            // rest state diag(0, P, P, P) on the D populated directions, boosted
            // to the lab (eq. double-boost); lambda = gamma lambda_0 (eq. traces3)
            const double P = n / gam * mu, lam = gam * lambda_rest(mu, D);
            const double v[3] = {vx, 0.0, vz}, p0[3] = {D >= 3.0 ? P : 0.0, D >= 3.0 ? P : 0.0, P};
            double th[3][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double acc = 0.0;
                    for (int m = 0; m < 3; ++m) {
                        const double Lim = (i == m ? 1.0 : 0.0) + (uu > 0.0 ? (gam - 1.0) * v[i] * v[m] / uu : 0.0);
                        const double Ljm = (j == m ? 1.0 : 0.0) + (uu > 0.0 ? (gam - 1.0) * v[j] * v[m] / uu : 0.0);
                        acc += Lim * Ljm * p0[m];
                    }
                    th[i][j] = acc;
                }
            A[1 * nc + c] = n * lam;
            A[2 * nc + c] = n * lam * vz;
            if (g.dims == 1) {
                A[3 * nc + c] = lam * th[2][2];
            } else {
                A[3 * nc + c] = n * lam * vx;
                A[4 * nc + c] = lam * th[2][2];
                A[5 * nc + c] = lam * th[0][0];
                A[6 * nc + c] = lam * th[1][1];
                A[7 * nc + c] = lam * th[0][2];
            }
        }
    }
    return upload_and_init(s, A, uz, ux);
}

lbw_status lbw_init_moments(lbw_sim *s, double mu, const double *Ah, const double *uzh, const double *uxh)
{
    if (!s || !Ah) return fail(s, LBW_ERR_ARG, "NULL argument");
    if (!(mu >= 0.0)) return fail(s, LBW_ERR_ARG, "mu must be >= 0");
    lbw_status st = reset_common(s, mu);
    if (st != LBW_OK) return st;
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    std::vector<double> A(Ah, Ah + (size_t)s->L.K * nc), uz(nc, 0.0), ux(nc, 0.0);
    if (uzh) uz.assign(uzh, uzh + nc);
    if (uxh && s->g.dims == 2) ux.assign(uxh, uxh + nc);
    return upload_and_init(s, A, uz, ux);
}

lbw_status lbw_init_driver(lbw_sim *s, const lbw_driver_desc *d, int init_fields)
{
    if (!s || !d) return fail(s, LBW_ERR_ARG, "NULL argument");
    if (!s->initialized) return fail(s, LBW_ERR_STATE, "init_plasma first");
    if (d->alpha != 0.0 && (!(d->sigma_z > 0) || (s->g.dims == 2 && !(d->sigma_x > 0))))
        return fail(s, LBW_ERR_ARG, "bunch widths must be positive");
    if (s->g.geom == LBW_GEOM_AXI && d->x0 != 0.0)
        return fail(s, LBW_ERR_ARG, "the axisymmetric driver sits on the axis (x0 = 0)");
    if (d->nslices < 0 || d->nslices > MAX_SLICES || (d->nslices > 0 && !d->slice_w) ||
        (d->nslices > 0 && !(d->slice_zmax > d->slice_zmin)))
        return fail(s, LBW_ERR_ARG, "invalid slice description");
    const bool set_fields = init_fields && d->alpha != 0.0;
    if (set_fields && !s->canonical) return fail(s, LBW_ERR_STATE, "fields can only be set on a canonical state");
    Driver v{};
    v.alpha = d->alpha;
    v.sigma_z = d->sigma_z;
    v.sigma_x = d->sigma_x;
    v.z0 = d->z0;
    v.x0 = d->x0;
    v.nslices = d->nslices;
    v.slice_zmin = d->slice_zmin;
    v.slice_zmax = d->slice_zmax;
    v.slice_w = (const double *)(s->ws + s->L.slice);
    v.inv2sz2 = d->sigma_z > 0 ? 1.0 / (2.0 * d->sigma_z * d->sigma_z) : 0.0;
    v.inv2sx2 = d->sigma_x > 0 ? 1.0 / (2.0 * d->sigma_x * d->sigma_x) : 0.0;
    if (d->nslices > 0)
        HIPCHK(s, hipMemcpyAsync(s->ws + s->L.slice, d->slice_w, d->nslices * sizeof(double),
                                 hipMemcpyHostToDevice, s->stream));
    s->drv = v;
    if (set_fields) {
        StepArgs a = base_args(s);
        const int nb = (a.ncell + 255) / 256;
        double *ez = (double *)(s->ws + s->L.fld[s->fcur][0]);
        double *ex = (double *)(s->ws + s->L.fld[s->fcur][1]);
        double *by = (double *)(s->ws + s->L.fld[s->fcur][2]);
        if (s->g.dims == 1)
            hipLaunchKernelGGL(k_init_fields<1>, dim3(nb), dim3(256), 0, s->stream, a, ez, ex, by);
        else
            hipLaunchKernelGGL(k_init_fields<2>, dim3(nb), dim3(256), 0, s->stream, a, ez, ex, by);
        HIPCHK(s, hipGetLastError());
    }
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return LBW_OK;
}

lbw_status lbw_set_field(lbw_sim *s, int which, const double *host, size_t count)
{
    if (!s || !host) return fail(s, LBW_ERR_ARG, "NULL argument");
    if (!s->initialized) return fail(s, LBW_ERR_STATE, "init_plasma first");
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    if (count != nc) return fail(s, LBW_ERR_ARG, "count must be nx*nz");
    if (which < 0 || which > 2 || (s->g.dims == 1 && which != LBW_EZ))
        return fail(s, LBW_ERR_ARG, "which must be a Yee array of this grid");
    HIPCHK(s, hipMemcpyAsync(s->ws + s->L.fld[s->fcur][which], host, nc * 8, hipMemcpyHostToDevice,
                             s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return LBW_OK;
}

// nsteps fused steps and the closing canonicalisation; with check set, the
// finish kernels raise the non-finite flag.
static lbw_status step_chunk(lbw_sim *s, int nsteps, bool check)
{
    const Ops ops = ops_for(s->g);
    if (s->timing) {
        if (s->ev_used + 2 > (int)s->ev.size()) {
            lbw_status st = drain_timing(s);
            if (st != LBW_OK) return st;
        }
        HIPCHK(s, hipEventRecord(s->ev[s->ev_used++], s->stream));
    }
    if (s->g.dims == 1 && s->persist < 0) s->persist = ops.persist_grid(s->g.nz);
    if (s->g.dims == 1 && s->persist > 0 && nsteps >= 2) {
        // 1D: every step of the call in one cooperative launch
        StepArgs a = base_args(s);
        set_io(s, a);
        a.do_pull = s->canonical ? 0 : 1;
        a.do_maxwell = s->canonical ? 0 : 1;
        a.lag_init = s->lag_valid ? 0 : 1;
        HIPCHK(s, ops.step_persist(a, nsteps, s->persist, s->stream));
        const int passes = persist_passes(nsteps);  // buffer swaps
        s->pcur ^= passes & 1;
        s->fcur ^= passes & 1;
        if (s->g.closure == LBW_WARMC) s->lcur ^= persist_multi_passes(nsteps) & 1;
        s->canonical = false;
        s->lag_valid = true;
        s->step += nsteps;
    } else {
        for (int t = 0; t < nsteps; ++t) {
            StepArgs a = base_args(s);
            set_io(s, a);
            a.do_pull = s->canonical ? 0 : 1;
            a.do_maxwell = s->canonical ? 0 : 1;
            a.lag_init = s->lag_valid ? 0 : 1;
            ops.step(a, s->stream);
            s->pcur ^= 1;
            s->fcur ^= 1;
            s->canonical = false;
            s->lag_valid = true;
            s->step++;
        }
    }
    HIPCHK(s, hipGetLastError());
    if (s->timing) {
        HIPCHK(s, hipEventRecord(s->ev[s->ev_used++], s->stream));
        s->pending_launches += nsteps;
    }
    // bring the state to canonical form (f^n, E^n, B^{n-1/2})
    StepArgs a = base_args(s);
    set_io(s, a);
    if (check) a.nonfinite = (unsigned int *)(s->ws + s->L.nonfinite);
    double *stage = (double *)(s->ws + s->L.stage);
    ops.finish(a, stage, stage + (size_t)a.ncell, s->stream);
    HIPCHK(s, hipGetLastError());
    s->pcur ^= 1;
    s->fcur ^= 1;
    s->canonical = true;
    return LBW_OK;
}

// The diagnostics of the canonical state into the next row of the caller's
// series (asynchronous; rows beyond its capacity are counted, not written).
static lbw_status record_diagnostics(lbw_sim *s)
{
    const long row = s->diag_rows++;
    if (row >= s->diag_capacity) return LBW_OK;
    StepArgs a = base_args(s);
    set_io(s, a);
    double *part = (double *)(s->ws + s->L.part);
    double *raw = (double *)(s->ws + s->L.diag);
    ops_for(s->g).diag(a, part, s->L.nblk_diag, raw, s->stream);
    hipLaunchKernelGGL(k_diag_publish, dim3(1), dim3(64), 0, s->stream, (const double *)raw,
                       (const unsigned int *)(s->ws + s->L.fallbacks), (double)s->g.nz * s->g.nx, s->step,
                       s->diag_series + 8 * row);
    HIPCHK(s, hipGetLastError());
    return LBW_OK;
}

lbw_status lbw_step(lbw_sim *s, int nsteps)
{
    if (!s) return LBW_ERR_ARG;
    if (!s->initialized) return fail(s, LBW_ERR_STATE, "init_plasma first");
    if (nsteps < 0) return fail(s, LBW_ERR_ARG, "nsteps must be >= 0");
    if (nsteps == 0) return LBW_OK;
    const long ce = s->check_every, de = s->diag_every;
    if (ce <= 0 && de <= 0) return step_chunk(s, nsteps, false);
    // chunks that end on multiples of check_every and of diag_every steps;
    // split calls equal one long call bit for bit
    int left = nsteps;
    while (left > 0) {
        long n = left;
        if (ce > 0) n = std::min<long>(n, ce - s->step % ce);
        if (de > 0) n = std::min<long>(n, de - s->step % de);
        const bool check = ce > 0 && (s->step + n) % ce == 0;
        lbw_status st = step_chunk(s, (int)n, check);
        if (st != LBW_OK) return st;
        left -= (int)n;
        if (de > 0 && s->step % de == 0) {
            st = record_diagnostics(s);
            if (st != LBW_OK) return st;
        }
        if (check) {
            unsigned int flag = 0;
            HIPCHK(s, hipMemcpyAsync(&flag, s->ws + s->L.nonfinite, sizeof(flag), hipMemcpyDeviceToHost, s->stream));
            HIPCHK(s, hipStreamSynchronize(s->stream));
            if (flag)
                return fail(s, LBW_ERR_NONFINITE,
                            "non-finite values in the state after step " + std::to_string(s->step));
        }
    }
    return LBW_OK;
}

lbw_status lbw_set_diagnostics_every(lbw_sim *s, int every, double *device_series, long capacity)
{
    if (!s) return LBW_ERR_ARG;
    if (every < 0 || capacity < 0) return fail(s, LBW_ERR_ARG, "every and capacity must be >= 0");
    if (every > 0 && (!device_series || capacity == 0))
        return fail(s, LBW_ERR_ARG, "recording needs a device buffer of at least one row");
    s->diag_every = every;
    s->diag_series = every > 0 ? device_series : nullptr;
    s->diag_capacity = every > 0 ? capacity : 0;
    s->diag_rows = 0;
    return LBW_OK;
}

long lbw_diagnostics_rows(const lbw_sim *s) { return s ? s->diag_rows : -1; }

lbw_status lbw_set_nonfinite_check(lbw_sim *s, int every)
{
    if (!s) return LBW_ERR_ARG;
    if (every < 0) return fail(s, LBW_ERR_ARG, "every must be >= 0");
    s->check_every = every;
    return LBW_OK;
}

static lbw_status read_common(lbw_sim *s, int which, double *dev_out)
{
    StepArgs a = base_args(s);
    set_io(s, a);
    ops_for(s->g).read_moment(a, which, dev_out, s->stream);
    HIPCHK(s, hipGetLastError());
    return LBW_OK;
}

lbw_status lbw_read_moment(lbw_sim *s, int which, double *host_out, size_t count)
{
    if (!s || !host_out) return fail(s, LBW_ERR_ARG, "NULL argument");
    if (!s->initialized) return fail(s, LBW_ERR_STATE, "init_plasma first");
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    if (count != nc) return fail(s, LBW_ERR_ARG, "count must be nx*nz");
    if (which < 0 || which >= LBW_NMOMENTS) return fail(s, LBW_ERR_ARG, "unknown moment");
    double *stage = (double *)(s->ws + s->L.stage);
    lbw_status st = read_common(s, which, stage);
    if (st != LBW_OK) return st;
    HIPCHK(s, hipMemcpyAsync(host_out, stage, nc * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return LBW_OK;
}

lbw_status lbw_read_moment_device(lbw_sim *s, int which, double *dev_out)
{
    if (!s || !dev_out) return fail(s, LBW_ERR_ARG, "NULL argument");
    if (!s->initialized) return fail(s, LBW_ERR_STATE, "init_plasma first");
    if (which < 0 || which >= LBW_NMOMENTS) return fail(s, LBW_ERR_ARG, "unknown moment");
    return read_common(s, which, dev_out);
}

lbw_status lbw_read_field(lbw_sim *s, int which, int at_nodes, double *host_out, size_t count)
{
    if (!s || !host_out) return fail(s, LBW_ERR_ARG, "NULL argument");
    if (!s->initialized) return fail(s, LBW_ERR_STATE, "init_plasma first");
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    if (count != nc) return fail(s, LBW_ERR_ARG, "count must be nx*nz");
    if (which < 0 || which >= LBW_NFIELDS || (which == LBW_WAKE_X && !at_nodes))
        return fail(s, LBW_ERR_ARG, "unknown field");
    StepArgs a = base_args(s);
    set_io(s, a);
    double *stage = (double *)(s->ws + s->L.stage);
    const int nb = (a.ncell + 255) / 256;
    if (s->g.dims == 1)
        hipLaunchKernelGGL(k_read_field<1>, dim3(nb), dim3(256), 0, s->stream, a, which, at_nodes, stage);
    else
        hipLaunchKernelGGL(k_read_field<2>, dim3(nb), dim3(256), 0, s->stream, a, which, at_nodes, stage);
    HIPCHK(s, hipGetLastError());
    HIPCHK(s, hipMemcpyAsync(host_out, stage, nc * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return LBW_OK;
}

lbw_status lbw_diagnostics(lbw_sim *s, double *out)
{
    if (!s || !out) return fail(s, LBW_ERR_ARG, "NULL argument");
    if (!s->initialized) return fail(s, LBW_ERR_STATE, "init_plasma first");
    StepArgs a = base_args(s);
    set_io(s, a);
    double *part = (double *)(s->ws + s->L.part);
    double *dout = (double *)(s->ws + s->L.diag);
    ops_for(s->g).diag(a, part, s->L.nblk_diag, dout, s->stream);
    HIPCHK(s, hipGetLastError());
    double d[NDIAG];
    unsigned int fb = 0;
    HIPCHK(s, hipMemcpyAsync(d, dout, sizeof(d), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(&fb, s->ws + s->L.fallbacks, sizeof(fb), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    const double nc = (double)s->g.nz * s->g.nx;
    out[0] = d[0];
    out[1] = d[1];
    out[2] = d[2];
    out[3] = std::sqrt(d[3] / nc);
    out[4] = d[5];
    out[5] = d[4];
    out[6] = (double)fb;
    out[7] = (double)s->step;
    if (d[4] > 0 || !std::isfinite(d[0])) return fail(s, LBW_ERR_NONFINITE, "non-finite values in the state");
    return LBW_OK;
}

// Device address of this GPU's static scratch (the device that holds the
// simulation's workspace), taken once per device.
static lbw_status static_scratch(lbw_sim *s, double **out)
{
    hipPointerAttribute_t attr{};
    HIPCHK(s, hipPointerGetAttributes(&attr, s->ws));
    const int dev = attr.device;
    if (dev < 0 || dev >= STATIC_DEVICES) return fail(s, LBW_ERR_UNSUPPORTED, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        HIPCHK(s, hipGetDevice(&cur));
        if (cur != dev) HIPCHK(s, hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) HIPCHK(s, hipSetDevice(cur));
        if (e != hipSuccess || !p)
            return fail(s, LBW_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return LBW_OK;
}

lbw_status lbw_diagnostics_static(lbw_sim *s, double *device_out)
{
    if (!s || !device_out) return fail(s, LBW_ERR_ARG, "NULL argument");
    if (!s->initialized) return fail(s, LBW_ERR_STATE, "init_plasma first");
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    if (nc > STATIC_DIAG_MAX_NODES)
        return fail(s, LBW_ERR_UNSUPPORTED, "grid larger than the static scratch of lbw_diagnostics_static allows (" +
                                                std::to_string(STATIC_DIAG_MAX_NODES) + " nodes)");
    double *ptr = nullptr;
    lbw_status st = static_scratch(s, &ptr);
    if (st != LBW_OK) return st;
    StepArgs a = base_args(s);
    set_io(s, a);
    const int nblk = s->L.nblk_diag;
    double *part = ptr, *raw = ptr + (size_t)NDIAG * STATIC_DIAG_MAX_BLOCKS;
    ops_for(s->g).diag(a, part, nblk, raw, s->stream);
    hipLaunchKernelGGL(k_diag_publish, dim3(1), dim3(64), 0, s->stream, (const double *)raw,
                       (const unsigned int *)(s->ws + s->L.fallbacks), (double)nc, s->step, device_out);
    HIPCHK(s, hipGetLastError());
    return LBW_OK;
}

// ---------------------------------------------------------------------------
// Checkpoint format: a fixed header followed by the canonical populations,
// the three Yee arrays and the lagged values.
namespace {
struct StateHeader {
    char magic[8];
    int dims, nz, nx, closure, storage, lag_valid;
    long step;
    double mu;
    unsigned int fallbacks, pad;
};
}  // namespace

size_t lbw_state_bytes(const lbw_sim *s)
{
    if (!s) return 0;
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    return sizeof(StateHeader) + nc * s->L.K * s->L.Q * storage_size(s->g.storage) + 3 * nc * 8 +
           (size_t)nlag(s->g.dims, s->g.closure) * nc * 8;
}

// The header into the host buffer, then the device parts (and the header's
// fallback count) queued on the simulation's stream.
static lbw_status enqueue_save(lbw_sim *s, void *host, size_t bytes)
{
    if (!s || !host) return fail(s, LBW_ERR_ARG, "NULL argument");
    if (!s->initialized) return fail(s, LBW_ERR_STATE, "init_plasma first");
    if (bytes < lbw_state_bytes(s)) return fail(s, LBW_ERR_ARG, "buffer too small");
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    StateHeader h{};
    std::memcpy(h.magic, "LBWSTAT2", 8);
    h.dims = s->g.dims; h.nz = s->g.nz; h.nx = s->g.nx; h.closure = s->g.closure;
    h.storage = s->g.storage; h.lag_valid = s->lag_valid; h.step = s->step; h.mu = s->mu;
    std::memcpy(host, &h, sizeof(h));
    HIPCHK(s, hipMemcpyAsync((char *)host + offsetof(StateHeader, fallbacks), s->ws + s->L.fallbacks, 4,
                             hipMemcpyDeviceToHost, s->stream));
    char *p = (char *)host + sizeof(StateHeader);
    const size_t popb = nc * s->L.K * s->L.Q * storage_size(s->g.storage);
    HIPCHK(s, hipMemcpyAsync(p, s->ws + s->L.pop[s->pcur], popb, hipMemcpyDeviceToHost, s->stream));
    p += popb;
    for (int f = 0; f < 3; ++f, p += nc * 8)
        HIPCHK(s, hipMemcpyAsync(p, s->ws + s->L.fld[s->fcur][f], nc * 8, hipMemcpyDeviceToHost, s->stream));
    const size_t lagb = (size_t)nlag(s->g.dims, s->g.closure) * nc * 8;
    if (lagb) HIPCHK(s, hipMemcpyAsync(p, lag_cur(s), lagb, hipMemcpyDeviceToHost, s->stream));
    return LBW_OK;
}

lbw_status lbw_save_state(lbw_sim *s, void *host, size_t bytes)
{
    lbw_status rc = enqueue_save(s, host, bytes);
    if (rc != LBW_OK) return rc;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return LBW_OK;
}

lbw_status lbw_save_state_async(lbw_sim *s, void *host, size_t bytes) { return enqueue_save(s, host, bytes); }

lbw_status lbw_load_state(lbw_sim *s, const void *host, size_t bytes)
{
    if (!s || !host) return fail(s, LBW_ERR_ARG, "NULL argument");
    if (bytes < lbw_state_bytes(s)) return fail(s, LBW_ERR_ARG, "buffer too small");
    StateHeader h;
    std::memcpy(&h, host, sizeof(h));
    if (std::memcmp(h.magic, "LBWSTAT2", 8) != 0 || h.dims != s->g.dims || h.nz != s->g.nz ||
        h.nx != s->g.nx || h.closure != s->g.closure || h.storage != s->g.storage)
        return fail(s, LBW_ERR_ARG, "state does not match this grid");
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    s->mu = h.mu;
    fill_aref(s);
    HIPCHK(s, hipMemcpyAsync(s->ws + s->L.aref, s->aref_host, 8 * sizeof(double), hipMemcpyHostToDevice,
                             s->stream));
    s->pcur = s->fcur = 0;
    const char *p = (const char *)host + sizeof(StateHeader);
    const size_t popb = nc * s->L.K * s->L.Q * storage_size(s->g.storage);
    HIPCHK(s, hipMemcpyAsync(s->ws + s->L.pop[0], p, popb, hipMemcpyHostToDevice, s->stream));
    p += popb;
    for (int f = 0; f < 3; ++f, p += nc * 8)
        HIPCHK(s, hipMemcpyAsync(s->ws + s->L.fld[0][f], p, nc * 8, hipMemcpyHostToDevice, s->stream));
    const size_t lagb = (size_t)nlag(s->g.dims, s->g.closure) * nc * 8;
    s->lcur = 0;
    if (lagb) HIPCHK(s, hipMemcpyAsync(s->ws + s->L.lag, p, lagb, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->ws + s->L.fallbacks, &h.fallbacks, 4, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemsetAsync(s->ws + s->L.nonfinite, 0, 8, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    s->step = h.step;
    s->lag_valid = h.lag_valid != 0;
    s->canonical = true;
    s->initialized = true;
    return LBW_OK;
}

// ---------------------------------------------------------------------------
// Device-side copies of the canonical state, and the discrete adjoint.
namespace {
struct DevStateLayout {
    size_t pop, fld[3], lag, total;
};
DevStateLayout dev_state_layout(const lbw_sim *s)
{
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    DevStateLayout d{};
    size_t off = 0;
    d.pop = off; off += align_up(nc * s->L.K * s->L.Q * storage_size(s->g.storage));
    for (int f = 0; f < 3; ++f) { d.fld[f] = off; off += align_up(nc * 8); }
    d.lag = off; off += align_up((size_t)nlag(s->g.dims, s->g.closure) * nc * 8);
    d.total = off;
    return d;
}
constexpr int ADJ_SCRATCH_PLANES = 12;  // B', F_z, F_x, En_z, En_x, Bn_y, Bh adjoints; A' adjoint (3); forward Bh; X
}  // namespace

size_t lbw_state_device_bytes(const lbw_sim *s) { return s ? dev_state_layout(s).total : 0; }

lbw_status lbw_save_state_device(lbw_sim *s, void *dev)
{
    if (!s || !dev) return fail(s, LBW_ERR_ARG, "NULL argument");
    if (!s->initialized) return fail(s, LBW_ERR_STATE, "init_plasma first");
    if (((uintptr_t)dev % ALIGN) != 0) return fail(s, LBW_ERR_ARG, "device buffer must be 256-byte aligned");
    const DevStateLayout d = dev_state_layout(s);
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    char *p = (char *)dev;
    HIPCHK(s, hipMemcpyAsync(p + d.pop, s->ws + s->L.pop[s->pcur], nc * s->L.K * s->L.Q * storage_size(s->g.storage),
                             hipMemcpyDeviceToDevice, s->stream));
    for (int f = 0; f < 3; ++f)
        HIPCHK(s, hipMemcpyAsync(p + d.fld[f], s->ws + s->L.fld[s->fcur][f], nc * 8, hipMemcpyDeviceToDevice,
                                 s->stream));
    const size_t lagb = (size_t)nlag(s->g.dims, s->g.closure) * nc * 8;
    if (lagb) HIPCHK(s, hipMemcpyAsync(p + d.lag, lag_cur(s), lagb, hipMemcpyDeviceToDevice, s->stream));
    return LBW_OK;
}

lbw_status lbw_step_record(lbw_sim *s, int nsteps, void *dev, size_t stride)
{
    if (!s || !dev) return fail(s, LBW_ERR_ARG, "NULL argument");
    if (!s->initialized) return fail(s, LBW_ERR_STATE, "init_plasma first");
    if (nsteps < 0) return fail(s, LBW_ERR_ARG, "nsteps must be >= 0");
    if (((uintptr_t)dev % ALIGN) != 0) return fail(s, LBW_ERR_ARG, "device buffer must be 256-byte aligned");
    const DevStateLayout d = dev_state_layout(s);
    if (stride < d.total || stride % ALIGN != 0)
        return fail(s, LBW_ERR_ARG, "stride must be a multiple of 256 of at least lbw_state_device_bytes()");
    if (nsteps == 0) return LBW_OK;
    if (!s->canonical) return fail(s, LBW_ERR_STATE, "state is not canonical");
    const Ops ops = ops_for(s->g);
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    const size_t lagb = (size_t)nlag(s->g.dims, s->g.closure) * nc * 8;
    char *base = (char *)dev;
    double *stage = (double *)(s->ws + s->L.stage);
    for (int m = 0; m < nsteps; ++m) {
        // fused step from the canonical state (the simulation's own buffers,
        // then the previous record) into the workspace's other buffers
        StepArgs a = base_args(s);
        set_io(s, a);
        if (m > 0) {
            const char *in = base + (size_t)(m - 1) * stride;
            a.src = in + d.pop;
            a.ez_in = (const double *)(in + d.fld[0]);
            a.ex_in = (const double *)(in + d.fld[1]);
            a.by_in = (const double *)(in + d.fld[2]);
        }
        a.do_pull = 0;
        a.do_maxwell = 0;
        a.lag_init = s->lag_valid ? 0 : 1;
        ops.step(a, s->stream);
        s->lag_valid = true;
        s->step++;
        // canonicalisation from the workspace into record m
        StepArgs f = base_args(s);
        char *out = base + (size_t)m * stride;
        f.src = s->ws + s->L.pop[1 - s->pcur];
        f.dst = out + d.pop;
        f.ez_in = (const double *)(s->ws + s->L.fld[1 - s->fcur][0]);
        f.ex_in = (const double *)(s->ws + s->L.fld[1 - s->fcur][1]);
        f.by_in = (const double *)(s->ws + s->L.fld[1 - s->fcur][2]);
        f.ez_out = (double *)(out + d.fld[0]);
        f.ex_out = (double *)(out + d.fld[1]);
        f.by_out = (double *)(out + d.fld[2]);
        ops.finish(f, stage, stage + nc, s->stream);
        if (lagb) HIPCHK(s, hipMemcpyAsync(out + d.lag, lag_cur(s), lagb, hipMemcpyDeviceToDevice, s->stream));
        HIPCHK(s, hipGetLastError());
    }
    // the simulation's own canonical buffers take the last record
    const char *last = base + (size_t)(nsteps - 1) * stride;
    HIPCHK(s, hipMemcpyAsync(s->ws + s->L.pop[s->pcur], last + d.pop, nc * s->L.K * s->L.Q * storage_size(s->g.storage),
                             hipMemcpyDeviceToDevice, s->stream));
    for (int f = 0; f < 3; ++f)
        HIPCHK(s, hipMemcpyAsync(s->ws + s->L.fld[s->fcur][f], last + d.fld[f], nc * 8, hipMemcpyDeviceToDevice,
                                 s->stream));
    s->canonical = true;
    return LBW_OK;
}

lbw_status lbw_step_record_post(lbw_sim *s, int nsteps, void *dev, size_t stride)
{
    if (!s || !dev) return fail(s, LBW_ERR_ARG, "NULL argument");
    if (!s->initialized) return fail(s, LBW_ERR_STATE, "init_plasma first");
    if (nsteps < 0) return fail(s, LBW_ERR_ARG, "nsteps must be >= 0");
    if (((uintptr_t)dev % ALIGN) != 0) return fail(s, LBW_ERR_ARG, "device buffer must be 256-byte aligned");
    const DevStateLayout d = dev_state_layout(s);
    if (stride < d.total || stride % ALIGN != 0)
        return fail(s, LBW_ERR_ARG, "stride must be a multiple of 256 of at least lbw_state_device_bytes()");
    if (nsteps == 0) return LBW_OK;
    if (!s->canonical) return fail(s, LBW_ERR_STATE, "state is not canonical");
    const Ops ops = ops_for(s->g);
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    char *base = (char *)dev;
    for (int m = 0; m < nsteps; ++m) {
        // the fused launches of lbw_step, reading the previous record (the
        // first one the canonical state) and writing record m
        StepArgs a = base_args(s);
        set_io(s, a);
        if (m > 0) {
            const char *in = base + (size_t)(m - 1) * stride;
            a.src = in + d.pop;
            a.ez_in = (const double *)(in + d.fld[0]);
            a.ex_in = (const double *)(in + d.fld[1]);
            a.by_in = (const double *)(in + d.fld[2]);
        }
        char *out = base + (size_t)m * stride;
        a.dst = out + d.pop;
        a.ez_out = (double *)(out + d.fld[0]);
        a.ex_out = (double *)(out + d.fld[1]);
        a.by_out = (double *)(out + d.fld[2]);
        a.do_pull = m > 0 ? 1 : 0;
        a.do_maxwell = m > 0 ? 1 : 0;
        a.lag_init = s->lag_valid ? 0 : 1;
        ops.step(a, s->stream);
        s->lag_valid = true;
        s->step++;
    }
    // canonicalisation of the last record into the simulation's own buffers
    const char *last = base + (size_t)(nsteps - 1) * stride;
    StepArgs f = base_args(s);
    f.src = last + d.pop;
    f.dst = s->ws + s->L.pop[s->pcur];
    f.ez_in = (const double *)(last + d.fld[0]);
    f.ex_in = (const double *)(last + d.fld[1]);
    f.by_in = (const double *)(last + d.fld[2]);
    f.ez_out = (double *)(s->ws + s->L.fld[s->fcur][0]);
    f.ex_out = (double *)(s->ws + s->L.fld[s->fcur][1]);
    f.by_out = (double *)(s->ws + s->L.fld[s->fcur][2]);
    double *stage = (double *)(s->ws + s->L.stage);
    ops.finish(f, stage, stage + nc, s->stream);
    HIPCHK(s, hipGetLastError());
    s->canonical = true;
    return LBW_OK;
}

lbw_status lbw_load_state_device(lbw_sim *s, const void *dev, long step)
{
    if (!s || !dev) return fail(s, LBW_ERR_ARG, "NULL argument");
    if (!s->initialized) return fail(s, LBW_ERR_STATE, "init_plasma first");
    if (((uintptr_t)dev % ALIGN) != 0) return fail(s, LBW_ERR_ARG, "device buffer must be 256-byte aligned");
    if (step < 0) return fail(s, LBW_ERR_ARG, "step must be >= 0");
    const DevStateLayout d = dev_state_layout(s);
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    const char *p = (const char *)dev;
    s->pcur = s->fcur = 0;
    HIPCHK(s, hipMemcpyAsync(s->ws + s->L.pop[0], p + d.pop, nc * s->L.K * s->L.Q * storage_size(s->g.storage),
                             hipMemcpyDeviceToDevice, s->stream));
    for (int f = 0; f < 3; ++f)
        HIPCHK(s, hipMemcpyAsync(s->ws + s->L.fld[0][f], p + d.fld[f], nc * 8, hipMemcpyDeviceToDevice, s->stream));
    const size_t lagb = (size_t)nlag(s->g.dims, s->g.closure) * nc * 8;
    s->lcur = 0;
    if (lagb) HIPCHK(s, hipMemcpyAsync(s->ws + s->L.lag, p + d.lag, lagb, hipMemcpyDeviceToDevice, s->stream));
    HIPCHK(s, hipMemsetAsync(s->ws + s->L.nonfinite, 0, 8, s->stream));
    s->step = step;
    s->lag_valid = step > 0;
    s->canonical = true;
    return LBW_OK;
}

size_t lbw_adjoint_bytes(const lbw_sim *s)
{
    if (!s) return 0;
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    return ((size_t)s->L.K * s->L.Q + 3) * nc * 8;
}

size_t lbw_adjoint_workspace_bytes(const lbw_sim *s)
{
    if (!s) return 0;
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    return ((size_t)s->L.K * s->L.Q + ADJ_SCRATCH_PLANES) * align_up(nc * 8) + align_up((size_t)s->g.nz * 16);
}

static lbw_status adj_args(lbw_sim *s, double *adj, double *grad, void *scratch, AdjArgs &a)
{
    if (!s || !adj || !grad || !scratch) return fail(s, LBW_ERR_ARG, "NULL argument");
    if (!s->initialized) return fail(s, LBW_ERR_STATE, "init_plasma first");
    if (s->g.dims != 2 || s->g.closure != LBW_LEC || s->g.geom != LBW_GEOM_SLAB)
        return fail(s, LBW_ERR_UNSUPPORTED, "the adjoint covers the 2D local-equilibrium closure in slab geometry");
    if (s->drv.nslices <= 0) return fail(s, LBW_ERR_STATE, "the driver has no slices to differentiate");
    if (((uintptr_t)scratch % ALIGN) != 0) return fail(s, LBW_ERR_ARG, "scratch must be 256-byte aligned");
    if (((uintptr_t)adj % 16) != 0) return fail(s, LBW_ERR_ARG, "adj must be 16-byte aligned");
    const size_t nc = (size_t)s->g.nz * s->g.nx;
    a = AdjArgs{};
    a.lf = adj;
    a.lez = adj + (size_t)s->L.K * s->L.Q * nc;
    a.lex = a.lez + nc;
    a.lby = a.lex + nc;
    char *p = (char *)scratch;
    const size_t pl = align_up(nc * 8);
    a.s_fs = (double *)p; p += (size_t)s->L.K * s->L.Q * pl;
    double *pls[ADJ_SCRATCH_PLANES];
    for (int k = 0; k < ADJ_SCRATCH_PLANES; ++k) { pls[k] = (double *)p; p += pl; }
    a.s_byt = pls[0]; a.s_fz = pls[1]; a.s_fx = pls[2]; a.s_enz = pls[3]; a.s_enx = pls[4];
    a.s_bny = pls[5]; a.s_bht = pls[6]; a.s_ab = pls[7]; a.s_bhf = pls[10]; a.s_x = pls[11];
    // s_ab spans planes 7, 8, 9 (one per advected scalar, indexed k * ncell
    // from plane 7: within the three planes since a plane is >= ncell values)
    a.aref = (const double *)(s->ws + s->L.aref);
    a.grad = grad;
    a.nz = s->g.nz; a.nx = s->g.nx; a.ncell = (int)nc; a.bcz = s->g.bc_z; a.bcx = s->g.bc_x;
    a.delta = s->g.delta; a.dt = s->g.dt; a.omega = 1.0 / s->g.tau_tilde; a.lam = s->g.delta / s->g.dt;
    a.mu = s->mu; a.a_lec = (1.0 + 0.5 * s->g.dvel) * s->mu; a.two_over_d = 2.0 / s->g.dvel;
    a.dvel = s->g.dvel;
    a.dcode = s->g.dvel == 1.0 ? 1 : (s->g.dvel == 3.0 ? 3 : 0);
    a.drv = s->drv;
    return LBW_OK;
}

extern "C++" {
// Columns [i0, i1) of the grid that can hold the slice span at time t for
// positions (i + zoff) delta (one column of margin each side).
static void slice_window(const AdjArgs &a, double t, double zoff, int &i0, int &i1)
{
    const double lo = (a.drv.slice_zmin + a.drv.z0 + t) / a.delta - zoff;
    const double hi = (a.drv.slice_zmax + a.drv.z0 + t) / a.delta - zoff;
    i0 = (int)std::floor(lo) - 1;
    i1 = (int)std::ceil(hi) + 2;
    i0 = i0 < 0 ? 0 : (i0 > a.nz ? a.nz : i0);
    i1 = i1 < i0 ? i0 : (i1 > a.nz ? a.nz : i1);
}

template <class ST>
static void adj_step_launch(const AdjArgs &a, double *col, hipStream_t st, bool pulled_n, bool pulled_n1)
{
    const int nb = (a.ncell + 255) / 256;
    if (pulled_n1) hipLaunchKernelGGL((k_adj_maxwell<ST, true>), dim3(nb), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_adj_maxwell<ST, false>), dim3(nb), dim3(256), 0, st, a);
    // slice derivatives read the adjoint of E^{n+1} before it is overwritten
    const double th = (a.step + 0.5) * a.dt;
    int i0, i1;
    slice_window(a, th, 0.5, i0, i1);
    if (i1 > i0) {
        hipLaunchKernelGGL(k_adj_drv_cols, dim3(i1 - i0), dim3(256), 0, st, a, (const double *)a.lez, th, 0.5, i0,
                           col);
        hipLaunchKernelGGL(k_adj_slices, dim3((i1 - i0 + 255) / 256), dim3(256), 0, st, a, (const double *)col, i0, i1,
                           a.dt);
    }
    hipLaunchKernelGGL(k_adj_stream, dim3(nb), dim3(256), 0, st, a);
    if (pulled_n) hipLaunchKernelGGL((k_adj_collide<ST, true>), dim3(nb), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_adj_collide<ST, false>), dim3(nb), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_adj_bh, dim3(nb), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_adj_fields, dim3(nb), dim3(256), 0, st, a);
}
}  // extern "C++"

// One reverse step: pops_n holds state n's populations (canonical, or the
// post-collision values of step n - 1 when pulled_n), pops_n1 state n + 1's
// (likewise), fields holds state n's E^n and B^{n-1/2}.
static lbw_status adjoint_step(lbw_sim *s, const char *pops_n, bool pulled_n, const char *pops_n1, bool pulled_n1,
                               const char *fields, long n, double *adj, double *grad, void *scratch)
{
    AdjArgs a;
    lbw_status rc = adj_args(s, adj, grad, scratch, a);
    if (rc != LBW_OK) return rc;
    if (n < 0) return fail(s, LBW_ERR_ARG, "step must be >= 0");
    const DevStateLayout d = dev_state_layout(s);
    a.fn = pops_n + d.pop;
    a.fn1 = pops_n1 + d.pop;
    a.ez = (const double *)(fields + d.fld[0]);
    a.ex = (const double *)(fields + d.fld[1]);
    a.by = (const double *)(fields + d.fld[2]);
    a.step = n;
    double *col = (double *)((char *)scratch + ((size_t)s->L.K * s->L.Q + ADJ_SCRATCH_PLANES) *
                                                   align_up((size_t)a.ncell * 8));
    if (s->g.storage == LBW_FP64) adj_step_launch<double>(a, col, s->stream, pulled_n, pulled_n1);
    else if (s->g.storage == LBW_FP32) adj_step_launch<float>(a, col, s->stream, pulled_n, pulled_n1);
    else adj_step_launch<__half>(a, col, s->stream, pulled_n, pulled_n1);
    HIPCHK(s, hipGetLastError());
    return LBW_OK;
}

lbw_status lbw_adjoint_step(lbw_sim *s, const void *state_n, const void *state_n1, long n, double *adj,
                            double *grad, void *scratch)
{
    if (s && (!state_n || !state_n1)) return fail(s, LBW_ERR_ARG, "NULL state");
    return adjoint_step(s, (const char *)state_n, false, (const char *)state_n1, false, (const char *)state_n, n,
                        adj, grad, scratch);
}

lbw_status lbw_adjoint_step_post(lbw_sim *s, const void *pops_n, int pops_n_post, const void *rec_n, long n,
                                 double *adj, double *grad, void *scratch)
{
    if (s && (!pops_n || !rec_n)) return fail(s, LBW_ERR_ARG, "NULL state");
    return adjoint_step(s, (const char *)pops_n, pops_n_post != 0, (const char *)rec_n, true, (const char *)rec_n,
                        n, adj, grad, scratch);
}

lbw_status lbw_adjoint_init_fields(lbw_sim *s, const double *adj, double *grad, void *scratch)
{
    AdjArgs a;
    lbw_status rc = adj_args(s, (double *)adj, grad, scratch, a);
    if (rc != LBW_OK) return rc;
    double *col = (double *)((char *)scratch + ((size_t)s->L.K * s->L.Q + ADJ_SCRATCH_PLANES) *
                                                   align_up((size_t)a.ncell * 8));
    // E_x(0) at zeta = i delta - z0; B_y(-dt/2) at zeta = (i + 1/2) delta - z0 + dt/2
    int i0, i1;
    slice_window(a, 0.0, 0.0, i0, i1);
    if (i1 > i0) {
        hipLaunchKernelGGL(k_adj_init_cols, dim3(i1 - i0), dim3(256), 0, s->stream, a, (const double *)a.lex, 0.0,
                           0.0, i0, col);
        hipLaunchKernelGGL(k_adj_slices, dim3((i1 - i0 + 255) / 256), dim3(256), 0, s->stream, a, (const double *)col, i0,
                           i1, 1.0);
    }
    slice_window(a, -0.5 * a.dt, 0.5, i0, i1);
    if (i1 > i0) {
        hipLaunchKernelGGL(k_adj_init_cols, dim3(i1 - i0), dim3(256), 0, s->stream, a, (const double *)a.lby,
                           -0.5 * a.dt, 0.5, i0, col);
        hipLaunchKernelGGL(k_adj_slices, dim3((i1 - i0 + 255) / 256), dim3(256), 0, s->stream, a, (const double *)col, i0,
                           i1, 1.0);
    }
    HIPCHK(s, hipGetLastError());
    return LBW_OK;
}

}  // extern "C"
