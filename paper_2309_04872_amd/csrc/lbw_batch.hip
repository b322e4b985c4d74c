// lbw_batch.hip -- batched 1D parameter scans: many independent 1D runs of
// the moment-matching LB wake scheme advanced by one persistent launch.
//
// One workgroup owns one instance for the whole launch. It sweeps its nodes
// in passes of (threads x nodes-per-thread) nodes, separates time steps with a
// workgroup barrier and finishes on the canonical state (f^n, E^n) inside the
// same launch. The per-node arithmetic is the 1D fused step of
// lbw_kernels.hpp: pull streaming (Sec. 2.1, eq. open-bc), moments, LEC
// (Sec. 3.1) or WARMC (Sec. 4.1) recovery, forces, the E_z update from the
// plasma and bunch currents (Sec. 5) and the BGK collision with the source of
// eq. lsource. Everything an instance needs between launches (buffer parity,
// step counter, whether its lagged values exist) lives in device memory, so a
// launch has no per-call argument but the step count and can be replayed from
// a HIP graph.
#include "../../include/lbwake.h"
#include "lbw_kernels.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

using namespace lbw;

namespace {

constexpr int MAX_INST = 65536;
// Steps per pass of the batched kernel after the first step (temporal
// blocking). Measured on the 256-instance scan (1024 threads, per step): 112.3
// us with one step per pass, 73.1 with 2, 54.6 with 4, 44.2 with 8, 42.5 with
// 16: the longest warm-closure instance bounds the launch, and each pass over
// one of its tiles pays a memory round trip that the deeper pass shares.
#ifndef LBW_BATCH_DEPTH
#define LBW_BATCH_DEPTH 16
#endif
constexpr int BATCH_DEPTH = LBW_BATCH_DEPTH;
constexpr int PAD = 64;  // node padding of every plane (one wavefront)
constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// Per-instance constants (device, read-only in the step kernel).
struct BInst {
    int nz, nzp, closure, bc, dcode, K;
    size_t pop, fld, lag;  // element offsets of its populations, E_z, lagged values
    double delta, dt, inv2d, omega, lam, mu, a_lec, two_over_d, dvel;
    Driver drv;
};

// Per-instance mutable state (device); written only by the instance's own
// workgroup at the end of a launch.
struct BState {
    long step;      // steps taken
    int cur;        // population buffer holding the canonical f^n
    int lag_valid;  // warm closure lagged values exist
    int nonfinite;  // non-finite nodes at the end of the last launch
    int ecur;       // E_z / lagged-value buffer holding the current values
    int pad[2];
};

// Work of each workgroup: items woff[w] .. woff[w + 1] - 1 of `items`, each
// (instance, part, parts), run one after another. With one workgroup per
// instance every list holds one whole instance (part 0 of 1), longest first.
// Under the split schedule a workgroup's list starts with at most one part of
// a shared instance, followed by whole short instances, so that all parts of
// every shared instance run at the same time.
struct BatchArgs {
    const BInst *inst;
    const int *woff, *items;
    unsigned int *bar;  // per instance (arrivals, generation) of its parts' barrier
    double *pop0, *pop1, *ez, *lag;
    BState *st;
    int nsteps;
};

// Barrier among the `parts` workgroups that share one instance under the
// split schedule. Only valid when all of them are resident at once, which the
// cooperative launch of that schedule guarantees. Arrivals count up to parts
// and return to zero; the last arrival bumps the generation the others wait
// on, so the barrier needs no reset between launches. The workgroup barrier
// first makes every wave's stores complete in L2 (the L1 writes through);
// thread 0's agent-scope release then writes the L2 back for the other XCDs,
// and its acquire invalidates this CU's L1 and the L2's stale lines before
// the second workgroup barrier lets the other waves load. One thread per
// workgroup does the cache maintenance: it acts on whole caches.
__device__ __forceinline__ void instance_barrier(unsigned int *bar, int parts)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned int gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned int arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == (unsigned int)parts - 1u) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bar[1], gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen)
                __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
    }
    __syncthreads();
}

// LDS for the recovered quantities whose z-derivatives the forces need:
// LEC phi | WARMC theta^0z, theta^zz, lambda u_z, one value per slot of a
// pass (its nodes plus one ring node on each side).
template <int T, int CPT> struct Lds {
    double g[3][T * CPT];
    double xc[4][2][T * CPT];  // multi-step pass: post-collision +z / -z populations
    int bad;
};

template <int CL> struct Node1 {
    static constexpr int K = NScal<1, CL>::K;
    double s[K][3];
    double A[K];
    double uz;
    WarmRec w;
};

// Store a node's K x 3 populations in the layout of lbw_device.hpp (Pops).
template <int CL, class N>
__device__ __forceinline__ void store_node(double *dst, size_t nzp, int z, const N &nd)
{
    constexpr int K = NScal<1, CL>::K;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = nd.s[k][q];
        Pops<double, K, 3>::template st_all<false>(dst, q, nzp, z, v);
    }
}

template <int CL>
__device__ __forceinline__ void pull_node(const BInst &P, const double *src, int gz, bool do_pull,
                                          Node1<CL> &nd)
{
    using L = Lattice<1>;
    constexpr int K = NScal<1, CL>::K;
    const size_t nzp = (size_t)P.nzp;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int c = fix_node(do_pull ? gz - L::ez(q) : gz, P.nz, P.bc);
        double v[K];
        Pops<double, K, 3>::ld_all(src, q, nzp, c, v);
#pragma unroll
        for (int k = 0; k < K; ++k) nd.s[k][q] = v[k];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) acc += nd.s[k][q];
        nd.A[k] = 0.0 + acc;
    }
}

// Recovery of one node; writes the quantities the forces differentiate into
// LDS slot r.
template <int CL, int T, int CPT>
__device__ __forceinline__ void recover_node(const BInst &P, Node1<CL> &nd, Lds<T, CPT> &sh, int r)
{
    if constexpr (CL == LEC) {
        LecRec l;
        lec_recover(nd.A[0], nd.A[1], 0.0, P.a_lec, P.dcode, P.two_over_d, l);
        nd.uz = l.uz;
        sh.g[0][r] = l.phi;
    } else {
        warm_recover<1>(nd.A, nd.w);
        nd.uz = nd.w.uz;
        sh.g[0][r] = nd.w.th0z;
        sh.g[1][r] = nd.w.thzz;
        sh.g[2][r] = nd.w.luz;
    }
}

// Forcing (LEC: eq. lb-ade-lec-comps-F; WARMC: eq. lb-ade-warmc-comps-F, 1D,
// time derivatives against the lagged values) and BGK collision with source
// of one node whose E_z is already updated; rp / rm are the LDS slots of its
// +z / -z neighbours. lag_out receives the values lagged for the next step.
template <int CL, int T, int CPT>
__device__ __forceinline__ void force_collide(const BInst &P, Node1<CL> &v, double Ez, const double *lag_in,
                                              bool lag_init, double *lag_out, const Lds<T, CPT> &sh, int rp,
                                              int rm)
{
    constexpr int K = NScal<1, CL>::K;
    const double n = v.A[0], uz = v.uz, dt = P.dt;
    auto Dz = [&](int g) { return (sh.g[g][rp] - sh.g[g][rm]) * P.inv2d; };
    double F[K];
    if constexpr (CL == LEC) {
        F[0] = 0.0;
        F[1] = -P.mu * Dz(0) - n * Ez;
    } else {
        const double th0z = v.w.th0z, thzz = v.w.thzz, luz = v.w.luz, th00 = v.w.th00;
        const double l00 = lag_init ? th00 : lag_in[0], l0z = lag_init ? th0z : lag_in[1];
        const double lluz = lag_init ? luz : lag_in[2];
        lag_out[0] = th00;
        lag_out[1] = th0z;
        lag_out[2] = luz;
        const double idt = 1.0 / dt;
        F[0] = 0.0;
        F[1] = -(th00 - l00) * idt - Dz(0) - n * (Ez * uz);
        F[2] = -(th0z - l0z) * idt - Dz(1) - n * Ez;
        F[3] = -2.0 * th0z * ((luz - lluz) * idt) - 2.0 * thzz * Dz(2) - 2.0 * (Ez * th0z);
    }
    const double zero[K] = {};
    collide_all<1, K, double>(v.s, v.A, zero, F, uz, 0.0, P.lam, P.omega, dt);
}

// Nodes a pass owns: each of the T*CPT slots recovers one node (slot r holds
// node base - 1 + r), the first and last slots being the ring that the
// forces' central differences need; the slots in between collide.
template <int T, int CPT> constexpr int pass_width() { return T * CPT - 2; }

// One pass of the fused step over nodes [base, base + pass_width) of one instance.
template <int CL, int T, int CPT>
__device__ __forceinline__ void step_pass(const BInst &P, const double *src, double *dst, double *ez,
                                          double *lag, int base, bool do_pull, bool do_maxwell,
                                          bool lag_init, long step, Lds<T, CPT> &sh)
{
    constexpr int K = NScal<1, CL>::K;
    constexpr int W = pass_width<T, CPT>();
    const int tid = threadIdx.x;
    const int nz = P.nz;
    const size_t nzp = (size_t)P.nzp;
    Node1<CL> nd[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) pull_node<CL>(P, src, base - 1 + tid + j * T, do_pull, nd[j]);
    // the own nodes' E_z and lagged values are loaded with the populations, so
    // that one memory round trip per pass serves them all
    double ezv[CPT], lgv[CPT][3];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int slot = tid + j * T, gz = base - 1 + slot;
        const bool own = slot >= 1 && slot <= W && gz < nz;
        ezv[j] = own ? ez[gz] : 0.0;
#pragma unroll
        for (int g = 0; g < 3; ++g)
            lgv[j][g] = (CL == WARMC && own && !lag_init) ? lag[(size_t)g * nzp + gz] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) recover_node<CL, T, CPT>(P, nd[j], sh, tid + j * T);
    __syncthreads();
    const double dt = P.dt;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int slot = tid + j * T;
        const int gz = base - 1 + slot;
        if (slot < 1 || slot > W || gz >= nz) continue;
        Node1<CL> &v = nd[j];
        const double n = v.A[0], uz = v.uz;
        double Ez = ezv[j];
        if (do_maxwell) {
            const double jb = driver_density<1>(P.drv, gz * P.delta, 0.0, (step - 0.5) * dt);
            Ez = Ez + dt * (n * uz + jb);
        }
        ez[gz] = Ez;
        const int rp = map_node(gz + 1, nz, P.bc) - (base - 1);
        const int rm = map_node(gz - 1, nz, P.bc) - (base - 1);
        double lnew[3];
        force_collide<CL, T, CPT>(P, v, Ez, lgv[j], lag_init, lnew, sh, rp, rm);
        if constexpr (CL == WARMC) {
#pragma unroll
            for (int g = 0; g < 3; ++g) lag[(size_t)g * nzp + gz] = lnew[g];
        }
        store_node<CL>(dst, nzp, gz, v);
    }
    __syncthreads();  // the next pass reuses the LDS slots
}

// S steps in one pass (temporal blocking). Slot r of the NS = T*CPT slots
// holds node fix(base - (2S - 1) + r) (the copy or wrap rule of the
// boundary): step 0 of the pass runs on slots [1, NS - 1); each later step m
// takes its +z / -z populations from the previous one through LDS (the rest
// population, E_z and the lagged values stay in registers), recovers on
// slots [2m, NS - 2m) and collides on [2m + 1, NS - 2m - 1), so the last step
// writes the own slots, nodes [base, base + NS - 4S + 2). Populations, E_z and
// lagged values are read once and written once per S steps; E_z and the
// lagged values are read from one buffer and written to the other, because
// the ring slots read values that a neighbouring pass of the same sweep
// updates.
template <int T, int CPT, int S> constexpr int passs_width() { return T * CPT - 4 * S + 2; }

template <int CL, int T, int CPT, int S>
__device__ __forceinline__ void step_passs(const BInst &P, const double *src, double *dst, const double *ez_in,
                                           double *ez_out, const double *lag_in, double *lag_out, int base,
                                           long step, Lds<T, CPT> &sh)
{
    constexpr int K = NScal<1, CL>::K;
    constexpr int NS = T * CPT;
    static_assert(S >= 2 && passs_width<T, CPT, S>() > 0, "pass depth");
    const int tid = threadIdx.x;
    const int nz = P.nz, bc = P.bc;
    const size_t nzp = (size_t)P.nzp;
    const double dt = P.dt;
    const int off = base - (2 * S - 1);  // node of slot 0 before the boundary rule
    // LDS slot of the node next to slot r's node (r's node is fix(off + r))
    auto nb = [&](int r, int d) {
        return bc == BC_PERIODIC ? r + d : map_node(fix_node(off + r, nz, bc) + d, nz, bc) - off;
    };
    // ---- step 0 on every slot: pull, E_z, lagged values, recovery into LDS
    Node1<CL> nd[CPT];
    double ezv[CPT], lgv[CPT][3];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int z = fix_node(off + tid + j * T, nz, bc);
        pull_node<CL>(P, src, z, true, nd[j]);
        ezv[j] = ez_in[z];
#pragma unroll
        for (int g = 0; g < 3; ++g) lgv[j][g] = CL == WARMC ? lag_in[(size_t)g * nzp + z] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) recover_node<CL, T, CPT>(P, nd[j], sh, tid + j * T);
    __syncthreads();
    double rest[CPT][K];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int r = tid + j * T;
        if (r < 1 || r >= NS - 1) continue;
        const int z = fix_node(off + r, nz, bc);
        Node1<CL> &v = nd[j];
        const double jb = driver_density<1>(P.drv, z * P.delta, 0.0, (step - 0.5) * dt);
        ezv[j] = ezv[j] + dt * (v.A[0] * v.uz + jb);
        double lnew[3];
        force_collide<CL, T, CPT>(P, v, ezv[j], lgv[j], false, lnew, sh, nb(r, 1), nb(r, -1));
#pragma unroll
        for (int g = 0; g < 3; ++g) lgv[j][g] = lnew[g];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            rest[j][k] = v.s[k][0];
            sh.xc[k][0][r] = v.s[k][1];
            sh.xc[k][1][r] = v.s[k][2];
        }
    }
    __syncthreads();  // movers in LDS; every value of g has been read
    // ---- steps 1 .. S - 1
    for (int m = 1; m < S; ++m) {
        // pull from LDS on slots [2m, NS - 2m), recovery into LDS
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int r = tid + j * T;
            if (r < 2 * m || r >= NS - 2 * m) continue;
            Node1<CL> &v = nd[j];
            const int rm = nb(r, -1), rp = nb(r, 1);  // sources of +z and -z movers
#pragma unroll
            for (int k = 0; k < K; ++k) {
                v.s[k][0] = rest[j][k];
                v.s[k][1] = sh.xc[k][0][rm];
                v.s[k][2] = sh.xc[k][1][rp];
                double acc = 0.0;
#pragma unroll
                for (int q = 0; q < 3; ++q) acc += v.s[k][q];
                v.A[k] = 0.0 + acc;
            }
            recover_node<CL, T, CPT>(P, v, sh, r);
        }
        __syncthreads();  // g visible; every mover has been read
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int r = tid + j * T;
            if (r < 2 * m + 1 || r >= NS - 2 * m - 1) continue;
            const int z = fix_node(off + r, nz, bc);
            Node1<CL> &v = nd[j];
            const double jb = driver_density<1>(P.drv, z * P.delta, 0.0, (step + m - 0.5) * dt);
            ezv[j] = ezv[j] + dt * (v.A[0] * v.uz + jb);
            double lnew[3];
            force_collide<CL, T, CPT>(P, v, ezv[j], lgv[j], false, lnew, sh, nb(r, 1), nb(r, -1));
            if (m < S - 1) {
#pragma unroll
                for (int g = 0; g < 3; ++g) lgv[j][g] = lnew[g];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    rest[j][k] = v.s[k][0];
                    sh.xc[k][0][r] = v.s[k][1];
                    sh.xc[k][1][r] = v.s[k][2];
                }
            } else {
                const int zo = off + r;
                if (zo < nz) {
                    ez_out[zo] = ezv[j];
                    if constexpr (CL == WARMC) {
#pragma unroll
                        for (int g = 0; g < 3; ++g) lag_out[(size_t)g * nzp + zo] = lnew[g];
                    }
                    store_node<CL>(dst, nzp, zo, v);
                }
            }
        }
        __syncthreads();  // movers in LDS (or the pass done); every value of g has been read
    }
}

// Finish: stream f*^{n-1} into f^n, E^n = E^{n-1} + dt (n u + n_b) at
// t^{n-1/2}; returns the number of non-finite nodes this thread saw.
template <int CL, int T, int CPT>
__device__ __forceinline__ int finish_pass(const BInst &P, const double *src, double *dst, double *ez,
                                           int base, long step)
{
    constexpr int K = NScal<1, CL>::K;
    const size_t nzp = (size_t)P.nzp;
    int bad = 0;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int gz = base + threadIdx.x + j * T;
        if (gz >= P.nz) continue;
        Node1<CL> v;
        pull_node<CL>(P, src, gz, true, v);
        store_node<CL>(dst, nzp, gz, v);
        double uz;
        if constexpr (CL == LEC) {
            LecRec l;
            lec_recover(v.A[0], v.A[1], 0.0, P.a_lec, P.dcode, P.two_over_d, l);
            uz = l.uz;
        } else {
            warm_recover<1>(v.A, v.w);
            uz = v.w.uz;
        }
        const double jb = driver_density<1>(P.drv, gz * P.delta, 0.0, (step - 0.5) * P.dt);
        const double e = ez[gz] + P.dt * (v.A[0] * uz + jb);
        ez[gz] = e;
        if (!isfinite(v.A[0]) || !isfinite(uz) || !isfinite(e)) ++bad;
    }
    return bad;
}

// part / parts: under the split schedule the instance's workgroups take
// contiguous runs of every sweep's tiles and meet at instance_barrier after
// each sweep (the next sweep reads ring nodes another workgroup wrote); with
// parts = 1 the workgroup barrier that ends every pass is enough.
template <int CL, int T, int CPT, bool SPLIT>
__device__ void run_instance(const BatchArgs &a, const BInst &P, BState *st, Lds<T, CPT> &sh, int part, int parts,
                             unsigned int *bar)
{
    constexpr int W = pass_width<T, CPT>();
    constexpr int W2 = passs_width<T, CPT, 2>();
    constexpr int WD = passs_width<T, CPT, BATCH_DEPTH>();
    constexpr int WF = T * CPT;  // finish passes own every slot
    const int nsteps = a.nsteps;
    int cur = st->cur, ec = st->ecur;
    const long step0 = st->step;
    const bool lag_init = st->lag_valid == 0;
    const size_t nzp = (size_t)P.nzp;
    double *pop[2] = {a.pop0 + P.pop, a.pop1 + P.pop};
    double *ez[2] = {a.ez + P.fld, a.ez + P.fld + nzp};
    double *lag[2] = {a.lag + P.lag, a.lag + P.lag + (CL == WARMC ? NLAG1 * nzp : 0)};
    // this part's run [b0, b1) of a sweep's tile bases (tiles of `width` nodes)
    auto span = [&](int width, int &b0, int &b1) {
        if constexpr (!SPLIT) {
            b0 = 0;
            b1 = P.nz;
        } else {
            const long nt = (P.nz + width - 1) / width;
            b0 = (int)(nt * part / parts) * width;
            b1 = (int)(nt * (part + 1) / parts) * width;
            if (b1 > P.nz) b1 = P.nz;
        }
    };
    auto sweep_done = [&]() {
        if constexpr (SPLIT)
            if (parts > 1) instance_barrier(bar, parts);
    };
    if (SPLIT && parts > 1 && part == 0 && threadIdx.x == 0) st->nonfinite = 0;  // summed by every part below
    int b0, b1;
    // schedule: the first step from the canonical state, then passes of
    // BATCH_DEPTH steps, pairs of steps for what is left, then a last single
    // step if one is left. Every pass ends on a barrier, so each step's stores
    // are visible to the whole workgroup before the next step reads its
    // neighbours.
    long s = 0;
    if (nsteps > 0) {
        span(W, b0, b1);
        for (int base = b0; base < b1; base += W)
            step_pass<CL, T, CPT>(P, pop[cur], pop[cur ^ 1], ez[ec], lag[ec], base, false, false, lag_init,
                                  step0, sh);
        sweep_done();
        cur ^= 1;
        s = 1;
    }
    for (; s > 0 && s + BATCH_DEPTH <= nsteps; s += BATCH_DEPTH) {
        span(WD, b0, b1);
        for (int base = b0; base < b1; base += WD)
            step_passs<CL, T, CPT, BATCH_DEPTH>(P, pop[cur], pop[cur ^ 1], ez[ec], ez[ec ^ 1], lag[ec],
                                                lag[ec ^ 1], base, step0 + s, sh);
        sweep_done();
        cur ^= 1;
        ec ^= 1;
    }
    for (; s > 0 && s + 2 <= nsteps; s += 2) {
        span(W2, b0, b1);
        for (int base = b0; base < b1; base += W2)
            step_passs<CL, T, CPT, 2>(P, pop[cur], pop[cur ^ 1], ez[ec], ez[ec ^ 1], lag[ec], lag[ec ^ 1], base,
                                      step0 + s, sh);
        sweep_done();
        cur ^= 1;
        ec ^= 1;
    }
    if (s < nsteps) {
        span(W, b0, b1);
        for (int base = b0; base < b1; base += W)
            step_pass<CL, T, CPT>(P, pop[cur], pop[cur ^ 1], ez[ec], lag[ec], base, true, true, false, step0 + s,
                                  sh);
        sweep_done();
        cur ^= 1;
    }
    if (threadIdx.x == 0) sh.bad = 0;
    __syncthreads();
    int bad = 0;
    span(WF, b0, b1);
    for (int base = b0; base < b1; base += WF)
        bad += finish_pass<CL, T, CPT>(P, pop[cur], pop[cur ^ 1], ez[ec], base, step0 + nsteps);
    if (bad) atomicAdd(&sh.bad, bad);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (SPLIT && parts > 1) {
            if (sh.bad) atomicAdd(&st->nonfinite, sh.bad);
        } else {
            st->nonfinite = sh.bad;
        }
        if (part == 0) {
            st->cur = cur ^ 1;
            st->ecur = ec;
            st->step = step0 + nsteps;
            st->lag_valid = 1;
        }
    }
}

// One workgroup per instance (workgroup w runs the instance of work item w).
template <int T, int CPT>
__global__ __launch_bounds__(T) void k_batch1d(BatchArgs a)
{
    __shared__ Lds<T, CPT> sh;
    const int i = a.items[3 * blockIdx.x];
    const BInst P = a.inst[i];
    if (P.closure == LEC)
        run_instance<LEC, T, CPT, false>(a, P, a.st + i, sh, 0, 1, nullptr);
    else
        run_instance<WARMC, T, CPT, false>(a, P, a.st + i, sh, 0, 1, nullptr);
}

// Split schedule: each workgroup runs its work list (a part of a shared
// instance first, then whole short instances).
template <int T, int CPT>
__global__ __launch_bounds__(T) void k_batch1d_split(BatchArgs a)
{
    __shared__ Lds<T, CPT> sh;
    const int end = a.woff[blockIdx.x + 1];
    for (int it = a.woff[blockIdx.x]; it < end; ++it) {
        const int i = a.items[3 * it], part = a.items[3 * it + 1], parts = a.items[3 * it + 2];
        const BInst P = a.inst[i];
        unsigned int *bar = a.bar + 2 * (size_t)i;
        if (P.closure == LEC)
            run_instance<LEC, T, CPT, true>(a, P, a.st + i, sh, part, parts, bar);
        else
            run_instance<WARMC, T, CPT, true>(a, P, a.st + i, sh, part, parts, bar);
        __syncthreads();  // the next item reuses the LDS
    }
}

// Launch configurations: threads per workgroup, nodes per thread per pass,
// and the schedule: one workgroup per instance (split = 0; a plain launch,
// no workgroup waits on another), or split = 1: every workgroup that can be
// resident at once, the long instances shared by several of them that meet
// at a barrier after each sweep (a cooperative launch, whose grid the
// occupancy query proves co-resident).
// (1024 threads with two nodes each would spill registers at the 128-VGPR
// limit of 1024-thread workgroups)
struct Config {
    int threads, cpt, split;
};
const Config CONFIGS[] = {{256, 1, 0}, {256, 2, 0}, {512, 1, 0}, {512, 2, 0}, {1024, 1, 0},
                          {256, 2, 1}, {512, 1, 1}, {512, 2, 1}, {1024, 1, 1}};
constexpr int NCONFIG = sizeof(CONFIGS) / sizeof(CONFIGS[0]);
constexpr int MAX_SPLIT_WG = 8192;  // workgroups of a split launch (resident ones only)

template <int T, int CPT> const void *kernel_of(bool split)
{
    return split ? (const void *)k_batch1d_split<T, CPT> : (const void *)k_batch1d<T, CPT>;
}
const void *config_kernel(int ci)
{
    const Config &c = CONFIGS[ci];
    const bool sp = c.split != 0;
    if (c.threads == 256) return c.cpt == 1 ? kernel_of<256, 1>(sp) : kernel_of<256, 2>(sp);
    if (c.threads == 512) return c.cpt == 1 ? kernel_of<512, 1>(sp) : kernel_of<512, 2>(sp);
    return kernel_of<1024, 1>(sp);
}

hipError_t launch_config(int ci, const BatchArgs &a, int nblocks, hipStream_t s)
{
    const Config &c = CONFIGS[ci];
    BatchArgs aa = a;
    void *args[] = {&aa};
    if (c.split) return hipLaunchCooperativeKernel(config_kernel(ci), dim3(nblocks), dim3(c.threads), args, 0, s);
    return hipLaunchKernel(config_kernel(ci), dim3(nblocks), dim3(c.threads), args, 0, s);
}

// Deep-pass tile width of a configuration (nodes a workgroup owns per pass).
int deep_width(const Config &c) { return c.threads * c.cpt - 4 * BATCH_DEPTH + 2; }

// Workgroups of configuration ci that can all be resident (0: no
// cooperative launch on this device).
int resident_workgroups(int ci)
{
    int dev = 0, coop = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, config_kernel(ci), CONFIGS[ci].threads, 0) != hipSuccess)
        return 0;
    return per * cus;
}

// Work lists, as woff (nwg + 1 offsets) followed by the (instance, part,
// parts) items.
struct Plan {
    std::vector<int> woff, items;
};

// One workgroup per instance, longest first.
Plan plan_whole(const std::vector<int> &order)
{
    Plan p;
    p.woff.push_back(0);
    for (int i : order) {
        p.items.insert(p.items.end(), {i, 0, 1});
        p.woff.push_back((int)p.items.size() / 3);
    }
    return p;
}

// Split schedule on nwg workgroups for the instances' deep-sweep tile counts
// (the sweeps of one launch all split in the same proportions): the smallest
// L for which instances of more than L tiles, cut into ceil(tiles / L) parts
// that each lead a workgroup, and the remaining whole instances, packed
// largest first into the least loaded workgroups, leave no workgroup with
// more than L tiles. L is then the most tiles any workgroup sweeps (one
// workgroup per instance gives the largest instance's count).
Plan plan_split(const std::vector<lbw_instance_desc> &d, const std::vector<int> &order, int width, int nwg)
{
    const int n = (int)d.size();
    std::vector<int> tiles(n);
    int hi = 1, lo = 1;
    long total = 0;
    for (int i = 0; i < n; ++i) {
        tiles[i] = (d[i].nz + width - 1) / width;
        hi = std::max(hi, tiles[i]);
        total += tiles[i];
    }
    lo = std::max<long>(1, (total + nwg - 1) / nwg);
    // try(L): the lists, or empty when L does not fit
    auto attempt = [&](int L, std::vector<std::vector<int>> &lists) {
        lists.assign(nwg, {});
        std::vector<int> load(nwg, 0);
        int w = 0;
        for (int i : order) {  // longest first: the shared instances lead their lists
            if (tiles[i] <= L) continue;
            const int parts = (tiles[i] + L - 1) / L;
            for (int j = 0; j < parts; ++j) {
                if (w >= nwg) return false;
                lists[w] = {i, j, parts};
                load[w] = (int)((long)tiles[i] * (j + 1) / parts - (long)tiles[i] * j / parts);
                ++w;
            }
        }
        for (int i : order) {
            if (tiles[i] > L) continue;
            int best = 0;
            for (int k = 1; k < nwg; ++k)
                if (load[k] < load[best]) best = k;
            if (load[best] + tiles[i] > L) return false;
            lists[best].insert(lists[best].end(), {i, 0, 1});
            load[best] += tiles[i];
        }
        return true;
    };
    std::vector<std::vector<int>> lists, best_lists;
    if (!attempt(hi, best_lists)) return plan_whole(order);  // fewer workgroups than instances
    while (lo < hi) {
        const int mid = (lo + hi) / 2;
        if (attempt(mid, lists)) {
            hi = mid;
            best_lists = lists;
        } else {
            lo = mid + 1;
        }
    }
    Plan p;
    p.woff.push_back(0);
    for (const auto &l : best_lists) {
        if (l.empty()) continue;  // unused workgroups are not launched
        p.items.insert(p.items.end(), l.begin(), l.end());
        p.woff.push_back((int)p.items.size() / 3);
    }
    return p;
}

struct BLayout {
    size_t inst, plan[2], bar, st, pop[2], ez, lag, snap_pop, snap_ez, snap_lag, snap_st, zeros, total;
    size_t pop_elems, fld_elems, lag_elems;
};

bool inst_valid(const lbw_instance_desc &d, std::string *why)
{
    auto bad = [&](const char *m) { if (why) *why = m; return false; };
    if (d.nz < 4) return bad("nz must be >= 4");
    if (d.nz > (1 << 24)) return bad("nz must be <= 2^24");
    if (d.closure != LBW_LEC && d.closure != LBW_WARMC) return bad("unknown closure");
    if (!(d.dvel > 0)) return bad("dvel must be positive");
    if (!(d.mu >= 0) || !std::isfinite(d.mu)) return bad("mu must be >= 0");
    if (!(d.delta > 0) || !(d.dt > 0)) return bad("delta and dt must be positive");
    if (d.bc != LBW_BC_OPEN && d.bc != LBW_BC_PERIODIC) return bad("unknown bc");
    if (!std::isfinite(d.alpha)) return bad("alpha must be finite");
    if (d.alpha != 0.0 && !(d.sigma_z > 0)) return bad("sigma_z must be positive");
    return true;
}

int nscal1(int closure) { return closure == LBW_LEC ? 2 : 4; }
size_t padded(int nz) { return ((size_t)nz + PAD - 1) / PAD * PAD; }

BLayout make_blayout(const lbw_instance_desc *d, int n)
{
    BLayout L{};
    size_t pe = 0, fe = 0, le = 0;
    for (int i = 0; i < n; ++i) {
        const size_t np = padded(d[i].nz);
        pe += (size_t)nscal1(d[i].closure) * 3 * np;
        fe += 2 * np;
        if (d[i].closure == LBW_WARMC) le += 2 * NLAG1 * np;
    }
    L.pop_elems = pe;
    L.fld_elems = fe;
    L.lag_elems = le;
    size_t off = 0;
    L.inst = off; off += align_up(n * sizeof(BInst));
    // work lists: one workgroup per instance (plan[0]) and the split schedule
    // (plan[1]): at most MAX_SPLIT_WG + 1 offsets and n + MAX_SPLIT_WG items
    for (int k = 0; k < 2; ++k) {
        L.plan[k] = off;
        off += align_up(((size_t)MAX_SPLIT_WG + 1 + 3 * ((size_t)n + MAX_SPLIT_WG)) * sizeof(int));
    }
    L.bar = off; off += align_up((size_t)2 * n * sizeof(unsigned int));
    L.st = off; off += align_up(n * sizeof(BState));
    L.pop[0] = off; off += align_up(pe * 8);
    L.pop[1] = off; off += align_up(pe * 8);
    L.ez = off; off += align_up(fe * 8);
    L.lag = off; off += align_up(le * 8 + 8);
    L.snap_pop = off; off += align_up(pe * 8);
    L.snap_ez = off; off += align_up(fe * 8);
    L.snap_lag = off; off += align_up(le * 8 + 8);
    L.snap_st = off; off += align_up(n * sizeof(BState));
    L.zeros = off; off += align_up(8 * 8);
    L.total = off;
    return L;
}

double lambda_rest1(double mu, double D) { return 0.5 * (D * mu + std::sqrt(D * D * mu * mu + 4.0)); }

}  // namespace

struct lbw_batch {
    std::vector<lbw_instance_desc> d;
    std::vector<BInst> inst;
    std::vector<int> order;
    BLayout L;
    char *ws;
    hipStream_t stream, capture_stream;
    hipEvent_t ev[2];
    bool ev_recorded;
    int cfg;
    int nwg;          // workgroups of the current configuration's launch
    int plan_nwg[2];  // workgroups of the plans in the workspace (one per instance; split)
    int plan1_cfg;    // configuration whose split plan is in the workspace (-1: none)
    bool initialized;
    long step;
    int cur;   // host mirror of every instance's population buffer parity
    int ecur;  // host mirror of the E_z / lagged-value buffer index
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;
    std::vector<hipGraph_t> graph_defs;
    std::string err;
};

static lbw_status bfail(lbw_batch *b, lbw_status code, const std::string &m)
{
    if (b) b->err = m;
    return code;
}

#define BHIPCHK(b, call)                                                                     \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return bfail((b), LBW_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

static BatchArgs batch_args(lbw_batch *b, int nsteps)
{
    BatchArgs a{};
    a.inst = (const BInst *)(b->ws + b->L.inst);
    const int k = CONFIGS[b->cfg].split;
    a.woff = (const int *)(b->ws + b->L.plan[k]);
    a.items = a.woff + b->plan_nwg[k] + 1;
    a.bar = (unsigned int *)(b->ws + b->L.bar);
    a.pop0 = (double *)(b->ws + b->L.pop[0]);
    a.pop1 = (double *)(b->ws + b->L.pop[1]);
    a.ez = (double *)(b->ws + b->L.ez);
    a.lag = (double *)(b->ws + b->L.lag);
    a.st = (BState *)(b->ws + b->L.st);
    a.nsteps = nsteps;
    return a;
}

// One instance seen as a single 1D run by the initialisation and read-out
// kernels shared with lbw_step: its planes are nzp nodes apart, so those
// kernels run over ncell = nzp nodes (the padding nodes are never read by
// the step).
static StepArgs instance_args(lbw_batch *b, int i)
{
    const BInst &P = b->inst[i];
    StepArgs a{};
    a.nz = P.nz;
    a.nx = 1;
    a.ncell = P.nzp;
    a.bcz = P.bc;
    a.bcx = BC_OPEN;
    a.delta = P.delta;
    a.dt = P.dt;
    a.inv2d = P.inv2d;
    a.omega = P.omega;
    a.lam = P.lam;
    a.mu = P.mu;
    a.a_lec = P.a_lec;
    a.two_over_d = P.two_over_d;
    a.dcode = P.dcode;
    a.aref = (const double *)(b->ws + b->L.zeros);
    a.drv = P.drv;
    a.step = b->step;
    a.src = (double *)(b->ws + b->L.pop[b->cur]) + P.pop;
    a.dst = nullptr;
    a.ez_in = (const double *)(b->ws + b->L.ez) + P.fld + (size_t)b->ecur * P.nzp;
    a.ez_out = (double *)(b->ws + b->L.ez) + P.fld + (size_t)b->ecur * P.nzp;
    return a;
}

extern "C" {

size_t lbw_batch_workspace_bytes(const lbw_instance_desc *d, int n)
{
    if (!d || n < 1 || n > MAX_INST) return 0;
    for (int i = 0; i < n; ++i)
        if (!inst_valid(d[i], nullptr)) return 0;
    return make_blayout(d, n).total;
}

lbw_status lbw_batch_create(const lbw_instance_desc *d, int n, void *ws, size_t ws_bytes, void *stream,
                            lbw_batch **out)
{
    if (!out) return LBW_ERR_ARG;
    *out = nullptr;
    if (!d || n < 1 || n > MAX_INST) return LBW_ERR_ARG;
    for (int i = 0; i < n; ++i) {
        if (!inst_valid(d[i], nullptr)) return LBW_ERR_ARG;
        if (!(d[i].tau_tilde > 0.5)) return LBW_ERR_UNSTABLE;
        if (d[i].dt > d[i].delta * (1.0 + 1e-12)) return LBW_ERR_UNSTABLE;
    }
    const BLayout L = make_blayout(d, n);
    if (!ws || ws_bytes < L.total || ((uintptr_t)ws % ALIGN) != 0) return LBW_ERR_WORKSPACE;
    lbw_batch *b = new lbw_batch();
    b->d.assign(d, d + n);
    b->L = L;
    b->ws = (char *)ws;
    b->stream = (hipStream_t)stream;
    b->capture_stream = nullptr;
    b->ev_recorded = false;
    b->cfg = 4;  // 1024 threads, one node per thread, one workgroup per instance
    b->nwg = n;
    b->plan_nwg[0] = n;
    b->plan_nwg[1] = 0;
    b->plan1_cfg = -1;
    b->initialized = false;
    b->step = 0;
    b->cur = 0;
    b->ecur = 0;
    size_t pe = 0, fe = 0, le = 0;
    for (int i = 0; i < n; ++i) {
        const lbw_instance_desc &q = d[i];
        BInst P{};
        P.nz = q.nz;
        P.nzp = (int)padded(q.nz);
        P.closure = q.closure;
        P.bc = q.bc;
        P.dcode = q.dvel == 1.0 ? 1 : (q.dvel == 3.0 ? 3 : 0);
        P.K = nscal1(q.closure);
        P.pop = pe;
        P.fld = fe;
        P.lag = le;
        pe += (size_t)P.K * 3 * P.nzp;
        fe += 2 * (size_t)P.nzp;  // two E_z buffers
        if (q.closure == LBW_WARMC) le += 2 * NLAG1 * (size_t)P.nzp;
        P.delta = q.delta;
        P.dt = q.dt;
        P.inv2d = 1.0 / (2.0 * q.delta);
        P.omega = 1.0 / q.tau_tilde;
        P.lam = q.delta / q.dt;
        P.mu = q.mu;
        P.a_lec = (1.0 + 0.5 * q.dvel) * q.mu;
        P.two_over_d = 2.0 / q.dvel;
        P.dvel = q.dvel;
        Driver v{};
        v.alpha = q.alpha;
        v.sigma_z = q.sigma_z;
        v.z0 = q.z0;
        v.inv2sz2 = q.sigma_z > 0 ? 1.0 / (2.0 * q.sigma_z * q.sigma_z) : 0.0;
        v.nslices = 0;
        v.slice_w = nullptr;
        P.drv = v;
        b->inst.push_back(P);
    }
    b->order.resize(n);
    std::iota(b->order.begin(), b->order.end(), 0);
    // longest first (ties by index): the longest runs start first
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](int x, int y) { return d[x].nz > d[y].nz; });
    lbw_status rc = LBW_OK;
    auto chk = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && rc == LBW_OK) rc = bfail(b, LBW_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    };
    chk(hipEventCreate(&b->ev[0]), "hipEventCreate");
    chk(hipEventCreate(&b->ev[1]), "hipEventCreate");
    chk(hipMemcpyAsync(b->ws + L.inst, b->inst.data(), n * sizeof(BInst), hipMemcpyHostToDevice, b->stream),
        "hipMemcpyAsync");
    const Plan whole = plan_whole(b->order);
    std::vector<int> buf(whole.woff);
    buf.insert(buf.end(), whole.items.begin(), whole.items.end());
    chk(hipMemcpyAsync(b->ws + L.plan[0], buf.data(), buf.size() * sizeof(int), hipMemcpyHostToDevice, b->stream),
        "hipMemcpyAsync");
    chk(hipMemsetAsync(b->ws + L.zeros, 0, 64, b->stream), "hipMemsetAsync");
    chk(hipMemsetAsync(b->ws + L.bar, 0, (size_t)2 * n * sizeof(unsigned int), b->stream), "hipMemsetAsync");
    chk(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    if (rc != LBW_OK) {
        lbw_batch_destroy(b);
        return rc;
    }
    *out = b;
    return LBW_OK;
}

void lbw_batch_destroy(lbw_batch *b)
{
    if (!b) return;
    for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    for (hipGraph_t g : b->graph_defs) (void)hipGraphDestroy(g);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    (void)hipEventDestroy(b->ev[0]);
    (void)hipEventDestroy(b->ev[1]);
    delete b;
}

const char *lbw_batch_last_error(const lbw_batch *b) { return b ? b->err.c_str() : "NULL batch"; }

long lbw_batch_step_count(const lbw_batch *b) { return b ? b->step : -1; }

lbw_status lbw_batch_init(lbw_batch *b, const double *n_init)
{
    if (!b) return LBW_ERR_ARG;
    const int n = (int)b->inst.size();
    b->initialized = false;
    b->step = 0;
    b->cur = 0;
    b->ecur = 0;
    std::vector<BState> st(n);
    for (auto &x : st) x = BState{0, 0, 0, 0, 0, {0, 0}};
    BHIPCHK(b, hipMemcpyAsync(b->ws + b->L.st, st.data(), n * sizeof(BState), hipMemcpyHostToDevice, b->stream));
    BHIPCHK(b, hipMemsetAsync(b->ws + b->L.ez, 0, b->L.fld_elems * 8, b->stream));
    BHIPCHK(b, hipMemsetAsync(b->ws + b->L.lag, 0, b->L.lag_elems * 8 + 8, b->stream));
    BHIPCHK(b, hipMemsetAsync(b->ws + b->L.bar, 0, (size_t)2 * n * sizeof(unsigned int), b->stream));
    size_t off = 0;
    std::vector<double> A;
    for (int i = 0; i < n; ++i) {
        const BInst &P = b->inst[i];
        const size_t nz = P.nz, np = P.nzp;
        const int K = P.K;
        // moments A [K][nzp] and a zero velocity [2][nzp], staged in the
        // instance's second population buffer (K x 3 x nzp >= (K + 2) x nzp)
        A.assign((size_t)(K + 2) * np, 0.0);
        for (size_t c = 0; c < np; ++c) {
            double dens = 1.0;
            if (c < nz && n_init) {
                dens = n_init[off + c];
                if (!(dens > 0.0) || !std::isfinite(dens))
                    return bfail(b, LBW_ERR_NONFINITE, "initial density must be positive and finite");
            }
            A[c] = dens;
            if (P.closure == LBW_WARMC) {
                // rest state: n lambda_0 (eq. traces3) and lambda_0 theta^zz, theta^zz = n mu
                const double l0 = lambda_rest1(P.mu, P.dvel);
                A[1 * np + c] = dens * l0;
                A[3 * np + c] = l0 * dens * P.mu;
            }
        }
        off += nz;
        double *stage = (double *)(b->ws + b->L.pop[1]) + P.pop;
        BHIPCHK(b, hipMemcpyAsync(stage, A.data(), A.size() * 8, hipMemcpyHostToDevice, b->stream));
        StepArgs a = instance_args(b, i);
        const double *uz = stage + (size_t)K * np, *ux = uz + np;
        const int nb = (int)((np + 255) / 256);
        double *dst = (double *)(b->ws + b->L.pop[0]) + P.pop;
        if (P.closure == LBW_LEC)
            hipLaunchKernelGGL((k_init_pops<1, LEC, double>), dim3(nb), dim3(256), 0, b->stream, (void *)dst,
                               (const double *)stage, uz, ux, a.aref, (int)np, P.lam);
        else
            hipLaunchKernelGGL((k_init_pops<1, WARMC, double>), dim3(nb), dim3(256), 0, b->stream,
                               (void *)dst, (const double *)stage, uz, ux, a.aref, (int)np, P.lam);
        BHIPCHK(b, hipGetLastError());
        if (P.drv.alpha != 0.0) {
            // causal field of the bunch (as lbw_init_driver with init_fields)
            StepArgs f = a;
            f.ncell = P.nz;
            double *ez = (double *)(b->ws + b->L.ez) + P.fld;
            hipLaunchKernelGGL(k_init_fields<1>, dim3((P.nz + 255) / 256), dim3(256), 0, b->stream, f, ez,
                               (double *)nullptr, (double *)nullptr);
            BHIPCHK(b, hipGetLastError());
        }
        BHIPCHK(b, hipStreamSynchronize(b->stream));  // the host staging vector is reused
    }
    b->initialized = true;
    return LBW_OK;
}

static lbw_status launch_step(lbw_batch *b, int nsteps, int use_graph)
{
    const BatchArgs a = batch_args(b, nsteps);
    const int nblocks = b->nwg;
    if (!use_graph) {
        BHIPCHK(b, launch_config(b->cfg, a, nblocks, b->stream));
        BHIPCHK(b, hipGetLastError());
        return LBW_OK;
    }
    const auto key = std::make_pair(nsteps, b->cfg);
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
        // capture on a private stream: the caller's may be the null stream
        if (!b->capture_stream) BHIPCHK(b, hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        BHIPCHK(b, hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
        const hipError_t le = launch_config(b->cfg, a, nblocks, b->capture_stream);
        const hipError_t ce = hipStreamEndCapture(b->capture_stream, &g);
        (void)hipGetLastError();
        BHIPCHK(b, le);
        BHIPCHK(b, ce);
        b->graph_defs.push_back(g);
        hipGraphExec_t ex = nullptr;
        BHIPCHK(b, hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
        it = b->graphs.emplace(key, ex).first;
    }
    BHIPCHK(b, hipGraphLaunch(it->second, b->stream));
    return LBW_OK;
}

lbw_status lbw_batch_step(lbw_batch *b, int nsteps, int use_graph)
{
    if (!b) return LBW_ERR_ARG;
    if (!b->initialized) return bfail(b, LBW_ERR_STATE, "lbw_batch_init first");
    if (nsteps < 0) return bfail(b, LBW_ERR_ARG, "nsteps must be >= 0");
    if (nsteps == 0) return LBW_OK;
    BHIPCHK(b, hipEventRecord(b->ev[0], b->stream));
    lbw_status rc = launch_step(b, nsteps, use_graph);
    if (rc != LBW_OK) return rc;
    BHIPCHK(b, hipEventRecord(b->ev[1], b->stream));
    b->ev_recorded = true;
    // the launch's schedule (run_instance): one single step, (nsteps - 1) /
    // BATCH_DEPTH deep sweeps, then two-step sweeps and one more single step
    // for the remainder, the finish; each sweep and the finish swap the
    // population buffers, each multi-step sweep swaps the E_z / lagged-value
    // buffers
    const int deep = (nsteps - 1) / BATCH_DEPTH, tail = (nsteps - 1) % BATCH_DEPTH;
    const int pairs = tail / 2, single_tail = tail % 2;
    b->step += nsteps;
    b->cur ^= (1 + deep + pairs + single_tail + 1) & 1;
    b->ecur ^= (deep + pairs) & 1;
    return LBW_OK;
}

lbw_status lbw_batch_get_timing(lbw_batch *b, double *ms)
{
    if (!b || !ms) return LBW_ERR_ARG;
    if (!b->ev_recorded) return bfail(b, LBW_ERR_STATE, "no lbw_batch_step yet");
    BHIPCHK(b, hipEventSynchronize(b->ev[1]));
    float f = 0.0f;
    BHIPCHK(b, hipEventElapsedTime(&f, b->ev[0], b->ev[1]));
    *ms = f;
    return LBW_OK;
}

// Make configuration ci current: for the split schedule, check that enough
// workgroups can be resident, plan the work lists and upload them (graphs
// captured for another split configuration then go: they read the lists).
static lbw_status apply_config(lbw_batch *b, int ci)
{
    const int n = (int)b->inst.size();
    if (!CONFIGS[ci].split) {
        b->cfg = ci;
        b->nwg = n;
        return LBW_OK;
    }
    if (b->plan1_cfg != ci) {
        const int resident = std::min(resident_workgroups(ci), MAX_SPLIT_WG);
        if (resident < n)
            return bfail(b, LBW_ERR_UNSUPPORTED,
                         "split schedule: fewer co-resident workgroups than instances, or no cooperative launch");
        const Plan p = plan_split(b->d, b->order, deep_width(CONFIGS[ci]), resident);
        std::vector<int> buf(p.woff);
        buf.insert(buf.end(), p.items.begin(), p.items.end());
        BHIPCHK(b, hipStreamSynchronize(b->stream));  // no launch still reads the old lists
        BHIPCHK(b, hipMemcpyAsync(b->ws + b->L.plan[1], buf.data(), buf.size() * sizeof(int), hipMemcpyHostToDevice,
                                  b->stream));
        BHIPCHK(b, hipStreamSynchronize(b->stream));  // the host buffer goes out of scope
        for (auto it = b->graphs.begin(); it != b->graphs.end();) {
            if (CONFIGS[it->first.second].split) {
                (void)hipGraphExecDestroy(it->second);
                it = b->graphs.erase(it);
            } else {
                ++it;
            }
        }
        b->plan_nwg[1] = (int)p.woff.size() - 1;
        b->plan1_cfg = ci;
    }
    b->cfg = ci;
    b->nwg = b->plan_nwg[1];
    return LBW_OK;
}

static int find_config(int threads, int cpt, int split)
{
    for (int i = 0; i < NCONFIG; ++i)
        if (CONFIGS[i].threads == threads && CONFIGS[i].cpt == cpt && CONFIGS[i].split == split) return i;
    return -1;
}

lbw_status lbw_batch_set_config(lbw_batch *b, int threads, int cpt)
{
    if (!b) return LBW_ERR_ARG;
    const int ci = find_config(threads, cpt, 0);
    if (ci < 0)
        return bfail(b, LBW_ERR_ARG,
                     "configuration must be 256 or 512 threads with 1 or 2 nodes each, or 1024 threads with 1");
    return apply_config(b, ci);
}

lbw_status lbw_batch_set_schedule(lbw_batch *b, int threads, int cpt, int split)
{
    if (!b) return LBW_ERR_ARG;
    const int ci = find_config(threads, cpt, split ? 1 : 0);
    if (ci < 0) return bfail(b, LBW_ERR_ARG, "no such launch configuration");
    return apply_config(b, ci);
}

lbw_status lbw_batch_get_schedule(const lbw_batch *b, int *threads, int *cpt, int *split, int *workgroups)
{
    if (!b || !threads || !cpt || !split || !workgroups) return LBW_ERR_ARG;
    *threads = CONFIGS[b->cfg].threads;
    *cpt = CONFIGS[b->cfg].cpt;
    *split = CONFIGS[b->cfg].split;
    *workgroups = b->nwg;
    return LBW_OK;
}

lbw_status lbw_batch_get_config(const lbw_batch *b, int *threads, int *cpt)
{
    if (!b || !threads || !cpt) return LBW_ERR_ARG;
    *threads = CONFIGS[b->cfg].threads;
    *cpt = CONFIGS[b->cfg].cpt;
    return LBW_OK;
}

static lbw_status snapshot(lbw_batch *b, bool save)
{
    const BLayout &L = b->L;
    // the canonical state: the current population buffer, E_z, lagged
    // values and the per-instance state records
    const size_t pairs[4][3] = {{L.pop[b->cur], L.snap_pop, L.pop_elems * 8},
                                {L.ez, L.snap_ez, L.fld_elems * 8},
                                {L.lag, L.snap_lag, L.lag_elems * 8},
                                {L.st, L.snap_st, b->inst.size() * sizeof(BState)}};
    for (auto &p : pairs) {
        if (p[2] == 0) continue;
        char *live = b->ws + p[0], *copy = b->ws + p[1];
        BHIPCHK(b, hipMemcpyAsync(save ? copy : live, save ? live : copy, p[2], hipMemcpyDeviceToDevice, b->stream));
    }
    return LBW_OK;
}

lbw_status lbw_batch_autotune(lbw_batch *b, int probe_steps, int *threads, int *cpt)
{
    if (!b) return LBW_ERR_ARG;
    if (!b->initialized) return bfail(b, LBW_ERR_STATE, "lbw_batch_init first");
    if (probe_steps < 1) return bfail(b, LBW_ERR_ARG, "probe_steps must be >= 1");
    const long step0 = b->step;
    const int cur0 = b->cur, ecur0 = b->ecur;
    lbw_status rc = snapshot(b, true);
    if (rc != LBW_OK) return rc;
    double best = 1e300;
    int best_i = b->cfg;
    for (int i = 0; i < NCONFIG; ++i) {
        if (apply_config(b, i) != LBW_OK) {  // a split schedule the device cannot hold
            rc = LBW_OK;
            continue;
        }
        // one untimed launch (first use of this kernel), then the timed one
        for (int rep = 0; rep < 2; ++rep) {
            rc = snapshot(b, false);
            b->step = step0;
            b->cur = cur0;
            b->ecur = ecur0;
            if (rc == LBW_OK) rc = lbw_batch_step(b, probe_steps, 0);
            if (rc != LBW_OK) break;
        }
        double ms = 0.0;
        if (rc == LBW_OK) rc = lbw_batch_get_timing(b, &ms);
        if (rc != LBW_OK) break;
        if (ms < best) {
            best = ms;
            best_i = i;
        }
    }
    b->step = step0;
    b->cur = cur0;
    b->ecur = ecur0;
    lbw_status rc2 = snapshot(b, false);
    if (rc == LBW_OK) rc = rc2;
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    rc2 = apply_config(b, best_i);
    if (rc == LBW_OK) rc = rc2;
    if (threads) *threads = CONFIGS[best_i].threads;
    if (cpt) *cpt = CONFIGS[best_i].cpt;
    return rc;
}

lbw_status lbw_batch_read(lbw_batch *b, int i, int which, double *host_out, size_t count)
{
    if (!b || !host_out) return bfail(b, LBW_ERR_ARG, "NULL argument");
    if (!b->initialized) return bfail(b, LBW_ERR_STATE, "lbw_batch_init first");
    if (i < 0 || i >= (int)b->inst.size()) return bfail(b, LBW_ERR_ARG, "instance index out of range");
    const BInst &P = b->inst[i];
    if (count != (size_t)P.nz) return bfail(b, LBW_ERR_ARG, "count must be the instance's nz");
    if (!((which >= 0 && which < LBW_NMOMENTS) || which == LBW_BATCH_EZ))
        return bfail(b, LBW_ERR_ARG, "unknown observable");
    StepArgs a = instance_args(b, i);
    // output staged in the instance's free population buffer
    double *out = (double *)(b->ws + b->L.pop[b->cur ^ 1]) + P.pop;
    const int nb = (P.nzp + 255) / 256;
    if (which == LBW_BATCH_EZ)
        hipLaunchKernelGGL(k_read_field<1>, dim3(nb), dim3(256), 0, b->stream, a, 0, 1, out);
    else if (P.closure == LBW_LEC)
        hipLaunchKernelGGL((k_read_moment<1, LEC, double>), dim3(nb), dim3(256), 0, b->stream, a, which, out);
    else
        hipLaunchKernelGGL((k_read_moment<1, WARMC, double>), dim3(nb), dim3(256), 0, b->stream, a, which, out);
    BHIPCHK(b, hipGetLastError());
    BHIPCHK(b, hipMemcpyAsync(host_out, out, count * 8, hipMemcpyDeviceToHost, b->stream));
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    return LBW_OK;
}

lbw_status lbw_batch_nonfinite(lbw_batch *b, int *counts)
{
    if (!b || !counts) return bfail(b, LBW_ERR_ARG, "NULL argument");
    const int n = (int)b->inst.size();
    std::vector<BState> st(n);
    BHIPCHK(b, hipMemcpyAsync(st.data(), b->ws + b->L.st, n * sizeof(BState), hipMemcpyDeviceToHost, b->stream));
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    for (int i = 0; i < n; ++i) counts[i] = st[i].nonfinite;
    return LBW_OK;
}

}  // extern "C"
