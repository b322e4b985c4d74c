// lbw_kernels.hpp -- fused time-step kernels of the moment-matching LB scheme
// for warm relativistic plasma wakes (Simeoni et al., arXiv 2309.04872), plus
// the small kernels around them (finish, init, read-out, diagnostics).
//
// Time levels. The state between two fused launches is (f*^{n-1}, E^{n-1},
// B^{n-3/2}, lag^{n-1}): launch n pulls f^n (streaming, Sec. 2.1), recovers
// n^n, u^n (Sec. 3.1 / 4.1), completes the Yee update of step n-1 with the
// current J^n = -n^n u^n (E^{n-1} -> E^n, B^{n-3/2} -> B^{n-1/2}), forms
// B^n = B^{n-1/2} - dt/2 curl E^n, the forcing F^n and collides (eq. lbe,
// eq. ade-feq, S_i = w_i F) into f*^n. A canonical state (f^n post-stream,
// E^n, B^{n-1/2}) enters with do_pull = do_maxwell = 0.
#pragma once

#include "lbw_device.hpp"

#include <type_traits>

namespace lbw {

constexpr int NLAG2 = 5;  // theta^00, theta^0z, theta^0x, lambda u_z, lambda u_x
constexpr int NLAG1 = 3;  // theta^00, theta^0z, lambda u_z

struct StepArgs {
    const void *src;   // populations in: f*^{n-1} (pull) or canonical f^n
    void *dst;         // populations out: f*^n
    const double *ez_in, *ex_in, *by_in;
    double *ez_out, *ex_out, *by_out;
    double *lag;                 // warm closure lagged values, [NLAG][ncell], in place
    double *lag_alt;             // 1D warm closure: the other lagged-value buffer (multi-step passes)
    unsigned int *fallbacks;     // LEC recovery fallback counter
    const double *aref;          // per-scalar storage reference A_ref (device, K values)
    int nz, nx, ncell;
    int bcz, bcx;
    double delta, dt, inv2d, omega, lam, mu, a_lec, two_over_d;
    int dcode;                   // 1, 3 or 0 (general D)
    int do_pull, do_maxwell, lag_init;
    int axi;                     // 2D: axisymmetric (z, r) geometry
    long step;
    Driver drv;
    unsigned int *nonfinite;     // set by the finish kernels when a node is not finite (null: no check)
};

// Advected scalars that change sign under r -> -r in the axisymmetric
// geometry: the radial momentum A_r (LEC), n lambda u_r and lambda theta^{rz}
// (WARMC, 2D order of NScal).
template <int CL> __device__ __forceinline__ constexpr bool odd_in_r(int k)
{
    return CL == LEC ? k == 2 : (k == 3 || k == 7);
}

// ---------------------------------------------------------------------------
// Collision of all scalars in deviation form (A_ref = 0 gives the plain form):
// s*_{k,q} = (1 - omega) s_{k,q} + w_q (omega dA_k + dt F_k + omega A_k P_q),
// P_q = 3 (e_q.u)/Lambda + 9/2 (e_q.u)^2/Lambda^2 - 3/2 u^2/Lambda^2, which is
// f_eq_q / (w_q A) - 1 of eq. ade-feq with nu^2 = Lambda^2 / 3; P_q is shared
// by every scalar since they all move with the same u (Sec. 3.1, Sec. 4.1).
template <int DIM, int K, class CT>
__device__ __forceinline__ void collide_all(CT (*s)[Lattice<DIM>::Q], const double *A,
                                            const double *aref, const double *F, double uz,
                                            double ux, double lam, double omega, double dt)
{
    using L = Lattice<DIM>;
    constexpr int Q = L::Q;
    const CT uzc = (CT)uz, uxc = (CT)ux;
    const CT c1 = (CT)(3.0 / lam), c2 = (CT)(4.5 / (lam * lam));
    const CT c3uu = (CT)(1.5 * (uz * uz + ux * ux) / (lam * lam));
    CT P[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const CT eu = uzc * (CT)L::ez(q) + uxc * (CT)L::ex(q);
        P[q] = c1 * eu + c2 * eu * eu - c3uu;
    }
    const CT om = (CT)omega, keep = (CT)(1.0 - omega);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const CT al = (CT)(omega * (A[k] - aref[k]) + dt * F[k]);
        const CT be = (CT)(omega * A[k]);
#pragma unroll
        for (int q = 0; q < Q; ++q) s[k][q] = keep * s[k][q] + (CT)L::w(q) * (al + be * P[q]);
    }
}

// ---------------------------------------------------------------------------
// 2D fused step. Tile TZ x TX nodes per workgroup, CPT nodes per thread (rows
// lx, lx + TX/CPT, ...: every thread issues the loads of all its nodes before
// it waits on any). Recovery runs on the tile plus a one-node ring (LDS), the
// Yee update on a two-node field halo (LDS).
// AXI: axisymmetric (z, r) geometry of Sec. 2.2 and App. A. x is r, node
// row j sits at r_j = (j + 1/2) delta, rows below the axis are mirror images
// (populations of the mirrored direction, the scalars odd in r negated; the
// ring row -1 then holds the image's recovered values, which radial
// differences at row 0 read), every advected scalar gets the source
// -u_r A / r plus, for the warm closure, the cylindrical parts of the tensor
// divergences, and the E_z update takes the cylindrical curl
// (1/r) d_r (r B_phi); E_r and B_phi vanish on the axis.
// STRIP > 1: inside an XCD's band the tiles run z-major through strips of
// STRIP tile-rows, so that the rows a tile shares with the tiles above and
// below are still in that XCD's L2 when they are read again.
// NTS: the post-collision populations are stored with the non-temporal hint,
// and for the warm closure the fields and lagged values too (warm FP64 slab
// 4096 x 1024: 1150.5 -> 1142.8 us, FP32 669.4 -> 662.8 us).
// Minimum waves per SIMD asked of the compiler: 3 for the axisymmetric warm
// closure with FP32 / FP16 populations, which would otherwise take 177-179
// VGPRs and 2 waves; at 168 VGPRs with a few bytes per lane spilled the
// 3000 x 600 step is faster (FP32 370 -> 357 us with one population per
// access, FP16 220.1 -> 213.5 us with the 16-byte groups), and its LDS lets
// three 256-thread workgroups share a compute unit.
template <int CL, class ST, bool AXI> constexpr int step2d_min_waves()
{
    return (AXI && CL == WARMC && !std::is_same<ST, double>::value) ? 3 : 1;
}
template <int CL, class ST, int TZ, int TX, int CPT, bool AXI = false, int STRIP = 1, bool NTS = false>
__global__ __launch_bounds__(TZ *TX / CPT, (step2d_min_waves<CL, ST, AXI>())) void k_step2d(StepArgs a)
{
    using L = Lattice<2>;
    using CT = typename Store<ST>::ct;
    constexpr int Q = L::Q;
    constexpr int K = NScal<2, CL>::K;
    using PopL = Pops<ST, K, Q>;
    constexpr int NT = TZ * TX / CPT;
    constexpr int XS = TX / CPT;             // row stride between a thread's nodes
    constexpr int RZ = TZ + 2, RX = TX + 2;  // recovery region (ring of 1)
    constexpr int FZ = TZ + 4, FX = TX + 4;  // field region (halo of 2)
    constexpr int NG = CL == LEC ? 1 : 7;    // gradient quantities
    constexpr int NRING = 2 * RZ + 2 * TX;
    static_assert(TX % CPT == 0, "tile rows must split evenly over a thread's nodes");

    __shared__ double s_ez[FX][FZ], s_ex[FX][FZ], s_by[FX][FZ], s_bn[FX][FZ];
    __shared__ double s_jz[RX][RZ], s_jx[RX][RZ];
    __shared__ double s_g[NG][RX][RZ];

    const int tid = threadIdx.x;
    const int nz = a.nz, nx = a.nx, bcz = a.bcz, bcx = a.bcx;
    const size_t nc = (size_t)a.ncell;
    const int ntz = (nz + TZ - 1) / TZ;
    const int tile = xcd_band_tile(blockIdx.x, gridDim.x);
    int z0, x0;
    if constexpr (STRIP == 1) {
        z0 = (tile % ntz) * TZ;
        x0 = (tile / ntz) * TX;
    } else {
        const int ntx = (nx + TX - 1) / TX;
        const int strip = tile / (STRIP * ntz), rr = tile % (STRIP * ntz);
        const int rows = ntx - strip * STRIP < STRIP ? ntx - strip * STRIP : STRIP;  // last strip
        z0 = (rr / rows) * TZ;
        x0 = (strip * STRIP + rr % rows) * TX;
    }
    const ST *src = (const ST *)a.src;
    ST *dst = (ST *)a.dst;

    // ---- 1. old fields into LDS (E^{n-1}, B^{n-3/2}; or E^n, B^{n-1/2}). Every
    // load of a thread's slots is issued before the first LDS write, so the
    // halo costs one memory round trip instead of one per slot (4096 x 1024
    // warm FP64 1073 -> 1035 us, FP16 365 -> 333 us; 2048 x 512 local
    // equilibrium FP64 106.5 -> 98.8 us)
    {
        constexpr int NI = (FZ * FX + NT - 1) / NT;
        double fez[NI], fex[NI], fby[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int p = tid + i * NT;
            if (p < FZ * FX) {
                const int fz = p % FZ, fx = p / FZ;
                const int gz = z0 - 2 + fz, gx = x0 - 2 + fx;
                fez[i] = a.ez_in[(size_t)fix_node(gx, nx, bcx) * nz + fix_stag(gz, nz, bcz)];
                fex[i] = a.ex_in[(size_t)fix_stag(gx, nx, bcx) * nz + fix_node(gz, nz, bcz)];
                fby[i] = a.by_in[(size_t)fix_stag(gx, nx, bcx) * nz + fix_stag(gz, nz, bcz)];
            }
        }
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int p = tid + i * NT;
            if (p < FZ * FX) {
                const int fz = p % FZ, fx = p / FZ;
                s_ez[fx][fz] = fez[i];
                s_ex[fx][fz] = fex[i];
                s_by[fx][fz] = fby[i];
            }
        }
    }

    const double two_over_d = a.two_over_d, a_lec = a.a_lec;
    double aref[K];
#pragma unroll
    for (int k = 0; k < K; ++k) aref[k] = a.aref[k];

    // source node of direction q: (gx - e_x, gz - e_z) when streaming. AXI:
    // a source row -1 - m below the axis is the image of row m, whose
    // direction mx(q) carries f_q there, with the scalars odd in r negated;
    // this also makes the ghost ring row -1 the image of row 0.
    auto load = [&](int gz, int gx, CT (*s)[Q]) {
        const int sh = a.do_pull ? 1 : 0;
        int zs[3], xs[3];
        bool rf[3];
#pragma unroll
        for (int e = -1; e <= 1; ++e) {
            int sx = gx - sh * e;
            rf[e + 1] = AXI && sx < 0;
            if (AXI && sx < 0) sx = -1 - sx;
            zs[e + 1] = fix_node(gz - sh * e, nz, bcz);
            xs[e + 1] = fix_node(sx, nx, bcx) * nz;
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int c = xs[L::ex(q) + 1] + zs[L::ez(q) + 1];
            CT v[K];
            if constexpr (AXI) {
                const bool m = rf[L::ex(q) + 1];
                const int qs = m ? L::mx(q) : q;
                PopL::ld_all(src, qs, nc, c, v);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    // deviation storage: f = s + w A_ref, and w is the same for q and mx(q)
                    s[k][q] = (odd_in_r<CL>(k) && m) ? (CT)(-v[k] - (CT)(2.0 * L::w(q) * aref[k])) : v[k];
                }
            } else {
                PopL::ld_all(src, q, nc, c, v);
#pragma unroll
                for (int k = 0; k < K; ++k) s[k][q] = v[k];
            }
        }
    };
    // zeroth moments in the storage type, promoted to FP64 (eq. disc-moments-ade)
    auto moments = [&](CT (*s)[Q], double *A) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            CT acc = 0;
#pragma unroll
            for (int q = 0; q < Q; ++q) acc += s[k][q];
            A[k] = aref[k] + (double)acc;
        }
    };

    // recovery of one node into the LDS ring/tile slot (rz, rx)
    auto recover_to_lds = [&](const double *A, int rz, int rx, double &uz, double &ux) {
        const double n = A[0];
        if constexpr (CL == LEC) {
            LecRec r;
            if (!lec_recover(n, A[1], A[2], a_lec, a.dcode, two_over_d, r)) {
                if (a.fallbacks) atomicAdd(a.fallbacks, 1u);
            }
            uz = r.uz;
            ux = r.ux;
            s_g[0][rx][rz] = r.phi;
        } else {
            WarmRec r;
            warm_recover<2>(A, r);
            uz = r.uz;
            ux = r.ux;
            s_g[0][rx][rz] = r.th0z;
            s_g[1][rx][rz] = r.th0x;
            s_g[2][rx][rz] = r.thzz;
            s_g[3][rx][rz] = r.thxx;
            s_g[4][rx][rz] = r.thxz;
            s_g[5][rx][rz] = r.luz;
            s_g[6][rx][rz] = r.lux;
        }
        s_jz[rx][rz] = -n * uz;
        s_jx[rx][rz] = -n * ux;
    };

    const int lz = tid % TZ, lxb = tid / TZ;
    const int gz = z0 + lz;
    CT s[CPT][K][Q];
    double A[CPT][K];
    double uz[CPT], ux[CPT];
    auto ring_node = [&](int t, int &rz, int &rx) {
        if (t < RZ) { rz = t; rx = 0; }
        else if (t < 2 * RZ) { rz = t - RZ; rx = RX - 1; }
        else { const int u = t - 2 * RZ; rx = 1 + u / 2; rz = (u & 1) ? RZ - 1 : 0; }
    };
    if constexpr (CL == LEC && NRING <= NT) {
        // ---- 2-3 (local equilibrium). Own nodes' loads first, then the ring
        // node's (at most one per thread), so that both are in flight together;
        // then the ring recovery and the own recoveries. Own populations stay
        // in registers.
#pragma unroll
        for (int r = 0; r < CPT; ++r) load(gz, x0 + lxb + r * XS, s[r]);
        int rz = 0, rx = 0;
        double Ar[K];
        if (tid < NRING) {
            ring_node(tid, rz, rx);
            CT sr[K][Q];
            load(z0 - 1 + rz, x0 - 1 + rx, sr);
            moments(sr, Ar);
            double uzr, uxr;
            recover_to_lds(Ar, rz, rx, uzr, uxr);
        }
    } else {
        // ---- 2. ring nodes: pull, recover, keep only the LDS results
        for (int t = tid; t < NRING; t += NT) {
            int rz, rx;
            ring_node(t, rz, rx);
            CT sr[K][Q];
            double Ar[K];
            load(z0 - 1 + rz, x0 - 1 + rx, sr);
            moments(sr, Ar);
            double uzr, uxr;
            recover_to_lds(Ar, rz, rx, uzr, uxr);
        }
        // ---- 3. own nodes: pull all of them; populations stay in registers
#pragma unroll
        for (int r = 0; r < CPT; ++r) load(gz, x0 + lxb + r * XS, s[r]);
    }
    // warm closure: the own nodes' lagged values travel with the populations
    // (one memory round trip for both)
    double lagv[CPT][CL == WARMC ? NLAG2 : 1];
    if constexpr (CL == WARMC) {
#pragma unroll
        for (int r = 0; r < CPT; ++r) {
            const int gx = x0 + lxb + r * XS;
            const bool own = gz < nz && gx < nx && !a.lag_init;
            const size_t c = (size_t)gx * nz + gz;
#pragma unroll
            for (int g = 0; g < NLAG2; ++g) lagv[r][g] = own ? a.lag[g * nc + c] : 0.0;
        }
    }
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
        moments(s[r], A[r]);
        recover_to_lds(A[r], lz + 1, lxb + r * XS + 1, uz[r], ux[r]);
    }
    __syncthreads();

    // Stages 4-6 read LDS through the boundary rule; tiles that touch no open
    // boundary (and every periodic direction) compile it away: their LDS
    // accesses are plain offsets from the thread's own slot.
    const bool edge = (bcz == BC_OPEN && (z0 < 2 || z0 + TZ + 3 > nz)) ||
                      (bcx == BC_OPEN && (x0 < 2 || x0 + TX + 3 > nx));
    auto rest = [&](auto edge_tag) {
        constexpr bool EDGE = decltype(edge_tag)::value;
        // local coordinates of a global (unwrapped) coordinate after the boundary rule
        auto fzn = [&](int g) { return (EDGE ? map_node(g, nz, bcz) : g) - (z0 - 2); };
        auto fzs = [&](int g) { return (EDGE ? map_stag(g, nz, bcz) : g) - (z0 - 2); };
        auto fxn = [&](int g) { return (EDGE ? map_node(g, nx, bcx) : g) - (x0 - 2); };
        auto fxs = [&](int g) { return (EDGE ? map_stag(g, nx, bcx) : g) - (x0 - 2); };
        auto rzn = [&](int g) { return (EDGE ? map_node(g, nz, bcz) : g) - (z0 - 1); };
        // AXI: row -1 of the recovery ring is the mirror image of row 0
        auto rxn = [&](int g) { return (EDGE && !(AXI && g < 0) ? map_node(g, nx, bcx) : g) - (x0 - 1); };
        const double dt = a.dt, hdt = 0.5 * a.dt, id = 1.0 / a.delta;
        // ---- 4. finish the Yee update of the previous step with J^n
        if (a.do_maxwell) {
            for (int p = tid; p < (FZ - 1) * (FX - 1); p += NT) {
                const int fz = p % (FZ - 1), fx = p / (FZ - 1);
                const int gzz = z0 - 2 + fz, gxx = x0 - 2 + fx;
                const double curl = ((s_ex[fxs(gxx)][fzn(gzz + 1)] - s_ex[fxs(gxx)][fzn(gzz)]) -
                                     (s_ez[fxn(gxx + 1)][fzs(gzz)] - s_ez[fxn(gxx)][fzs(gzz)])) * id;
                const double b1 = s_by[fx][fz] - hdt * curl;  // B^{n-1}
                s_by[fx][fz] = b1 - hdt * curl;               // B^{n-1/2}
            }
            __syncthreads();
            const double th = (a.step - 0.5) * dt;
            for (int p = tid; p < (FZ - 2) * (FX - 2); p += NT) {
                const int fz = 1 + p % (FZ - 2), fx = 1 + p / (FZ - 2);
                const int gzz = z0 - 2 + fz, gxx = x0 - 2 + fx;
                if (fx <= FX - 3) {  // E_x at (z_gzz, x_{gxx+1/2})
                    const double jx = 0.5 * (s_jx[rxn(gxx)][rzn(gzz)] + s_jx[rxn(gxx + 1)][rzn(gzz)]);
                    const double cx = -(s_by[fxs(gxx)][fzs(gzz)] - s_by[fxs(gxx)][fzs(gzz - 1)]) * id;
                    s_ex[fx][fz] = s_ex[fx][fz] + dt * (cx - jx);
                }
                if (fz <= FZ - 3) {  // E_z at (z_{gzz+1/2}, x_gxx)
                    const double jz = 0.5 * (s_jz[rxn(gxx)][rzn(gzz)] + s_jz[rxn(gxx)][rzn(gzz + 1)]);
                    const double jb = -driver_density<2>(a.drv, (gzz + 0.5) * a.delta,
                                                         node_x(gxx, nx, a.delta, AXI), th);
                    double cz;
                    if constexpr (AXI) {
                        // (1/r) d_r (r B_phi) at r_j from r_{j+1/2} = (j+1) delta and
                        // r_{j-1/2} = j delta (the axis for j = 0); rows below the
                        // axis are never read
                        const double bm = gxx > 0 ? s_by[fxs(gxx - 1)][fzs(gzz)] : 0.0;
                        cz = ((gxx + 1.0) * s_by[fxs(gxx)][fzs(gzz)] - gxx * bm) / ((gxx + 0.5) * a.delta);
                    } else {
                        cz = (s_by[fxs(gxx)][fzs(gzz)] - s_by[fxs(gxx - 1)][fzs(gzz)]) * id;
                    }
                    s_ez[fx][fz] = s_ez[fx][fz] + dt * (cz - jz - jb);
                }
            }
            __syncthreads();
        }

        // ---- 5. B^n = B^{n-1/2} - dt/2 curl E^n around the tile; write E^n, B^{n-1/2}
        for (int p = tid; p < (FZ - 3) * (FX - 3); p += NT) {
            const int fz = 1 + p % (FZ - 3), fx = 1 + p / (FZ - 3);
            const int gzz = z0 - 2 + fz, gxx = x0 - 2 + fx;
            const double curl = ((s_ex[fxs(gxx)][fzn(gzz + 1)] - s_ex[fxs(gxx)][fzn(gzz)]) -
                                 (s_ez[fxn(gxx + 1)][fzs(gzz)] - s_ez[fxn(gxx)][fzs(gzz)])) * id;
            s_bn[fx][fz] = s_by[fx][fz] - hdt * curl;
        }
#pragma unroll
        for (int r = 0; r < CPT; ++r) {
            const int lx = lxb + r * XS, gx = x0 + lx;
            if (gz < nz && gx < nx) {
                const size_t c = (size_t)gx * nz + gz;
                if constexpr (NTS && CL == WARMC) {
                    __builtin_nontemporal_store(s_ez[lx + 2][lz + 2], a.ez_out + c);
                    __builtin_nontemporal_store(s_ex[lx + 2][lz + 2], a.ex_out + c);
                    __builtin_nontemporal_store(s_by[lx + 2][lz + 2], a.by_out + c);
                } else {
                    a.ez_out[c] = s_ez[lx + 2][lz + 2];
                    a.ex_out[c] = s_ex[lx + 2][lz + 2];
                    a.by_out[c] = s_by[lx + 2][lz + 2];
                }
            }
        }
        __syncthreads();

        // ---- 6. node fields, forcing, collision
#pragma unroll
        for (int r = 0; r < CPT; ++r) {
            const int lx = lxb + r * XS, gx = x0 + lx;
            if (!(gz < nz && gx < nx)) continue;
            const double Ez = 0.5 * (s_ez[fxn(gx)][fzs(gz - 1)] + s_ez[fxn(gx)][fzs(gz)]);
            double Ex, By;
            if (AXI && gx == 0) {  // E_r and B_phi are zero on the axis r_{-1/2}
                Ex = 0.5 * s_ex[fxs(gx)][fzn(gz)];
                By = 0.25 * (s_bn[fxs(gx)][fzs(gz)] + s_bn[fxs(gx)][fzs(gz - 1)]);
            } else {
                Ex = 0.5 * (s_ex[fxs(gx - 1)][fzn(gz)] + s_ex[fxs(gx)][fzn(gz)]);
                By = 0.25 * (s_bn[fxs(gx)][fzs(gz)] + s_bn[fxs(gx)][fzs(gz - 1)] +
                             s_bn[fxs(gx - 1)][fzs(gz)] + s_bn[fxs(gx - 1)][fzs(gz - 1)]);
            }
            const int rzc = lz + 1, rxc = lx + 1;
            const int rzp = rzn(gz + 1), rzm = rzn(gz - 1), rxp = rxn(gx + 1), rxm = rxn(gx - 1);
            auto Dz = [&](int g) { return (s_g[g][rxc][rzp] - s_g[g][rxc][rzm]) * a.inv2d; };
            auto Dx = [&](int g) { return (s_g[g][rxp][rzc] - s_g[g][rxm][rzc]) * a.inv2d; };
            const double n = A[r][0], vz = uz[r], vx = ux[r];
            double F[K];
            const size_t c = (size_t)gx * nz + gz;
            if constexpr (CL == LEC) {
                // eq. lb-ade-lec-comps-F (q = -1): F = -mu grad n0^{1+2/D} - n (E + u x B)
                F[0] = 0.0;
                F[1] = -a.mu * Dz(0) - n * (Ez + vx * By);
                F[2] = -a.mu * Dx(0) - n * (Ex - vz * By);
                if constexpr (AXI) {
                    // App. A: the cylindrical part of the divergence, -u_r A_k / r
                    const double ir = 1.0 / ((gx + 0.5) * a.delta);
                    F[0] -= vx * n * ir;
                    F[1] -= vx * A[r][1] * ir;
                    F[2] -= vx * A[r][2] * ir;
                }
            } else {
                // App. A warm-closure right-hand sides, Cartesian slab (r -> x, phi -> y)
                const double th0z = s_g[0][rxc][rzc], th0x = s_g[1][rxc][rzc];
                const double thzz = s_g[2][rxc][rzc], thxx = s_g[3][rxc][rzc];
                const double thxz = s_g[4][rxc][rzc];
                const double luz = s_g[5][rxc][rzc], lux = s_g[6][rxc][rzc];
                const double th00 = vx * th0x + vz * th0z;
                double l00, l0z, l0x, lluz, llux;
                if (a.lag_init) {
                    l00 = th00; l0z = th0z; l0x = th0x; lluz = luz; llux = lux;
                } else {
                    l00 = lagv[r][0]; l0z = lagv[r][1]; l0x = lagv[r][2];
                    lluz = lagv[r][3]; llux = lagv[r][4];
                }
                const double lagn[NLAG2] = {th00, th0z, th0x, luz, lux};
#pragma unroll
                for (int g = 0; g < NLAG2; ++g) {
                    if constexpr (NTS) __builtin_nontemporal_store(lagn[g], a.lag + g * nc + c);
                    else a.lag[g * nc + c] = lagn[g];
                }
                const double idt = 1.0 / dt;
                const double dt00 = (th00 - l00) * idt, dt0z = (th0z - l0z) * idt;
                const double dt0x = (th0x - l0x) * idt;
                const double dtluz = (luz - lluz) * idt, dtlux = (lux - llux) * idt;
                F[0] = 0.0;
                F[1] = -dt00 - Dx(1) - Dz(0) - n * (Ex * vx + Ez * vz);
                F[2] = -dt0z - Dx(4) - Dz(2) - n * (Ez + vx * By);
                F[3] = -dt0x - Dx(3) - Dz(4) - n * (Ex - vz * By);
                F[4] = -2.0 * th0z * dtluz - 2.0 * thxz * Dx(5) - 2.0 * thzz * Dz(5) -
                       2.0 * (Ez * th0z + By * thxz);
                F[5] = -2.0 * th0x * dtlux - 2.0 * thxx * Dx(6) - 2.0 * thxz * Dz(6) -
                       2.0 * (Ex * th0x - By * thxz);
                F[6] = 0.0;
                F[7] = -th0z * dtlux - th0x * dtluz - thxz * Dx(6) - thxx * Dx(5) - thzz * Dz(6) -
                       thxz * Dz(5) - (Ex * th0z + Ez * th0x + By * (thxx - thzz));
                if constexpr (AXI) {
                    // App. A, warm closure: -u_r A_k / r for every scalar, the
                    // cylindrical parts of the divergences of theta^{0j} and
                    // theta^{ij}, and -3 lambda theta^{phiphi} u_r / r in total
                    const double ir = 1.0 / ((gx + 0.5) * a.delta);
                    const double thyy = A[r][6] / (A[r][1] / n);
                    F[0] -= vx * n * ir;
                    F[1] -= vx * A[r][1] * ir + th0x * ir;
                    F[2] -= vx * A[r][2] * ir + thxz * ir;
                    F[3] -= vx * A[r][3] * ir + (thxx - thyy) * ir;
                    F[4] -= vx * A[r][4] * ir;
                    F[5] -= vx * A[r][5] * ir;
                    F[6] -= 3.0 * vx * A[r][6] * ir;
                    F[7] -= vx * A[r][7] * ir;
                }
            }
            collide_all<2, K, CT>(s[r], A[r], aref, F, vz, vx, a.lam, a.omega, dt);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                CT v[K];
#pragma unroll
                for (int k = 0; k < K; ++k) v[k] = s[r][k][q];
                PopL::template st_all<NTS>(dst, q, nc, (int)c, v);
            }
        }
    };
    if (edge)
        rest(std::true_type{});
    else
        rest(std::false_type{});
}

// ---------------------------------------------------------------------------
// 1D fused step: TZ nodes per workgroup plus a ring of one node on each side;
// E_z sits on the nodes and its update is local: E^n = E^{n-1} + dt (n u + n_b).
template <int CL, class ST, int TZ>
__device__ __forceinline__ void step1d_tile(const StepArgs &a, int tile, double (*s_g)[TZ + 2])
{
    using L = Lattice<1>;
    using CT = typename Store<ST>::ct;
    constexpr int Q = L::Q;
    constexpr int K = NScal<1, CL>::K;
    using PopL = Pops<ST, K, Q>;

    const int tid = threadIdx.x;
    const int nz = a.nz, bcz = a.bcz;
    const size_t nc = (size_t)a.ncell;
    const int z0 = tile * TZ;
    const ST *src = (const ST *)a.src;
    ST *dst = (ST *)a.dst;
    const double two_over_d = a.two_over_d, a_lec = a.a_lec;
    double aref[K];
#pragma unroll
    for (int k = 0; k < K; ++k) aref[k] = a.aref[k];

    auto pull = [&](int gz, CT (*s)[Q], double *A) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int sz = a.do_pull ? gz - L::ez(q) : gz;
            const int c = fix_node(sz, nz, bcz);
            CT v[K];
            PopL::ld_all(src, q, nc, c, v);
#pragma unroll
            for (int k = 0; k < K; ++k) s[k][q] = v[k];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            CT acc = 0;
#pragma unroll
            for (int q = 0; q < Q; ++q) acc += s[k][q];
            A[k] = aref[k] + (double)acc;
        }
    };
    struct R1 { double uz, gamma, phi; WarmRec w; };
    auto recover = [&](const double *A, int rz, R1 &r) {
        if constexpr (CL == LEC) {
            LecRec l;
            if (!lec_recover(A[0], A[1], 0.0, a_lec, a.dcode, two_over_d, l)) {
                if (a.fallbacks) atomicAdd(a.fallbacks, 1u);
            }
            r.uz = l.uz;
            r.phi = l.phi;
            s_g[0][rz] = l.phi;
        } else {
            warm_recover<1>(A, r.w);
            r.uz = r.w.uz;
            s_g[0][rz] = r.w.th0z;
            s_g[1][rz] = r.w.thzz;
            s_g[2][rz] = r.w.luz;
        }
    };

    if (tid < 2) {
        const int rz = tid == 0 ? 0 : TZ + 1;
        CT sr[K][Q];
        double Ar[K];
        pull(z0 - 1 + rz, sr, Ar);
        R1 rr;
        recover(Ar, rz, rr);
    }
    const int gz = z0 + tid;
    const bool active = gz < nz;
    CT s[K][Q];
    double A[K];
    pull(gz, s, A);
    R1 r;
    recover(A, tid + 1, r);
    __syncthreads();
    if (active) {
        const double dt = a.dt;
        const double n = A[0], uz = r.uz;
        const size_t c = (size_t)gz;
        double Ez = a.ez_in[c];
        if (a.do_maxwell) {
            const double jb = driver_density<1>(a.drv, gz * a.delta, 0.0, (a.step - 0.5) * dt);
            Ez = Ez + dt * (n * uz + jb);
        }
        a.ez_out[c] = Ez;
        const int rp = map_node(gz + 1, nz, bcz) - (z0 - 1), rm = map_node(gz - 1, nz, bcz) - (z0 - 1);
        auto Dz = [&](int g) { return (s_g[g][rp] - s_g[g][rm]) * a.inv2d; };
        double F[K];
        if constexpr (CL == LEC) {
            F[0] = 0.0;
            F[1] = -a.mu * Dz(0) - n * Ez;
        } else {
            const double th0z = r.w.th0z, thzz = r.w.thzz, luz = r.w.luz, th00 = r.w.th00;
            double l00, l0z, lluz;
            if (a.lag_init) {
                l00 = th00; l0z = th0z; lluz = luz;
            } else {
                l00 = a.lag[0 * nc + c]; l0z = a.lag[1 * nc + c]; lluz = a.lag[2 * nc + c];
            }
            a.lag[0 * nc + c] = th00; a.lag[1 * nc + c] = th0z; a.lag[2 * nc + c] = luz;
            const double idt = 1.0 / dt;
            F[0] = 0.0;
            F[1] = -(th00 - l00) * idt - Dz(0) - n * (Ez * uz);
            F[2] = -(th0z - l0z) * idt - Dz(1) - n * Ez;
            F[3] = -2.0 * th0z * ((luz - lluz) * idt) - 2.0 * thzz * Dz(2) - 2.0 * (Ez * th0z);
        }
        collide_all<1, K, CT>(s, A, aref, F, uz, 0.0, a.lam, a.omega, dt);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            CT v[K];
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = s[k][q];
            PopL::template st_all<false>(dst, q, nc, (int)c, v);
        }
    }
    __syncthreads();  // the LDS slots are reused by the next tile or step
}

// One launch per step: one tile per workgroup.
template <int CL, class ST, int TZ>
__global__ __launch_bounds__(TZ) void k_step1d(StepArgs a)
{
    constexpr int NG = CL == LEC ? 1 : 3;  // phi | theta^0z, theta^zz, lambda u_z
    __shared__ double s_g[NG][TZ + 2];
    step1d_tile<CL, ST, TZ>(a, blockIdx.x, s_g);
}

// S 1D steps in one pass over a tile (temporal blocking). Slot r of the TZ
// threads holds node fix(z0 - (2S - 1) + r) under the boundary rule. Step 0
// of the pass recovers every slot and collides on slots [1, TZ - 1); each
// later step m pulls its +z / -z populations from the previous step's
// through LDS (rounded to the storage type as a store and reload would round
// them), recovers on slots [2m, TZ - 2m) and collides on [2m + 1, TZ - 2m - 1),
// so step S - 1 writes nodes [z0, z0 + TZ - 4S + 2). E_z and the warm
// closure's lagged values stay in registers; the lagged values are read from
// a.lag and written to a.lag_alt (ring slots read values that a neighbouring
// tile of the same pass rewrites). The per-node arithmetic is that of
// step1d_tile, so a pass equals S single steps bit for bit. Input: the
// mid-step state of the step before the pass (pull); E_z read from ez_in,
// written to ez_out.
template <int TZ, int S> constexpr int multi_width() { return TZ - 4 * S + 2; }

template <int CL, class ST, int TZ, int S>
__device__ __forceinline__ void step1d_multi(const StepArgs &a, int tile, double (*s_g)[TZ + 2],
                                             typename Store<ST>::ct (*xc)[2][TZ])
{
    static_assert(S >= 2 && multi_width<TZ, S>() > 0, "pass depth");
    using L = Lattice<1>;
    using CT = typename Store<ST>::ct;
    constexpr int Q = L::Q;
    constexpr int K = NScal<1, CL>::K;
    using PopL = Pops<ST, K, Q>;
    const int tid = threadIdx.x;
    const int nz = a.nz, bcz = a.bcz;
    const size_t nc = (size_t)a.ncell;
    const int off = tile * multi_width<TZ, S>() - (2 * S - 1);  // node of slot 0 before the boundary rule
    const ST *src = (const ST *)a.src;
    ST *dst = (ST *)a.dst;
    const double dt = a.dt;
    double aref[K];
#pragma unroll
    for (int k = 0; k < K; ++k) aref[k] = a.aref[k];
    // LDS slot holding the neighbour d of slot r's node
    auto nb = [&](int r, int d) {
        return bcz == BC_PERIODIC ? r + d : map_node(fix_node(off + r, nz, bcz) + d, nz, bcz) - off;
    };
    auto moments = [&](CT (*s)[Q], double *A) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            CT acc = 0;
#pragma unroll
            for (int q = 0; q < Q; ++q) acc += s[k][q];
            A[k] = aref[k] + (double)acc;
        }
    };
    WarmRec w;  // warm closure: the recovered node
    auto recover = [&](const double *A, int r, double &uz) {
        if constexpr (CL == LEC) {
            LecRec l;
            if (!lec_recover(A[0], A[1], 0.0, a.a_lec, a.dcode, a.two_over_d, l)) {
                if (a.fallbacks) atomicAdd(a.fallbacks, 1u);
            }
            uz = l.uz;
            s_g[0][r] = l.phi;
        } else {
            warm_recover<1>(A, w);
            uz = w.uz;
            s_g[0][r] = w.th0z;
            s_g[1][r] = w.thzz;
            s_g[2][r] = w.luz;
        }
    };
    // forcing with the lagged values lg (replaced by this step's) and collision
    auto force_collide = [&](CT (*s)[Q], const double *A, double uz, double Ez, int r, double *lg) {
        const int rp = nb(r, 1), rm = nb(r, -1);
        auto Dz = [&](int g) { return (s_g[g][rp] - s_g[g][rm]) * a.inv2d; };
        double F[K];
        F[0] = 0.0;
        if constexpr (CL == LEC) {
            F[1] = -a.mu * Dz(0) - A[0] * Ez;
        } else {
            const double n = A[0];
            const double th0z = w.th0z, thzz = w.thzz, luz = w.luz, th00 = w.th00;
            const double l00 = lg[0], l0z = lg[1], lluz = lg[2];
            lg[0] = th00; lg[1] = th0z; lg[2] = luz;
            const double idt = 1.0 / dt;
            F[1] = -(th00 - l00) * idt - Dz(0) - n * (Ez * uz);
            F[2] = -(th0z - l0z) * idt - Dz(1) - n * Ez;
            F[3] = -2.0 * th0z * ((luz - lluz) * idt) - 2.0 * thzz * Dz(2) - 2.0 * (Ez * th0z);
        }
        collide_all<1, K, CT>(s, A, aref, F, uz, 0.0, a.lam, a.omega, dt);
    };
    auto rnd = [](CT v) { return (CT)Store<ST>::rnd(v); };

    // ---- step 0 of the pass on every slot
    const int z = fix_node(off + tid, nz, bcz);
    CT s[K][Q];
    double A[K], uz;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int c = fix_node(z - L::ez(q), nz, bcz);
        CT v[K];
        PopL::ld_all(src, q, nc, c, v);
#pragma unroll
        for (int k = 0; k < K; ++k) s[k][q] = v[k];
    }
    double Ez = a.ez_in[z];
    double lg[3] = {0.0, 0.0, 0.0};
    if constexpr (CL == WARMC) {
#pragma unroll
        for (int g = 0; g < 3; ++g) lg[g] = a.lag[g * nc + z];
    }
    moments(s, A);
    recover(A, tid, uz);
    __syncthreads();
    CT rest[K];
    if (tid >= 1 && tid < TZ - 1) {
        const double jb = driver_density<1>(a.drv, z * a.delta, 0.0, (a.step - 0.5) * dt);
        Ez = Ez + dt * (A[0] * uz + jb);
        force_collide(s, A, uz, Ez, tid, lg);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            rest[k] = rnd(s[k][0]);
            xc[k][0][tid] = rnd(s[k][1]);
            xc[k][1][tid] = rnd(s[k][2]);
        }
    }
    __syncthreads();  // movers in LDS; every recovered value in LDS has been read
    // ---- steps 1 .. S - 1: pull from LDS, recovery, collision
    for (int m = 1; m < S; ++m) {
        if (tid >= 2 * m && tid < TZ - 2 * m) {
            const int rm = nb(tid, -1), rp = nb(tid, 1);  // sources of the +z and -z movers
#pragma unroll
            for (int k = 0; k < K; ++k) {
                s[k][0] = rest[k];
                s[k][1] = xc[k][0][rm];
                s[k][2] = xc[k][1][rp];
            }
            moments(s, A);
            recover(A, tid, uz);
        }
        __syncthreads();  // recovered values visible; every mover has been read
        if (tid >= 2 * m + 1 && tid < TZ - 2 * m - 1) {
            const int zm = fix_node(off + tid, nz, bcz);
            const double jb = driver_density<1>(a.drv, zm * a.delta, 0.0, (a.step + m - 0.5) * dt);
            Ez = Ez + dt * (A[0] * uz + jb);
            force_collide(s, A, uz, Ez, tid, lg);
            if (m < S - 1) {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    rest[k] = rnd(s[k][0]);
                    xc[k][0][tid] = rnd(s[k][1]);
                    xc[k][1][tid] = rnd(s[k][2]);
                }
            } else {
                const int zo = off + tid;
                if (zo < nz) {
                    a.ez_out[zo] = Ez;
                    if constexpr (CL == WARMC) {
#pragma unroll
                        for (int g = 0; g < 3; ++g) a.lag_alt[g * nc + zo] = lg[g];
                    }
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        CT v[K];
#pragma unroll
                        for (int k = 0; k < K; ++k) v[k] = s[k][q];
                        PopL::template st_all<false>(dst, q, nc, zo, v);
                    }
                }
            }
        }
        __syncthreads();  // movers in LDS (or the tile done); every recovered value has been read
    }
}

// Passes of the persistent 1D kernel for nsteps steps: the first step from
// the canonical state as a single step, then passes of PERSIST_DEPTH steps,
// pairs of steps for what is left, and a single step when one is left. Each
// pass swaps the population and E_z buffers once. Measured per step (local
// equilibrium, 4096 / 16384 nodes, 512 / 1024-node tiles): 3.10 / 4.51 us
// with passes of 2 steps, 2.41 / 3.70 (4), 2.02 / 2.88 (8), 1.89 / 2.58 (16),
// 1.83 / 2.48 (24), 1.82 / 2.45 (32): past 24 the pass's own step latency
// dominates and the redundant halo work (4 nodes per step) grows.
#ifndef LBW_PERSIST_DEPTH
#define LBW_PERSIST_DEPTH 24
#endif
constexpr int PERSIST_DEPTH = LBW_PERSIST_DEPTH;
__host__ __device__ inline int persist_passes(int nsteps)
{
    if (nsteps <= 1) return nsteps;
    const int rest = nsteps - 1, tail = rest % PERSIST_DEPTH;
    return 1 + rest / PERSIST_DEPTH + tail / 2 + (tail & 1);
}
// Multi-step passes among them: each swaps the warm closure's lagged-value
// buffers once.
__host__ __device__ inline int persist_multi_passes(int nsteps)
{
    if (nsteps <= 1) return 0;
    const int rest = nsteps - 1;
    return rest / PERSIST_DEPTH + (rest % PERSIST_DEPTH) / 2;
}

// All steps of one lbw_step call in one cooperative launch (1D grids small
// enough for every workgroup to be resident): the workgroups sweep their
// tiles, then wait for the whole grid before the next pass reads its
// neighbours. Buffers alternate per pass as between separate launches;
// a.src / a.dst and the E_z arrays are those of the first pass.
template <int CL, class ST, int TZ>
__global__ __launch_bounds__(TZ) void k_step1d_persist(StepArgs a, int nsteps)
{
    using CT = typename Store<ST>::ct;
    constexpr int NG = CL == LEC ? 1 : 3;
    __shared__ double s_g[NG][TZ + 2];
    __shared__ CT s_xc[NScal<1, CL>::K][2][TZ];
    const int ntiles = (a.nz + TZ - 1) / TZ;
    const int ntiles2 = (a.nz + multi_width<TZ, 2>() - 1) / multi_width<TZ, 2>();
    const int ntilesd = (a.nz + multi_width<TZ, PERSIST_DEPTH>() - 1) / multi_width<TZ, PERSIST_DEPTH>();
    int t = 0, pass = 0, lp = 0;  // lp: the warm closure's current lagged values are in a.lag_alt
    while (t < nsteps) {
        StepArgs b = a;
        if (pass & 1) {
            b.src = a.dst;
            b.dst = (void *)a.src;
            b.ez_in = a.ez_out;
            b.ez_out = (double *)a.ez_in;
        }
        if (lp) {
            b.lag = a.lag_alt;
            b.lag_alt = a.lag;
        }
        if (t > 0) {
            b.do_pull = 1;
            b.do_maxwell = 1;
            b.lag_init = 0;
        }
        b.step = a.step + t;
        if (t > 0 && nsteps - t >= PERSIST_DEPTH) {
            for (int tile = blockIdx.x; tile < ntilesd; tile += gridDim.x)
                step1d_multi<CL, ST, TZ, PERSIST_DEPTH>(b, tile, s_g, s_xc);
            t += PERSIST_DEPTH;
            lp ^= 1;
        } else if (t > 0 && nsteps - t >= 2) {
            for (int tile = blockIdx.x; tile < ntiles2; tile += gridDim.x) step1d_multi<CL, ST, TZ, 2>(b, tile, s_g, s_xc);
            t += 2;
            lp ^= 1;
        } else {
            for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) step1d_tile<CL, ST, TZ>(b, tile, s_g);
            t += 1;
        }
        ++pass;
        __ockl_grid_sync();
    }
}

// Zeroth moments A_k = A_ref_k + sum_q s_{k,q} of the populations a node
// holds (eq. disc-moments-ade), each sum in the storage's arithmetic type in
// the order q = 0 .. Q-1.
template <class PopL, class ST>
__device__ __forceinline__ void moments_at(const ST *src, size_t nc, int idx, const double *aref, double *A)
{
    using CT = typename PopL::CT;
    constexpr int K = PopL::NK, Q = PopL::NQ;
    CT acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        CT v[K];
        PopL::ld_all(src, q, nc, idx, v);
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += v[k];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) A[k] = aref[k] + (double)acc[k];
}

// ---------------------------------------------------------------------------
// Finish: bring a mid-step state (f*^{n-1}, E^{n-1}, B^{n-3/2}) to the
// canonical one (f^n, E^n, B^{n-1/2}). Pass 1 streams f* into the other
// buffer and records J^n = -n^n u^n; in 1D it also finishes E_z. NT: the
// populations are stored with the non-temporal hint. On the 2D slab the
// workgroups are renumbered into XCD bands, so that row segments whose pulls
// share cache lines run on one L2 (4096 x 1024 warm FP32 533 -> 462 us, FP64
// 972 -> 949 us); the axisymmetric grid keeps the dispatch order, which
// measured faster there (421 against 434 us on 3000 x 600 warm FP64).
template <int DIM, int CL, class ST, bool NT = false>
__global__ void k_finish_pull(StepArgs a, double *jz, double *jx)
{
    using L = Lattice<DIM>;
    constexpr int Q = L::Q;
    constexpr int K = NScal<DIM, CL>::K;
    using PopL = Pops<ST, K, Q>;
    const int blk = (DIM == 2 && !a.axi) ? xcd_band_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int idx = blk * blockDim.x + threadIdx.x;
    if (idx >= a.ncell) return;
    const int gz = idx % a.nz, gx = idx / a.nz;
    const size_t nc = (size_t)a.ncell;
    const ST *src = (const ST *)a.src;
    ST *dst = (ST *)a.dst;
    using CT = typename Store<ST>::ct;
    double A[K];
    CT acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int sz = gz - L::ez(q);
        int sx = gx - L::ex(q), qs = q;
        // axisymmetric: the row below the axis is the mirror image of row 0
        const bool m = DIM == 2 && a.axi && sx < 0;
        if (m) { sx = -1 - sx; qs = Lattice<2>::mx(q); }
        const int c = fix_node(sx, a.nx, a.bcx) * a.nz + fix_node(sz, a.nz, a.bcz);
        CT v[K];
        PopL::ld_all(src, qs, nc, c, v);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (m && odd_in_r<CL>(k)) v[k] = -v[k] - (CT)(2.0 * L::w(q) * a.aref[k]);
            acc[k] += v[k];
        }
        PopL::template st_all<NT>(dst, q, nc, idx, v);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) A[k] = a.aref[k] + (double)acc[k];
    double uz, ux;
    if constexpr (CL == LEC) {
        LecRec r;
        lec_recover(A[0], A[1], DIM == 2 ? A[K - 1] : 0.0, a.a_lec, a.dcode, a.two_over_d, r);
        uz = r.uz;
        ux = r.ux;
    } else {
        WarmRec r;
        warm_recover<DIM>(A, r);
        uz = r.uz;
        ux = r.ux;
    }
    double ezn = 0.0;
    if (DIM == 1) {
        const double jb = driver_density<1>(a.drv, gz * a.delta, 0.0, (a.step - 0.5) * a.dt);
        ezn = a.ez_in[idx] + a.dt * (A[0] * uz + jb);
        a.ez_out[idx] = ezn;
    } else {
        jz[idx] = -A[0] * uz;
        jx[idx] = -A[0] * ux;
    }
    if (a.nonfinite) {
        // a non-finite population makes its scalar's sum non-finite
        double sa = 0.0;
        for (int k = 0; k < K; ++k) sa += A[k];
        if (!isfinite(sa) || !isfinite(uz) || !isfinite(ux) || !isfinite(ezn)) atomicOr(a.nonfinite, 1u);
    }
}

// Pass 2 (2D): B^{n-1/2} = (B^{n-3/2} - dt/2 curl E^{n-1}) - dt/2 curl E^{n-1}.
static __global__ void k_finish_b2d(StepArgs a)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.ncell) return;
    const int i = idx % a.nz, j = idx / a.nz;
    const int nz = a.nz, nx = a.nx, bz = a.bcz, bx = a.bcx;
    auto EZ = [&](int jj, int ii) { return a.ez_in[(size_t)fix_node(jj, nx, bx) * nz + fix_stag(ii, nz, bz)]; };
    auto EX = [&](int jj, int ii) { return a.ex_in[(size_t)fix_stag(jj, nx, bx) * nz + fix_node(ii, nz, bz)]; };
    const double hdt = 0.5 * a.dt, id = 1.0 / a.delta;
    const double curl = ((EX(j, i + 1) - EX(j, i)) - (EZ(j + 1, i) - EZ(j, i))) * id;
    const double b1 = a.by_in[idx] - hdt * curl;
    a.by_out[idx] = b1 - hdt * curl;
}

// Pass 3 (2D): E^n = E^{n-1} + dt (curl B^{n-1/2} - J^n - J_b^{n-1/2});
// axisymmetric: the E_z curl is (1/r) d_r (r B_phi).
static __global__ void k_finish_e2d(StepArgs a, const double *jz, const double *jx)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.ncell) return;
    const int i = idx % a.nz, j = idx / a.nz;
    const int nz = a.nz, nx = a.nx, bz = a.bcz, bx = a.bcx;
    auto BY = [&](int jj, int ii) { return a.by_out[(size_t)fix_stag(jj, nx, bx) * nz + fix_stag(ii, nz, bz)]; };
    auto JN = [&](const double *J, int jj, int ii) { return J[(size_t)fix_node(jj, nx, bx) * nz + fix_node(ii, nz, bz)]; };
    const double dt = a.dt, id = 1.0 / a.delta;
    const double th = (a.step - 0.5) * dt;
    const double jxe = 0.5 * (JN(jx, j, i) + JN(jx, j + 1, i));
    const double cx = -(BY(j, i) - BY(j, i - 1)) * id;
    const double exn = a.ex_in[idx] + dt * (cx - jxe);
    a.ex_out[idx] = exn;
    const double jze = 0.5 * (JN(jz, j, i) + JN(jz, j, i + 1));
    const double jb = -driver_density<2>(a.drv, (i + 0.5) * a.delta, node_x(j, nx, a.delta, a.axi), th);
    const double cz = a.axi ? ((j + 1.0) * BY(j, i) - (j > 0 ? j * BY(j - 1, i) : 0.0)) / ((j + 0.5) * a.delta)
                            : (BY(j, i) - BY(j - 1, i)) * id;
    const double ezn = a.ez_in[idx] + dt * (cz - jze - jb);
    a.ez_out[idx] = ezn;
    if (a.nonfinite && !(isfinite(ezn) && isfinite(exn) && isfinite(a.by_out[idx])))
        atomicOr(a.nonfinite, 1u);
}

// ---------------------------------------------------------------------------
// Initial populations f_q = f_eq_q(A_k, u) from staged scalars A [K][ncell]
// and velocity (uz, ux), stored as deviations from A_ref.
template <int DIM, int CL, class ST>
__global__ void k_init_pops(void *dst_, const double *A, const double *uzv, const double *uxv,
                            const double *aref, int ncell, double lam)
{
    using L = Lattice<DIM>;
    constexpr int Q = L::Q;
    constexpr int K = NScal<DIM, CL>::K;
    using PopL = Pops<ST, K, Q>;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ncell) return;
    ST *dst = (ST *)dst_;
    const size_t nc = (size_t)ncell;
    const double uz = uzv[idx], ux = DIM == 2 ? uxv[idx] : 0.0;
    const double uu = uz * uz + ux * ux;
    double Ak[K];
#pragma unroll
    for (int k = 0; k < K; ++k) Ak[k] = A[(size_t)k * nc + idx];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const double eu = uz * L::ez(q) + ux * L::ex(q);
        const double P = 3.0 * eu / lam + 4.5 * eu * eu / (lam * lam) - 1.5 * uu / (lam * lam);
        const double w = L::w(q);
        typename Store<ST>::ct v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = (typename Store<ST>::ct)(w * (Ak[k] - aref[k]) + w * Ak[k] * P);
        PopL::template st_all<false>(dst, q, nc, idx, v);
    }
}

// Observable at each node from canonical populations f^n.
template <int DIM, int CL, class ST>
__global__ void k_read_moment(StepArgs a, int which, double *out)
{
    using L = Lattice<DIM>;
    constexpr int Q = L::Q;
    constexpr int K = NScal<DIM, CL>::K;
    using PopL = Pops<ST, K, Q>;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.ncell) return;
    const size_t nc = (size_t)a.ncell;
    const ST *src = (const ST *)a.src;
    double A[K];
    moments_at<PopL>(src, nc, idx, a.aref, A);
    const double n = A[0];
    double v = 0.0;
    if constexpr (CL == LEC) {
        LecRec r;
        lec_recover(n, A[1], DIM == 2 ? A[K - 1] : 0.0, a.a_lec, a.dcode, a.two_over_d, r);
        switch (which) {
        case 0: v = n; break;
        case 1: v = r.uz; break;
        case 2: v = r.ux; break;
        case 3: v = r.gamma; break;
        case 4: v = r.n0; break;
        case 5: case 11: v = a.mu * r.phi; break;
        case 12: v = n * r.gamma * r.uz; break;
        case 13: v = n * r.gamma * r.ux; break;
        default: v = 0.0;
        }
    } else {
        WarmRec r;
        warm_recover<DIM>(A, r);
        const double g = 1.0 / sqrt(1.0 - (r.uz * r.uz + r.ux * r.ux));
        switch (which) {
        case 0: v = n; break;
        case 1: v = r.uz; break;
        case 2: v = r.ux; break;
        case 3: v = g; break;
        case 4: v = n / g; break;
        case 5: v = r.thyy; break;
        case 6: v = r.lam; break;
        case 7: v = r.thzz; break;
        case 8: v = r.thxx; break;
        case 9: v = r.thyy; break;
        case 10: v = r.thxz; break;
        case 11: v = warm_ppar(r); break;
        case 12: v = n * g * r.uz; break;
        case 13: v = n * g * r.ux; break;
        default: v = 0.0;
        }
    }
    out[idx] = v;
}

// Fields of the canonical state: raw Yee (ghost slots as copies) or node
// averages of E^n and B^n = B^{n-1/2} - dt/2 curl E^n.
template <int DIM>
__global__ void k_read_field(StepArgs a, int which, int at_nodes, double *out)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.ncell) return;
    if (DIM == 1) {
        out[idx] = which == 0 ? a.ez_in[idx] : 0.0;
        return;
    }
    const int i = idx % a.nz, j = idx / a.nz;
    const int nz = a.nz, nx = a.nx, bz = a.bcz, bx = a.bcx;
    auto EZ = [&](int jj, int ii) { return a.ez_in[(size_t)fix_node(jj, nx, bx) * nz + fix_stag(ii, nz, bz)]; };
    auto EX = [&](int jj, int ii) { return a.ex_in[(size_t)fix_stag(jj, nx, bx) * nz + fix_node(ii, nz, bz)]; };
    auto BH = [&](int jj, int ii) { return a.by_in[(size_t)fix_stag(jj, nx, bx) * nz + fix_stag(ii, nz, bz)]; };
    const double hdt = 0.5 * a.dt, id = 1.0 / a.delta;
    // B^n at a staggered slot: the copy rule picks the real slot first, then
    // the curl is taken there
    auto BN = [&](int jj, int ii) {
        jj = fix_stag(jj, nx, bx);
        ii = fix_stag(ii, nz, bz);
        const double curl = ((EX(jj, ii + 1) - EX(jj, ii)) - (EZ(jj + 1, ii) - EZ(jj, ii))) * id;
        return BH(jj, ii) - hdt * curl;
    };
    double v;
    if (!at_nodes) {
        v = which == 0 ? EZ(j, i) : (which == 1 ? EX(j, i) : BH(j, i));
    } else {
        const double ez = 0.5 * (EZ(j, i - 1) + EZ(j, i));
        // axisymmetric row 0: E_r and B_phi vanish on the axis below it
        const bool ax = a.axi && j == 0;
        const double ex = ax ? 0.5 * EX(j, i) : 0.5 * (EX(j - 1, i) + EX(j, i));
        const double by = ax ? 0.25 * (BN(j, i) + BN(j, i - 1))
                             : 0.25 * (BN(j, i) + BN(j, i - 1) + BN(j - 1, i) + BN(j - 1, i - 1));
        v = which == 0 ? ez : (which == 1 ? ex : (which == 2 ? by : ex - by));
    }
    out[idx] = v;
}

// ---------------------------------------------------------------------------
// Diagnostics: per-node FP64 terms (n dV, field energy, kinetic energy,
// Gauss residual^2, non-finite flag, |u| / Lambda) reduced across each
// wavefront with butterfly exchanges, then across the workgroup's waves in
// wave order, then over the workgroups by one final workgroup (each lane
// takes a fixed strided set of partials in order). Sums for the first five,
// a maximum in which NaN wins for the last. The order is fixed, so the
// result is bitwise reproducible.
constexpr int NDIAG = 6;
constexpr int DIAG_THREADS = 256;

// Reduce v[NDIAG] over the workgroup; thread 0 gets the result.
__device__ __forceinline__ void block_reduce_diag(double *v, double (*red)[DIAG_THREADS / 64])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 0; d < NDIAG - 1; ++d) v[d] = wave_sum(v[d]);
    v[NDIAG - 1] = wave_max_nan(v[NDIAG - 1]);
    if (lane == 0)
#pragma unroll
        for (int d = 0; d < NDIAG; ++d) red[d][wave] = v[d];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int d = 0; d < NDIAG; ++d) v[d] = red[d][0];
        for (int w = 1; w < DIAG_THREADS / 64; ++w) {
#pragma unroll
            for (int d = 0; d < NDIAG - 1; ++d) v[d] += red[d][w];
            const double o = red[NDIAG - 1][w];
            if (o > v[NDIAG - 1] || o != o) v[NDIAG - 1] = o;
        }
    }
}

template <int DIM, int CL, class ST>
__global__ __launch_bounds__(DIAG_THREADS) void k_diag_partial(StepArgs a, double *part)
{
    using L = Lattice<DIM>;
    constexpr int Q = L::Q;
    constexpr int K = NScal<DIM, CL>::K;
    using PopL = Pops<ST, K, Q>;
    __shared__ double red[NDIAG][DIAG_THREADS / 64];
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    double v[NDIAG] = {0, 0, 0, 0, 0, 0};
    if (idx < a.ncell) {
        const size_t nc = (size_t)a.ncell;
        const ST *src = (const ST *)a.src;
        double A[K];
        moments_at<PopL>(src, nc, idx, a.aref, A);
        const double n = A[0];
        double uz, ux;
        if constexpr (CL == LEC) {
            LecRec r;
            lec_recover(n, A[1], DIM == 2 ? A[K - 1] : 0.0, a.a_lec, a.dcode, a.two_over_d, r);
            uz = r.uz;
            ux = r.ux;
        } else {
            WarmRec r;
            warm_recover<DIM>(A, r);
            uz = r.uz;
            ux = r.ux;
        }
        const double uu = uz * uz + ux * ux;
        const double g = 1.0 / sqrt(1.0 - uu);
        const int i = idx % a.nz, j = idx / a.nz;
        const int nz = a.nz, nx = a.nx, bz = a.bcz, bx = a.bcx;
        const bool axi = DIM == 2 && a.axi;
        // axisymmetric: 2 pi r per unit cell area; nodes at r_j, E_r and B_phi at r_{j+1/2}
        const double dV0 = DIM == 1 ? a.delta : a.delta * a.delta;
        const double dV = axi ? 2.0 * M_PI * node_x(j, nx, a.delta, true) * dV0 : dV0;
        const double dVh = axi ? 2.0 * M_PI * node_x(j + 0.5, nx, a.delta, true) * dV0 : dV0;
        double fe, div;
        const double t = a.step * a.dt;
        const double rho = 1.0 - n - driver_density<DIM>(a.drv, i * a.delta, node_x(j, nx, a.delta, axi), t);
        if (DIM == 1) {
            const double e = a.ez_in[idx];
            fe = 0.5 * e * e * dV;
            div = (a.ez_in[fix_node(i + 1, nz, bz)] - a.ez_in[fix_node(i - 1, nz, bz)]) * (0.5 / a.delta);
        } else {
            // energy of the real Yee slots only
            const bool rz = bz == BC_PERIODIC || i < nz - 1, rx = bx == BC_PERIODIC || j < nx - 1;
            const double ez = a.ez_in[idx], ex = a.ex_in[idx], by = a.by_in[idx];
            if (axi)
                fe = (rz ? 0.5 * ez * ez : 0.0) * dV + ((rx ? 0.5 * ex * ex : 0.0) + (rz && rx ? 0.5 * by * by : 0.0)) * dVh;
            else
                fe = ((rz ? 0.5 * ez * ez : 0.0) + (rx ? 0.5 * ex * ex : 0.0) + (rz && rx ? 0.5 * by * by : 0.0)) * dV;
            auto EZ = [&](int jj, int ii) { return a.ez_in[(size_t)fix_node(jj, nx, bx) * nz + fix_stag(ii, nz, bz)]; };
            auto EX = [&](int jj, int ii) { return a.ex_in[(size_t)fix_stag(jj, nx, bx) * nz + fix_node(ii, nz, bz)]; };
            if (axi) {
                const double em = j > 0 ? EX(j - 1, i) : 0.0;
                div = (EZ(j, i) - EZ(j, i - 1)) / a.delta + ((j + 1.0) * EX(j, i) - j * em) / ((j + 0.5) * a.delta);
            } else {
                div = (EZ(j, i) - EZ(j, i - 1)) / a.delta + (EX(j, i) - EX(j - 1, i)) / a.delta;
            }
        }
        const bool bad = !isfinite(n) || !isfinite(uz) || !isfinite(ux) || !isfinite(a.ez_in[idx]) ||
                         (DIM == 2 && (!isfinite(a.ex_in[idx]) || !isfinite(a.by_in[idx])));
        v[0] = n * dV;
        v[1] = fe;
        v[2] = n * (g - 1.0) * dV;
        v[3] = (div - rho) * (div - rho);
        v[4] = bad ? 1.0 : 0.0;
        v[5] = sqrt(uu) / a.lam;
    }
    block_reduce_diag(v, red);
    if (threadIdx.x == 0)
        for (int d = 0; d < NDIAG; ++d) part[(size_t)d * gridDim.x + blockIdx.x] = v[d];
}

static __global__ __launch_bounds__(DIAG_THREADS) void k_diag_final(const double *part, int nblocks, double *out)
{
    __shared__ double red[NDIAG][DIAG_THREADS / 64];
    double v[NDIAG] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += DIAG_THREADS) {
        for (int d = 0; d < NDIAG - 1; ++d) v[d] += part[(size_t)d * nblocks + b];
        const double o = part[(size_t)(NDIAG - 1) * nblocks + b];
        if (o > v[NDIAG - 1] || o != o) v[NDIAG - 1] = o;
    }
    block_reduce_diag(v, red);
    if (threadIdx.x == 0)
        for (int d = 0; d < NDIAG; ++d) out[d] = v[d];
}

// Analytic field of the bunch alone at t = 0 (Sec. 5). 1D: E_z(z) = alpha
// times the integral of the profile from z to +infinity, evaluated per slice.
// 2D: E_z = 0, E_x = -g(zeta) sigma_x sqrt(pi/2) erf(x / (sqrt 2 sigma_x)),
// B_y = E_x taken at t = -dt/2. Axisymmetric: the cylindrical Gauss law
// (1/r) d_r (r E_r) = -n_b gives E_r = -g(zeta) sigma_r^2 (1 - e^{-r^2/2 sigma_r^2}) / r.
template <int DIM>
__global__ void k_init_fields(StepArgs a, double *ez, double *ex, double *by)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.ncell) return;
    const int i = idx % a.nz, j = idx / a.nz;
    const Driver &d = a.drv;
    if (DIM == 1) {
        const double zeta = i * a.delta - d.z0;
        const double sz = d.sigma_z, c = sz * sqrt(M_PI / 2.0), r2s = sqrt(2.0) * sz;
        double acc;
        if (d.nslices <= 0) {
            acc = c * erfc(zeta / r2s);
        } else {
            const double h = (d.slice_zmax - d.slice_zmin) / d.nslices;
            acc = 0.0;
            for (int k = 0; k < d.nslices; ++k) {
                double lo = d.slice_zmin + k * h, hi = d.slice_zmin + (k + 1) * h;
                if (zeta >= hi) continue;
                if (zeta > lo) lo = zeta;
                acc += d.slice_w[k] * c * (erf(hi / r2s) - erf(lo / r2s));
            }
        }
        ez[idx] = d.alpha * acc;
        return;
    }
    const double xh = node_x(j + 0.5, a.nx, a.delta, a.axi) - d.x0;
    const double sx = d.sigma_x;
    const double tr = a.axi ? -sx * sx * (1.0 - exp(-xh * xh / (2.0 * sx * sx))) / xh
                            : -sx * sqrt(M_PI / 2.0) * erf(xh / (sqrt(2.0) * sx));
    const double ze = i * a.delta - d.z0;
    const double zb = (i + 0.5) * a.delta - d.z0 + 0.5 * a.dt;
    ez[idx] = 0.0;
    ex[idx] = driver_profile(d, ze) * tr;
    by[idx] = driver_profile(d, zb) * tr;
}

}  // namespace lbw
