// lbw_device.hpp -- device-side building blocks of the moment-matching LB
// step for warm relativistic plasma wakes (Simeoni et al., arXiv 2309.04872):
// lattice tables, equilibrium, closure recoveries, driver, boundary indexing.
// Written for gfx950 (CDNA4): 64-wide wavefronts, FP64 recovery in VGPRs.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>
#include <type_traits>

namespace lbw {

constexpr int LEC = 0;
constexpr int WARMC = 1;
constexpr int BC_OPEN = 0;
constexpr int BC_PERIODIC = 1;

// ---------------------------------------------------------------------------
// Velocity stencils: the 19-velocity 3D stencil of the paper (Sec. 2.1,
// Fig. 1) projected on one axis (D1Q3: 2/3, 1/6, 1/6) and on a plane
// (D2Q9: 4/9, 1/9, 1/36). Order of the 2D set: rest, +z, -z, +x, -x,
// (+z,+x), (-z,-x), (+z,-x), (-z,+x).
template <int DIM> struct Lattice;
template <> struct Lattice<1> {
    static constexpr int Q = 3;
    __device__ static constexpr int ez(int q) { return q == 0 ? 0 : (q == 1 ? 1 : -1); }
    __device__ static constexpr int ex(int) { return 0; }
    __device__ static constexpr double w(int q) { return q == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
};
template <> struct Lattice<2> {
    static constexpr int Q = 9;
    __device__ static constexpr int ez(int q)
    {
        return (q == 1 || q == 5 || q == 7) ? 1 : ((q == 2 || q == 6 || q == 8) ? -1 : 0);
    }
    __device__ static constexpr int ex(int q)
    {
        return (q == 3 || q == 5 || q == 8) ? 1 : ((q == 4 || q == 6 || q == 7) ? -1 : 0);
    }
    __device__ static constexpr double w(int q)
    {
        return q == 0 ? 4.0 / 9.0 : (q < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
    // direction with e_x reversed (reflection through the axis x = 0)
    __device__ static constexpr int mx(int q)
    {
        return q == 3 ? 4 : q == 4 ? 3 : q == 5 ? 7 : q == 7 ? 5 : q == 6 ? 8 : q == 8 ? 6 : q;
    }
};

// Number of advected scalars (eq. lb-ade-lec-comps-A, eq. lb-ade-warmc-comps-A):
// LEC (n, A_z[, A_x]); WARMC 1D (n, n lambda, n lambda u_z, lambda theta^zz),
// 2D (n, n lambda, n lambda u_z, n lambda u_x, lambda theta^zz, ^xx, ^yy, ^xz).
template <int DIM, int CL> struct NScal {
    static constexpr int K = CL == LEC ? 1 + DIM : (DIM == 1 ? 4 : 8);
};

// ---------------------------------------------------------------------------
// Population storage. Every stored value is a deviation s = f - w_q A_ref_k
// from a per-scalar reference (A_ref = 0 for FP64 storage, the uniform rest
// state for FP32 and FP16 storage); CT is the arithmetic type of the collision.
template <class ST> struct Store;
// Loads and stores take a uniform plane pointer and a 32-bit node offset.
// st_nt: the same store with the non-temporal hint (streamed past the caches).
// rnd(v): the value a store of v followed by a load returns.
template <> struct Store<double> {
    using ct = double;
    __device__ static double ld(const double *p, int i) { return p[i]; }
    __device__ static void st(double *p, int i, double v) { p[i] = v; }
    __device__ static void st_nt(double *p, int i, double v) { __builtin_nontemporal_store(v, p + i); }
    __device__ static double rnd(double v) { return v; }
};
template <> struct Store<float> {
    using ct = float;
    __device__ static float ld(const float *p, int i) { return p[i]; }
    __device__ static void st(float *p, int i, float v) { p[i] = v; }
    __device__ static void st_nt(float *p, int i, float v) { __builtin_nontemporal_store(v, p + i); }
    __device__ static float rnd(float v) { return v; }
};
template <> struct Store<__half> {
    using ct = float;
    __device__ static float ld(const __half *p, int i) { return __half2float(p[i]); }
    __device__ static void st(__half *p, int i, float v) { p[i] = __float2half_rn(v); }
    __device__ static void st_nt(__half *p, int i, float v)
    {
        __builtin_nontemporal_store(__half_as_ushort(__float2half_rn(v)), (unsigned short *)p + i);
    }
    __device__ static float rnd(float v) { return __half2float(__float2half_rn(v)); }
};

// Layout of the K x Q population planes over nc nodes. Scalars are held in
// groups of G (as many as fill 16 bytes, at most K, a power of two: FP64
// pairs; FP32 groups of 4, FP16 groups of 8 for the warm closure; pairs for
// the local equilibrium's three scalars), the G populations of one group,
// direction q and node c side by side: element ((j Q + q) nc + c) G + r of
// scalar k = j G + r. A scalar left over (the local equilibrium's third)
// keeps a plane of its own after the groups, element (k' Q + q) nc + c. A
// pull of direction q then brings a whole group with one 16-byte access, and
// its store is one 16-byte store, instead of G separate ones (the warm FP64
// step 1141 -> 1076 us, FP32 664 -> 567 us, FP16 485 -> 361 us on
// 4096 x 1024; each stored value and its rounding are those of Store<ST>).
template <class ST> struct RawOf {
    using type = ST;
};
template <> struct RawOf<__half> {
    using type = unsigned short;
};
template <class ST, int K, int Q> struct Pops {
    using CT = typename Store<ST>::ct;
    using RT = typename RawOf<ST>::type;
    static constexpr int G0 = 16 / (int)sizeof(ST);
    static constexpr int G = (G0 >= 8 && K >= 8) ? 8 : (G0 >= 4 && K >= 4) ? 4 : (G0 >= 2 && K >= 2) ? 2 : 1;
    static constexpr int KP = K / G * G;  // scalars held in groups of G
    static constexpr int NK = K, NQ = Q;
    // uniform pointer to population (k, q) of node 0, and the element step
    // from one node to the next
    template <class P> __device__ static P *plane(P *b, int k, int q, size_t nc)
    {
        if (k < KP) return b + (size_t)((k / G) * Q + q) * nc * G + (k % G);
        return b + (size_t)KP * Q * nc + (size_t)((k - KP) * Q + q) * nc;
    }
    __device__ static constexpr int step(int k) { return k < KP ? G : 1; }
    __device__ static CT ld(const ST *b, int k, int q, size_t nc, int c)
    {
        return Store<ST>::ld(plane(b, k, q, nc), c * step(k));
    }
    __device__ static void st(ST *b, int k, int q, size_t nc, int c, CT v)
    {
        Store<ST>::st(plane(b, k, q, nc), c * step(k), v);
    }
    __device__ static CT from_raw(RT r)
    {
        if constexpr (std::is_same<ST, __half>::value) return __half2float(__ushort_as_half(r));
        else return r;
    }
    __device__ static RT to_raw(CT v)
    {
        if constexpr (std::is_same<ST, __half>::value) return __half_as_ushort(__float2half_rn(v));
        else return v;
    }
    // every scalar of direction q at node c (v[k] = population k), and back;
    // NT: stores with the non-temporal hint
    __device__ static void ld_all(const ST *b, int q, size_t nc, int c, CT *v)
    {
        if constexpr (G > 1) {
            typedef RT VG __attribute__((ext_vector_type(G)));
#pragma unroll
            for (int k = 0; k < KP; k += G) {
                const VG w = ((const VG *)plane(b, k, q, nc))[c];
#pragma unroll
                for (int r = 0; r < G; ++r) v[k + r] = from_raw(w[r]);
            }
        }
#pragma unroll
        for (int k = KP; k < K; ++k) v[k] = Store<ST>::ld(plane(b, k, q, nc), c);
    }
    template <bool NT> __device__ static void st_all(ST *b, int q, size_t nc, int c, const CT *v)
    {
        if constexpr (std::is_same<ST, __half>::value && G > 1) {
            // FP16: each pair packed into a 32-bit word by its own two
            // conversions, so that every value is rounded to FP16 once from
            // the FP32 result of its own expression
            typedef unsigned VW __attribute__((ext_vector_type(G / 2)));
#pragma unroll
            for (int k = 0; k < KP; k += G) {
                VW w;
#pragma unroll
                for (int r = 0; r < G; r += 2)
                    w[r / 2] = (unsigned)to_raw(v[k + r]) | ((unsigned)to_raw(v[k + r + 1]) << 16);
                VW *p = (VW *)plane(b, k, q, nc) + c;
                if constexpr (NT) __builtin_nontemporal_store(w, p);
                else *p = w;
            }
        } else if constexpr (G > 1) {
            typedef RT VG __attribute__((ext_vector_type(G)));
#pragma unroll
            for (int k = 0; k < KP; k += G) {
                VG w;
#pragma unroll
                for (int r = 0; r < G; ++r) w[r] = to_raw(v[k + r]);
                VG *p = (VG *)plane(b, k, q, nc) + c;
                if constexpr (NT) __builtin_nontemporal_store(w, p);
                else *p = w;
            }
        }
#pragma unroll
        for (int k = KP; k < K; ++k) {
            if constexpr (NT) Store<ST>::st_nt(plane(b, k, q, nc), c, v[k]);
            else Store<ST>::st(plane(b, k, q, nc), c, v[k]);
        }
    }
};

// Workgroups are dispatched round-robin over the 8 XCDs of the chip. Renumber
// them so that XCD k sweeps one contiguous band of tiles: neighbouring tiles,
// whose halos overlap, then share one L2.
__device__ __forceinline__ int xcd_band_tile(int b, int nblocks)
{
    const int x = b & 7, slot = b >> 3;
    const int base = nblocks >> 3, rem = nblocks & 7;
    return x * base + (x < rem ? x : rem) + slot;
}

// ---------------------------------------------------------------------------
// FP64 reductions across the 64 lanes of a wavefront: butterfly exchanges
// (__shfl_xor, lane i pairs with lane i ^ o). Both partners of a pair add the
// same two values, so every lane ends with the same bits and the result does
// not depend on timing. Lanes outside the data must pass the identity.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// Maximum in which a NaN wins, so that a non-finite value is never hidden.
__device__ __forceinline__ double wave_max_nan(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o, 64);
        if (w > v || w != w) v = w;
    }
    return v;
}

// ---------------------------------------------------------------------------
// Boundary indexing. Open boundaries copy the nearest bulk node (eq. open-bc);
// periodic boundaries wrap. Yee arrays along a staggered direction have n - 1
// real half-integer slots between the n nodes under open boundaries.
__device__ __forceinline__ int fix_node(int i, int n, int bc)
{
    if (bc == BC_PERIODIC) {
        i %= n;
        return i < 0 ? i + n : i;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}
__device__ __forceinline__ int fix_stag(int i, int n, int bc)
{
    if (bc == BC_PERIODIC) return fix_node(i, n, bc);
    return i < 0 ? 0 : (i >= n - 1 ? n - 2 : i);
}
// Same rules without wrapping: the unwrapped coordinate a tile computes at.
__device__ __forceinline__ int map_node(int i, int n, int bc)
{
    return bc == BC_PERIODIC ? i : (i < 0 ? 0 : (i >= n ? n - 1 : i));
}
__device__ __forceinline__ int map_stag(int i, int n, int bc)
{
    return bc == BC_PERIODIC ? i : (i < 0 ? 0 : (i >= n - 1 ? n - 2 : i));
}

// Transverse node coordinate: slab x_j = (j - (nx-1)/2) delta; axisymmetric
// r_j = (j + 1/2) delta, so that the axis is the face below row 0 (ghost row
// -1 is the mirror image of row 0) and 1/r stays finite on every node.
__device__ __forceinline__ double node_x(double j, int nx, double delta, bool axi)
{
    return axi ? (j + 0.5) * delta : (j - 0.5 * (nx - 1)) * delta;
}

// ---------------------------------------------------------------------------
// Rigid bi-Gaussian driver at c along +z (eq. bunch-density, rms widths),
// optional piecewise-constant slice weights in zeta = z - z0 - t.
struct Driver {
    double alpha, sigma_z, sigma_x, z0, x0;
    double slice_zmin, slice_zmax;
    double inv2sz2, inv2sx2;  // 1 / (2 sigma^2)
    int nslices;
    const double *slice_w;  // device
};

__device__ __forceinline__ double slice_weight(const Driver &d, double zeta)
{
    if (d.nslices <= 0) return 1.0;
    if (!(zeta >= d.slice_zmin && zeta < d.slice_zmax)) return 0.0;
    int k = (int)floor((zeta - d.slice_zmin) / (d.slice_zmax - d.slice_zmin) * d.nslices);
    k = k < 0 ? 0 : (k >= d.nslices ? d.nslices - 1 : k);
    return d.slice_w[k];
}

__device__ __forceinline__ double driver_profile(const Driver &d, double zeta)
{
    return d.alpha * slice_weight(d, zeta) * exp(-zeta * zeta * d.inv2sz2);
}

// n_b(z, x, t); exp(-e) is exactly zero in FP64 once e exceeds 745.2, so the
// exponential is skipped there (most of the grid) without changing a bit.
template <int DIM>
__device__ __forceinline__ double driver_density(const Driver &d, double z, double x, double t)
{
    if (d.alpha == 0.0) return 0.0;
    const double zeta = z - d.z0 - t;
    double e = zeta * zeta * d.inv2sz2;
    if (DIM == 2) {
        const double dx = x - d.x0;
        e += dx * dx * d.inv2sx2;
    }
    if (e > 746.0) return 0.0;
    return d.alpha * slice_weight(d, zeta) * exp(-e);
}

// ---------------------------------------------------------------------------
// LEC transport-velocity recovery (Sec. 3.1): find |p| with
// p (1 + a (n / gamma)^{2/D}) = P, P = |A_1| / n, gamma = sqrt(1 + p^2),
// a = (1 + D/2) mu; the vector p keeps the direction of A_1.
//  D = 1: the paper's fixed point p_{k+1} = P / (1 + a n^2 / (1 + p_k^2)) from
//         p_0 = P (written without square roots), stopped when
//         |p_{k+1} - p_k| <= 1e-15 (1 + p), at most 64 passes, else bisection on
//         [0, P]. Several roots can exist for dense relativistic cells; the
//         fixed point selects the one the paper's iteration reaches.
//  D = 3: the root is unique (d/dp of the left side >= 1/3). Newton's method on
//         d = gamma^{1/3} - 1 >= 0, where with c = 1 + d, b = a n^{2/3},
//         S(c) = 1 + c + ... + c^5 (so that p^2 = c^6 - 1 = d S without
//         cancellation) and h = 1 + b / c^2:
//         G(d) = d S h^2 - P^2 = (p h)^2 - P^2 = 0, increasing in d;
//         no root or cube root inside the loop, quadratic convergence from the
//         lower bound p = P / (1 + b); stopped once a step falls below 1e-12 d,
//         at most 12 passes, else bisection. Quotients use rcp64 (hardware
//         reciprocal estimate plus two Newton-Raphson corrections).
//  other D: the fixed point with pow().
// Returns false when a fallback was needed.
struct LecRec {
    double uz, ux, gamma, n0, phi;  // phi = n0^{1+2/D}
};

__device__ __forceinline__ double lec_bisect(double n, double P, double a, int dcode, double two_over_d)
{
    double lo = 0.0, hi = P;
    for (int k = 0; k < 200 && hi - lo > 1e-17 * (1.0 + hi); ++k) {
        const double mid = 0.5 * (lo + hi);
        const double g2 = 1.0 + mid * mid;
        const double s = dcode == 1 ? n * n / g2 : pow(n / sqrt(g2), two_over_d);
        if (mid * (1.0 + a * s) - P > 0.0) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// 1/x to FP64 accuracy: the hardware estimate refined by two Newton-Raphson
// corrections (no IEEE division sequence).
__device__ __forceinline__ double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ bool lec_recover(double n, double a1z, double a1x, double a_lec,
                                            int dcode, double two_over_d, LecRec &r)
{
    // |A_1| without squaring tiny momenta (their squares would underflow)
    const double amax = fmax(fabs(a1z), fabs(a1x));
    const double amag = a1x == 0.0 ? fabs(a1z) : (amax < 1e-150 ? hypot(a1z, a1x) : sqrt(a1z * a1z + a1x * a1x));
    double p, g, n0, phi, ig = 1.0;
    bool ok = false;
    if (dcode == 3) {
        const double in = rcp64(n);
        const double P = amag * in;
        const double n23 = cbrt(n * n);
        const double b = a_lec * n23;
        const double P2 = P * P;
        const double p0 = P * rcp64(1.0 + b);
        double d = cbrt(sqrt(1.0 + p0 * p0)) - 1.0;
        // |p| < 1e-100: gamma = 1 far below rounding, p = P / (1 + b) exactly
        // (this also keeps subnormal P^2 out of the relative stopping test)
        if (P < 1e-100) {
            d = 0.0;
            ok = true;
        }
        for (int it = 0; it < 12 && !ok; ++it) {
            const double c = 1.0 + d, ic = rcp64(c);
            const double S = 1.0 + c * (1.0 + c * (1.0 + c * (1.0 + c * (1.0 + c))));
            const double dS = 1.0 + c * (2.0 + c * (3.0 + c * (4.0 + 5.0 * c)));
            const double h = 1.0 + b * ic * ic;          // 1 + a (n / gamma)^{2/3}
            const double G = d * S * h * h - P2;          // (p h)^2 - P^2, increasing in d
            const double dG = (S + d * dS) * h * h - 4.0 * d * S * h * b * ic * ic * ic;
            double dn = d - G * rcp64(dG);
            if (dn < 0.0) dn = 0.0;
            const double step = fabs(dn - d);
            d = dn;
            // quadratic convergence: after a step below 1e-12 d the iterate is
            // exact to rounding (a tighter test would chase rounding noise in G)
            if (step <= 1e-12 * d || step == 0.0) {
                ok = true;
                break;
            }
        }
        const double c = 1.0 + d, ic = rcp64(c);
        const double S = 1.0 + c * (1.0 + c * (1.0 + c * (1.0 + c * (1.0 + c))));
        // u = p_vec / gamma = A_1 p / (|A_1| gamma)
        double scale;
        if (ok && P < 1e-100) {
            // p / |A_1| = 1 / (n (1 + b)): no reciprocal of a |A_1| that may be subnormal
            p = p0;
            g = 1.0;
            n0 = n;
            phi = n0 * n23;
            scale = in * rcp64(1.0 + b);
        } else if (ok) {
            p = sqrt(d * S);
            g = c * c * c;
            ig = ic * ic * ic;
            n0 = n * ig;
            phi = n0 * (n23 * (ic * ic));
            scale = p * ig * rcp64(amag);  // |A_1| >= 1e-100 n here
        } else {
            p = lec_bisect(n, P, a_lec, dcode, two_over_d);
            g = sqrt(1.0 + p * p);
            ig = 1.0 / g;
            n0 = n * ig;
            phi = n0 * cbrt(n0 * n0);
            scale = P > 0.0 ? p / (P * n * g) : 0.0;
        }
        r.uz = a1z * scale;
        r.ux = a1x * scale;
        r.gamma = g;
        r.n0 = n0;
        r.phi = phi;
        return ok;
    } else {
        const double P = amag / n;
        const double an2 = dcode == 1 ? a_lec * n * n : 0.0;
        p = P;
        for (int it = 0; it < 64; ++it) {
            const double g2 = 1.0 + p * p;
            const double pn = dcode == 1 ? P * g2 / (g2 + an2)
                                         : P / (1.0 + a_lec * pow(n / sqrt(g2), two_over_d));
            const double dp = pn - p;
            p = pn;
            if (fabs(dp) <= 1e-15 * (1.0 + pn)) {
                ok = true;
                break;
            }
        }
        if (!ok) p = lec_bisect(n, P, a_lec, dcode, two_over_d);
        g = sqrt(1.0 + p * p);
        n0 = n / g;
        phi = dcode == 1 ? n0 * n0 * n0 : n0 * pow(n0, two_over_d);
        const double scale = P > 0.0 ? p / (P * n * g) : 0.0;  // u = p_vec / gamma
        r.uz = a1z * scale;
        r.ux = a1x * scale;
        r.gamma = g;
        r.n0 = n0;
        r.phi = phi;
        return ok;
    }
}

// WARMC recovery (Sec. 4.1, App. A): lambda = (n lambda)/n, u from n lambda u,
// theta^{ij} from lambda theta^{ij}; eq. traces4 gives theta^{0i} = u_j theta^{ij}
// and theta^{00} = u_i theta^{0i}.
struct WarmRec {
    double lam, uz, ux, thzz, thxx, thyy, thxz, th0z, th0x, th00, luz, lux;
};

template <int DIM>
__device__ __forceinline__ void warm_recover(const double *A, WarmRec &r)
{
    // two reciprocals (rcp64) instead of a division per quantity
    const double n = A[0], nl = A[1];
    const double in = rcp64(n), inl = rcp64(nl);
    const double ilam = n * inl;  // 1 / lambda
    r.lam = nl * in;
    if (DIM == 1) {
        r.uz = A[2] * inl;
        r.ux = 0.0;
        r.thzz = A[3] * ilam;
        r.thxx = r.thyy = r.thxz = 0.0;
        r.luz = A[2] * in;
        r.lux = 0.0;
    } else {
        r.uz = A[2] * inl;
        r.ux = A[3] * inl;
        r.thzz = A[4] * ilam;
        r.thxx = A[5] * ilam;
        r.thyy = A[6] * ilam;
        r.thxz = A[7] * ilam;
        r.luz = A[2] * in;
        r.lux = A[3] * in;
    }
    r.th0z = r.ux * r.thxz + r.uz * r.thzz;
    r.th0x = r.ux * r.thxx + r.uz * r.thxz;
    r.th00 = r.ux * r.th0x + r.uz * r.th0z;
}

// Rest-frame longitudinal pressure (App. A item 3, r -> x, phi -> y).
__device__ __forceinline__ double warm_ppar(const WarmRec &r)
{
    double uu = r.ux * r.ux + r.uz * r.uz;
    return -(-(r.thxx + r.thzz) + r.th00 * uu + r.thyy * (1.0 + r.ux * r.ux)) / (1.0 + r.uz * r.uz);
}

}  // namespace lbw
