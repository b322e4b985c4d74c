// lbw_device.hpp -- device-side building blocks of the moment-matching LB
// step for warm relativistic plasma wakes (Simeoni et al., arXiv 2309.04872):
// lattice tables, equilibrium, closure recoveries, driver, boundary indexing.
// Written for gfx950 (CDNA4): 64-wide wavefronts, FP64 recovery in VGPRs.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

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
};

// Number of advected scalars (eq. lb-ade-lec-comps-A, eq. lb-ade-warmc-comps-A):
// LEC (n, A_z[, A_x]); WARMC 1D (n, n lambda, n lambda u_z, lambda theta^zz),
// 2D (n, n lambda, n lambda u_z, n lambda u_x, lambda theta^zz, ^xx, ^yy, ^xz).
template <int DIM, int CL> struct NScal {
    static constexpr int K = CL == LEC ? 1 + DIM : (DIM == 1 ? 4 : 8);
};

// ---------------------------------------------------------------------------
// Population storage. Every stored value is a deviation s = f - w_q A_ref_k
// from a per-scalar reference (A_ref = 0 for FP64 and FP32 storage); CT is
// the arithmetic type of the collision.
template <class ST> struct Store;
template <> struct Store<double> {
    using ct = double;
    __device__ static double ld(const double *p, size_t i) { return p[i]; }
    __device__ static void st(double *p, size_t i, double v) { p[i] = v; }
};
template <> struct Store<float> {
    using ct = float;
    __device__ static float ld(const float *p, size_t i) { return p[i]; }
    __device__ static void st(float *p, size_t i, float v) { p[i] = v; }
};
template <> struct Store<__half> {
    using ct = float;
    __device__ static float ld(const __half *p, size_t i) { return __half2float(p[i]); }
    __device__ static void st(__half *p, size_t i, float v) { p[i] = __float2half_rn(v); }
};

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

// ---------------------------------------------------------------------------
// Rigid bi-Gaussian driver at c along +z (eq. bunch-density, rms widths),
// optional piecewise-constant slice weights in zeta = z - z0 - t.
struct Driver {
    double alpha, sigma_z, sigma_x, z0, x0;
    double slice_zmin, slice_zmax;
    int nslices;
    const double *slice_w;  // device
};

__device__ __forceinline__ double driver_profile(const Driver &d, double zeta)
{
    double s = 1.0;
    if (d.nslices > 0) {
        if (!(zeta >= d.slice_zmin && zeta < d.slice_zmax)) return 0.0;
        int k = (int)floor((zeta - d.slice_zmin) / (d.slice_zmax - d.slice_zmin) * d.nslices);
        k = k < 0 ? 0 : (k >= d.nslices ? d.nslices - 1 : k);
        s = d.slice_w[k];
    }
    return d.alpha * s * exp(-zeta * zeta / (2.0 * d.sigma_z * d.sigma_z));
}

template <int DIM>
__device__ __forceinline__ double driver_density(const Driver &d, double z, double x, double t)
{
    if (d.alpha == 0.0) return 0.0;
    double g = driver_profile(d, z - d.z0 - t);
    if (DIM == 2) {
        double dx = x - d.x0;
        g *= exp(-dx * dx / (2.0 * d.sigma_x * d.sigma_x));
    }
    return g;
}

// ---------------------------------------------------------------------------
// LEC transport-velocity recovery (Sec. 3.1). Fixed point on |p|:
// p_{k+1} = |A_1| / (n h(n / gamma_k)), gamma_k = sqrt(1 + p_k^2),
// h(n0) = 1 + (1 + D/2) mu n0^{2/D}; stop when |p_{k+1} - p_k| <= 1e-15 (1 + p),
// at most 64 passes, else bisection on [0, |A_1|/n]. The vector p keeps the
// direction of A_1. Returns false when the fallback was used.
__device__ __forceinline__ double pow_2_over_d(double x, int dcode, double two_over_d)
{
    if (dcode == 1) return x * x;          // D = 1
    if (dcode == 3) {                      // D = 3
        double c = cbrt(x);
        return c * c;
    }
    return pow(x, two_over_d);
}

struct LecRec {
    double uz, ux, gamma, n0, phi;  // phi = n0^{1+2/D}
};

__device__ __forceinline__ bool lec_recover(double n, double a1z, double a1x, double a_lec,
                                            int dcode, double two_over_d, LecRec &r)
{
    double P = sqrt(a1z * a1z + a1x * a1x) / n;
    double p = P;
    bool ok = false;
    for (int it = 0; it < 64; ++it) {
        double g = sqrt(1.0 + p * p);
        double pn = P / (1.0 + a_lec * pow_2_over_d(n / g, dcode, two_over_d));
        double dp = pn - p;
        p = pn;
        if (fabs(dp) <= 1e-15 * (1.0 + pn)) {
            ok = true;
            break;
        }
    }
    if (!ok) {
        double lo = 0.0, hi = P;
        for (int k = 0; k < 200 && hi - lo > 1e-17 * (1.0 + hi); ++k) {
            double mid = 0.5 * (lo + hi);
            double g = sqrt(1.0 + mid * mid);
            double res = mid * (1.0 + a_lec * pow_2_over_d(n / g, dcode, two_over_d)) - P;
            if (res > 0.0) hi = mid; else lo = mid;
        }
        p = 0.5 * (lo + hi);
    }
    double g = sqrt(1.0 + p * p);
    double scale = P > 0.0 ? p / (P * n * g) : 0.0;  // u = p_vec / gamma, p_vec = A_1 p / (n P)
    r.uz = a1z * scale;
    r.ux = a1x * scale;
    r.gamma = g;
    r.n0 = n / g;
    r.phi = r.n0 * pow_2_over_d(r.n0, dcode, two_over_d);
    return ok;
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
    double n = A[0], nl = A[1];
    r.lam = nl / n;
    if (DIM == 1) {
        r.uz = A[2] / nl;
        r.ux = 0.0;
        r.thzz = A[3] / r.lam;
        r.thxx = r.thyy = r.thxz = 0.0;
        r.luz = A[2] / n;
        r.lux = 0.0;
    } else {
        r.uz = A[2] / nl;
        r.ux = A[3] / nl;
        r.thzz = A[4] / r.lam;
        r.thxx = A[5] / r.lam;
        r.thyy = A[6] / r.lam;
        r.thxz = A[7] / r.lam;
        r.luz = A[2] / n;
        r.lux = A[3] / n;
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
