// lbw_adjoint.hpp -- discrete adjoint of one 2D local-equilibrium step
// (transposed Jacobian of the map (f^n, E^n, B^{n-1/2}) -> (f^{n+1}, E^{n+1},
// B^{n+1/2}) of lbw_step) and the derivatives of the driver terms with
// respect to the slice weights. All adjoint arithmetic is FP64.
//
// Forward map of one step (Sec. 2.2, Sec. 3.1, Sec. 5; the fused kernel and
// the finish kernels compute exactly this):
//   S1 A_k = sum_q f_kq                       S2 (u, phi) = recovery(A)
//   S3 Bh = B - dt/2 curlE(E);  node fields En_z, En_x (2-point), Bn_y (4-point of Bh)
//   S5 F_z = -mu d_z phi - n (En_z + u_x Bn_y), F_x = -mu d_x phi - n (En_x - u_z Bn_y)
//   S6 f*_kq = (1 - omega) f_kq + omega w_q A_k (1 + P_q(u)) + dt w_q F_k
//   S7 f'_kq(c) = f*_kq(fix(c - e_q))         S8 m' = n' u' = recovery(A')
//   S9 B' = Bh - dt/2 curlE(E);  E'_x = E_x + dt (curlB_x(B') + (m'_x(c) + m'_x(c + x))/2)
//      E'_z = E_z + dt (curlB_z(B') + (m'_z(c) + m'_z(c + z))/2 + n_b(w))
// The reverse step runs S9..S1 backwards. Every read of the forward goes
// through a boundary rule (copy ghost or wrap); its transpose gathers, for a
// target slot, from every slot whose read lands there (pre1 below), so the
// reverse step is a pure gather: deterministic, no atomics.
#pragma once

#include "lbw_device.hpp"

namespace lbw {

struct AdjArgs {
    const void *fn, *fn1;                 // populations of the states at steps n and n+1 (canonical,
                                          // or the post-collision values of the step before)
    const double *ez, *ex, *by;           // E^n, B^{n-1/2} (Yee arrays)
    double *lf, *lez, *lex, *lby;         // adjoint of the state, updated in place
    double *s_byt, *s_fs, *s_fz, *s_fx;   // scratch: adjoint of B', of f*, of F
    double *s_enz, *s_enx, *s_bny, *s_bht;
    double *s_ab;                         // adjoint of A at n+1 (3 planes), added in the stream gather
    double *s_bhf;                        // forward Bh = B^{n-1/2} - dt/2 curl E^n at every slot
    double *s_x;                          // adjoint(B') + adjoint(Bh)
    const double *aref;
    double *grad;                         // d loss / d slice weight, accumulated
    int nz, nx, ncell, bcz, bcx;
    double delta, dt, omega, lam, mu, a_lec, two_over_d, dvel;
    int dcode;
    long step;                            // n
    Driver drv;
};

// Positions c in [0, n) whose read of index c + d lands on y under the node
// (copy ghost) or staggered rule, or the periodic wrap; at most 3.
__device__ __forceinline__ int pre1(int y, int d, int n, int bc, bool stag, int *out)
{
    if (bc == BC_PERIODIC) {
        int c = (y - d) % n;
        out[0] = c < 0 ? c + n : c;
        return 1;
    }
    // away from the ends no clamped read lands on y (|d| <= 1): y - d only
    if (y >= 1 && y <= n - 3) {
        out[0] = y - d;
        return 1;
    }
    const int cand[4] = {y - d, 0, n - 2, n - 1};
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = cand[k];
        if (c < 0 || c >= n) continue;
        bool dup = false;
        for (int m = 0; m < cnt; ++m) dup |= out[m] == c;
        if (dup) continue;
        const int v = stag ? fix_stag(c + d, n, bc) : fix_node(c + d, n, bc);
        if (v == y) out[cnt++] = c;
    }
    return cnt;
}

// Sum over every slot c of X[c] whose read at (c_x + dx, c_z + dz) lands on
// (jy, iy) under the given rules (sx / sz: staggered along x / z).
__device__ __forceinline__ double gather2(const double *X, int jy, int iy, int dx, int dz, bool sx, bool sz,
                                          int nx, int nz, int bcx, int bcz)
{
    int cx[3], cz[3];
    const int nxc = pre1(jy, dx, nx, bcx, sx, cx);
    const int nzc = pre1(iy, dz, nz, bcz, sz, cz);
    double acc = 0.0;
    for (int a = 0; a < nxc; ++a)
        for (int b = 0; b < nzc; ++b) acc += X[(size_t)cx[a] * nz + cz[b]];
    return acc;
}

// Forward recovery of one node with the quantities its derivative needs.
// u = kappa a_1 with kappa = 1 / (n gamma h), h = 1 + s, s = a (n/gamma)^{2/D},
// t = (2/D) s; the root p of p h(p, n) = P = |a_1|/n has
// dp/dP = 1 / (h - t p^2/gamma^2), dp/dn = -(p t / n) dp/dP (implicit function
// of the fixed-point equation of Sec. 3.1).
struct LecJ {
    double n, az, ax, uz, ux, g, p, h, t, kappa, phi, dpdP, dpdn, P;
};

__device__ __forceinline__ void lec_jac(double n, double az, double ax, const AdjArgs &a, LecJ &J)
{
    LecRec r;
    lec_recover(n, az, ax, a.a_lec, a.dcode, a.two_over_d, r);
    J.n = n;
    J.az = az;
    J.ax = ax;
    J.uz = r.uz;
    J.ux = r.ux;
    J.g = r.gamma;
    J.phi = r.phi;
    J.p = r.gamma * hypot(r.uz, r.ux);
    const double x = n / r.gamma;
    const double s = a.a_lec * (a.dcode == 3 ? cbrt(x * x) : (a.dcode == 1 ? x * x : pow(x, a.two_over_d)));
    J.h = 1.0 + s;
    J.t = a.two_over_d * s;
    J.kappa = 1.0 / (n * r.gamma * J.h);
    const double Dd = J.h - J.t * J.p * J.p / (J.g * J.g);
    J.dpdP = 1.0 / Dd;
    J.dpdn = -(J.p * J.t / n) * J.dpdP;
    J.P = (ax == 0.0 ? fabs(az) : hypot(az, ax)) / n;
}

// Reverse of the recovery: adjoints (uzb, uxb) of u, phib of phi and nb of n
// itself -> adjoints of (A_0, A_1z, A_1x). The p-derivatives of kappa and phi
// carry a factor p, which cancels the 1/|a_1| of d|a_1|, so nothing divides
// by |a_1| (cells at rest have a_1 = 0).
__device__ __forceinline__ void lec_recover_adj(const LecJ &J, double uzb, double uxb, double phib, double nb,
                                                double e_phi, double *Ab)
{
    const double g2 = J.g * J.g;
    const double kb = uzb * J.az + uxb * J.ax;
    const double kp = -J.kappa * (1.0 - J.t / J.h) / g2;  // (d kappa / d p) / p
    const double kn = -(J.kappa / J.n) * (1.0 + J.t / J.h);
    const double pp = -e_phi * J.phi / g2;                 // (d phi / d p) / p
    const double pn = e_phi * J.phi / J.n;
    const double qv = kb * kp + phib * pp;                 // adjoint of p, divided by p
    nb += kb * kn + phib * pn;
    nb += qv * J.p * J.dpdn;
    nb -= qv * J.p * J.dpdP * J.P / J.n;
    const double c1 = qv * J.dpdP / (J.n * J.n * J.h);
    Ab[0] = nb;
    Ab[1] = J.kappa * uzb + c1 * J.az;
    Ab[2] = J.kappa * uxb + c1 * J.ax;
}

template <class ST>
__device__ __forceinline__ void moments3(const void *f, const AdjArgs &a, size_t c, double *A)
{
    using L = Lattice<2>;
    const ST *src = (const ST *)f;
    const size_t nc = (size_t)a.ncell;
    using PopL = Pops<ST, 3, L::Q>;
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        typename PopL::CT v[3];
        PopL::ld_all(src, q, nc, (int)c, v);
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k] += (double)v[k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) A[k] = a.aref[k] + acc[k];
}

// The same sums for populations held as the previous step's post-collision
// values f*: node (j, i)'s population q is the one streamed from
// (j - e_x, i - e_z) under the boundary rule (S7), as the canonicalisation
// copies it; the same values in the same order, so the same bits.
template <class ST>
__device__ __forceinline__ void moments3_pulled(const void *f, const AdjArgs &a, int j, int i, double *A)
{
    using L = Lattice<2>;
    const ST *src = (const ST *)f;
    const size_t nc = (size_t)a.ncell;
    using PopL = Pops<ST, 3, L::Q>;
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        const int c = fix_node(j - L::ex(q), a.nx, a.bcx) * a.nz + fix_node(i - L::ez(q), a.nz, a.bcz);
        typename PopL::CT v[3];
        PopL::ld_all(src, q, nc, c, v);
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k] += (double)v[k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) A[k] = a.aref[k] + acc[k];
}

// Moments of the state the pointer holds: canonical (PULLED = false) or the
// post-collision populations of the step before (PULLED = true).
template <class ST, bool PULLED>
__device__ __forceinline__ void moments_of(const void *f, const AdjArgs &a, int j, int i, size_t c, double *A)
{
    if constexpr (PULLED) moments3_pulled<ST>(f, a, j, i, A);
    else moments3<ST>(f, a, c, A);
}

// Forward node fields at node (j, i) from E^n and B^{n-1/2} (S3).
struct NodeF {
    double ez, ex, by;
};

__device__ __forceinline__ double curl_e_at(const AdjArgs &a, int j, int i)
{
    const int nz = a.nz, nx = a.nx, bz = a.bcz, bx = a.bcx;
    auto EZ = [&](int jj, int ii) { return a.ez[(size_t)fix_node(jj, nx, bx) * nz + fix_stag(ii, nz, bz)]; };
    auto EX = [&](int jj, int ii) { return a.ex[(size_t)fix_stag(jj, nx, bx) * nz + fix_node(ii, nz, bz)]; };
    return ((EX(j, i + 1) - EX(j, i)) - (EZ(j + 1, i) - EZ(j, i))) / a.delta;
}

__device__ __forceinline__ NodeF node_fields_at(const AdjArgs &a, int j, int i)
{
    const int nz = a.nz, nx = a.nx, bz = a.bcz, bx = a.bcx;
    auto EZ = [&](int jj, int ii) { return a.ez[(size_t)fix_node(jj, nx, bx) * nz + fix_stag(ii, nz, bz)]; };
    auto EX = [&](int jj, int ii) { return a.ex[(size_t)fix_stag(jj, nx, bx) * nz + fix_node(ii, nz, bz)]; };
    auto BH = [&](int jj, int ii) { return a.s_bhf[(size_t)fix_stag(jj, nx, bx) * nz + fix_stag(ii, nz, bz)]; };
    NodeF f;
    f.ez = 0.5 * (EZ(j, i - 1) + EZ(j, i));
    f.ex = 0.5 * (EX(j - 1, i) + EX(j, i));
    f.by = 0.25 * (BH(j, i) + BH(j, i - 1) + BH(j - 1, i) + BH(j - 1, i - 1));
    return f;
}

// The three FP64 adjoint populations of direction q at node c (the adjoint
// state and the scratch of the stream kernel), in the layout of the FP64
// population buffers (Pops: scalars 0 and 1 as one 16-byte pair per
// direction and node, scalar 2 in planes of its own after the pairs).
__device__ __forceinline__ void adj_pops_ld(const double *b, int q, size_t nc, size_t c, double *v)
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 w = ((const d2 *)(b + (size_t)q * nc * 2))[c];
    v[0] = w.x;
    v[1] = w.y;
    v[2] = b[(size_t)(18 + q) * nc + c];
}
__device__ __forceinline__ void adj_pops_st(double *b, int q, size_t nc, size_t c, const double *v)
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2 w;
    w.x = v[0];
    w.y = v[1];
    ((d2 *)(b + (size_t)q * nc * 2))[c] = w;
    b[(size_t)(18 + q) * nc + c] = v[2];
}

// The per-node kernels below (one thread per node or slot y, no LDS) take
// their workgroups in XCD bands, so that row segments whose gathers share
// cache lines run on one L2 (reverse step 115.8 -> 110.9 us on 1024 x 256,
// the same bits).

// (a) Reverse of S9 and S8 at every slot/node y: adjoint of B', the currents'
// adjoint m'b, through the recovery at n+1 into the adjoint of A' (every
// population of the node gets it; the stream gather adds it).

// PULLED: fn1 holds the post-collision populations of step n (f*^n).
template <class ST, bool PULLED>
__global__ __launch_bounds__(256) void k_adj_maxwell(AdjArgs a)
{
    const int y = xcd_band_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (y >= a.ncell) return;
    const int iy = y % a.nz, jy = y / a.nz;
    const int nz = a.nz, nx = a.nx, bz = a.bcz, bx = a.bcx;
    const double dt = a.dt, id = 1.0 / a.delta;
    // B'(slot y) is read by curlB_z of E'_z at (j, i) and (j - 1, i), by curlB_x
    // of E'_x at (j, i) and (j, i - 1)
    double byt = a.lby[y];
    byt += dt * id * (gather2(a.lez, jy, iy, 0, 0, true, true, nx, nz, bx, bz) -
                      gather2(a.lez, jy, iy, -1, 0, true, true, nx, nz, bx, bz));
    byt -= dt * id * (gather2(a.lex, jy, iy, 0, 0, true, true, nx, nz, bx, bz) -
                      gather2(a.lex, jy, iy, 0, -1, true, true, nx, nz, bx, bz));
    a.s_byt[y] = byt;
    // m'_z(node y) enters E'_z at (j, i) and at (j, i - 1) (edge averages)
    const double mzb = 0.5 * dt * (gather2(a.lez, jy, iy, 0, 0, false, false, nx, nz, bx, bz) +
                                   gather2(a.lez, jy, iy, 0, 1, false, false, nx, nz, bx, bz));
    const double mxb = 0.5 * dt * (gather2(a.lex, jy, iy, 0, 0, false, false, nx, nz, bx, bz) +
                                   gather2(a.lex, jy, iy, 1, 0, false, false, nx, nz, bx, bz));
    double A[3];
    moments_of<ST, PULLED>(a.fn1, a, jy, iy, y, A);
    LecJ J;
    lec_jac(A[0], A[1], A[2], a, J);
    // m = n u: adjoint of u is n m_b, n gets m_b . u
    double Ab[3];
    lec_recover_adj(J, A[0] * mzb, A[0] * mxb, 0.0, mzb * J.uz + mxb * J.ux, 1.0 + a.two_over_d, Ab);
    const size_t nc = (size_t)a.ncell;
#pragma unroll
    for (int k = 0; k < 3; ++k) a.s_ab[(size_t)k * nc + y] = Ab[k];
    // forward Bh at this slot, for the node fields of the collision kernel
    a.s_bhf[y] = a.by[y] - 0.5 * dt * curl_e_at(a, jy, iy);
}

// (b) Reverse of S7 (streaming): adjoint of f* gathered from the nodes that
// pulled from y (their adjoint of f' plus their adjoint of A'); adjoint of
// the forcing F_k = dt sum_q w_q fs_b.
__global__ __launch_bounds__(256) void k_adj_stream(AdjArgs a)
{
    using L = Lattice<2>;
    const int y = xcd_band_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (y >= a.ncell) return;
    const int iy = y % a.nz, jy = y / a.nz;
    const size_t nc = (size_t)a.ncell;
    double Fb[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        int cx[3], cz[3];
        const int nxc = pre1(jy, -L::ex(q), a.nx, a.bcx, false, cx);
        const int nzc = pre1(iy, -L::ez(q), a.nz, a.bcz, false, cz);
        double acc[3] = {0.0, 0.0, 0.0};
        for (int u = 0; u < nxc; ++u)
            for (int v = 0; v < nzc; ++v) {
                const size_t c = (size_t)cx[u] * a.nz + cz[v];
                double l[3];
                adj_pops_ld(a.lf, q, nc, c, l);
#pragma unroll
                for (int k = 0; k < 3; ++k) acc[k] += l[k] + a.s_ab[(size_t)k * nc + c];
            }
        adj_pops_st(a.s_fs, q, nc, (size_t)y, acc);
#pragma unroll
        for (int k = 0; k < 3; ++k) Fb[k] += L::w(q) * acc[k];
    }
    a.s_fz[y] = a.dt * Fb[1];
    a.s_fx[y] = a.dt * Fb[2];
}

// (c) Reverse of S6, S5, S2, S1 at node y: collision, forcing (the gradient
// of phi gathers the forcing adjoint of the neighbours), recovery; writes
// the adjoint of f^n and the node-field adjoints.
// PULLED: fn holds the post-collision populations of step n - 1 (f*^{n-1}).
template <class ST, bool PULLED>
__global__ __launch_bounds__(256) void k_adj_collide(AdjArgs a)
{
    using L = Lattice<2>;
    const int y = xcd_band_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (y >= a.ncell) return;
    const int iy = y % a.nz, jy = y / a.nz;
    const int nz = a.nz, nx = a.nx, bz = a.bcz, bx = a.bcx;
    const size_t nc = (size_t)a.ncell;
    double A[3];
    moments_of<ST, PULLED>(a.fn, a, jy, iy, y, A);
    LecJ J;
    lec_jac(A[0], A[1], A[2], a, J);
    const NodeF nf = node_fields_at(a, jy, iy);
    const double uz = J.uz, ux = J.ux, n = A[0];
    const double om = a.omega, lam = a.lam;
    const double c1 = 3.0 / lam, c2 = 9.0 / (lam * lam), c3 = 3.0 / (lam * lam);
    // collision adjoint
    double Ab[3], uzb = 0.0, uxb = 0.0;
    // the 27 adjoint populations stay in registers for the write-back below
    // (162 VGPRs, 3 waves per SIMD as with one scalar at a time and a second
    // read; one read: 134 -> 122 us per reverse step)
    double fsr[3][9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        double l[3];
        adj_pops_ld(a.s_fs, q, nc, (size_t)y, l);
#pragma unroll
        for (int k = 0; k < 3; ++k) fsr[k][q] = l[k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double sa = 0.0, sz = 0.0, sx = 0.0;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const double fb = fsr[k][q];
            const double ez = L::ez(q), ex = L::ex(q);
            const double eu = uz * ez + ux * ex;
            const double P = c1 * eu + 0.5 * c2 * eu * eu - 0.5 * c3 * (uz * uz + ux * ux);
            const double wf = L::w(q) * fb;
            sa += wf * (1.0 + P);
            sz += wf * (c1 * ez + c2 * eu * ez - c3 * uz);
            sx += wf * (c1 * ex + c2 * eu * ex - c3 * ux);
        }
        Ab[k] = om * sa;
        uzb += om * A[k] * sz;
        uxb += om * A[k] * sx;
    }
    // forcing adjoint (F_0 = 0)
    const double fzb = a.s_fz[y], fxb = a.s_fx[y];
    double nb = -fzb * (nf.ez + ux * nf.by) - fxb * (nf.ex - uz * nf.by);
    uxb += -n * nf.by * fzb;
    uzb += n * nf.by * fxb;
    a.s_enz[y] = -n * fzb;
    a.s_enx[y] = -n * fxb;
    a.s_bny[y] = -n * (ux * fzb - uz * fxb);
    // phi at y is read by d_z at (j, i - 1) (as i + 1) and (j, i + 1) (as i - 1)
    const double k2 = a.mu / (2.0 * a.delta);
    const double phib = -k2 * (gather2(a.s_fz, jy, iy, 0, 1, false, false, nx, nz, bx, bz) -
                               gather2(a.s_fz, jy, iy, 0, -1, false, false, nx, nz, bx, bz)) -
                        k2 * (gather2(a.s_fx, jy, iy, 1, 0, false, false, nx, nz, bx, bz) -
                              gather2(a.s_fx, jy, iy, -1, 0, false, false, nx, nz, bx, bz));
    double Rb[3];
    lec_recover_adj(J, uzb, uxb, phib, nb, 1.0 + a.two_over_d, Rb);
    const double keep = 1.0 - om;
    double tot[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) tot[k] = Ab[k] + Rb[k];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        double l[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) l[k] = keep * fsr[k][q] + tot[k];
        adj_pops_st(a.lf, q, nc, (size_t)y, l);
    }
}

// (d1) Adjoint of Bh at every staggered slot: from B' (S9) and from the
// 4-point node average of S3; it is also the adjoint of B^{n-1/2}.
__global__ __launch_bounds__(256) void k_adj_bh(AdjArgs a)
{
    const int y = xcd_band_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (y >= a.ncell) return;
    const int iy = y % a.nz, jy = y / a.nz;
    const int nz = a.nz, nx = a.nx, bz = a.bcz, bx = a.bcx;
    double b = a.s_byt[y];
    b += 0.25 * (gather2(a.s_bny, jy, iy, 0, 0, true, true, nx, nz, bx, bz) +
                 gather2(a.s_bny, jy, iy, 0, -1, true, true, nx, nz, bx, bz) +
                 gather2(a.s_bny, jy, iy, -1, 0, true, true, nx, nz, bx, bz) +
                 gather2(a.s_bny, jy, iy, -1, -1, true, true, nx, nz, bx, bz));
    a.s_bht[y] = b;
    a.s_x[y] = a.s_byt[y] + b;  // X: the adjoint both dt/2 curls of E^n see
}

// (d2) Adjoint of E^n (identity, node averages, and the two dt/2 curls of S3
// and S9, both taken of X = adjoint(B') + adjoint(Bh)) and of B^{n-1/2}.
__global__ __launch_bounds__(256) void k_adj_fields(AdjArgs a)
{
    const int y = xcd_band_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (y >= a.ncell) return;
    const int iy = y % a.nz, jy = y / a.nz;
    const int nz = a.nz, nx = a.nx, bz = a.bcz, bx = a.bcx;
    const double hdi = 0.5 * a.dt / a.delta;
    auto gX = [&](int dx, int dz, bool sx, bool sz) { return gather2(a.s_x, jy, iy, dx, dz, sx, sz, nx, nz, bx, bz); };
    // E_z slot (x node, z staggered): read by En_z at (j, i + 1) as i - 1 and at
    // (j, i); by curlE at (j - 1, i) as j + 1 (minus) and at (j, i) (plus)
    double ez = a.lez[y];
    ez += 0.5 * (gather2(a.s_enz, jy, iy, 0, -1, false, true, nx, nz, bx, bz) +
                 gather2(a.s_enz, jy, iy, 0, 0, false, true, nx, nz, bx, bz));
    ez -= hdi * (-gX(1, 0, false, true) + gX(0, 0, false, true));
    // E_x slot (x staggered, z node)
    double ex = a.lex[y];
    ex += 0.5 * (gather2(a.s_enx, jy, iy, -1, 0, true, false, nx, nz, bx, bz) +
                 gather2(a.s_enx, jy, iy, 0, 0, true, false, nx, nz, bx, bz));
    ex -= hdi * (gX(0, 1, true, false) - gX(0, 0, true, false));
    a.lez[y] = ez;
    a.lex[y] = ex;
    a.lby[y] = a.s_bht[y];
}


// Slice of position (i + zoff) delta at time t (the forward's slice_weight
// index rule), or -1 outside the slice span.
__device__ __forceinline__ int slice_of(const Driver &d, double zeta)
{
    if (!(zeta >= d.slice_zmin && zeta < d.slice_zmax)) return -1;
    int k = (int)floor((zeta - d.slice_zmin) / (d.slice_zmax - d.slice_zmin) * d.nslices);
    return k < 0 ? 0 : (k >= d.nslices ? d.nslices - 1 : k);
}

// Slice derivatives of the driver current: E'_z gains dt n_b at
// ((i + 1/2) delta, x_j, t^{n+1/2}), n_b = alpha w_s exp(-e). One workgroup per
// column of the bunch window [i0, i0 + gridDim.x) sums over x (tree
// reduction, fixed order) into col[i], with the column's slice in
// col[nz + i]; then the first thread of each slice's run of columns adds
// them in order.
__global__ __launch_bounds__(256) void k_adj_drv_cols(AdjArgs a, const double *lez, double t, double zoff, int i0,
                                                      double *col)
{
    __shared__ double red[256];
    const int i = i0 + blockIdx.x;
    const Driver &d = a.drv;
    const double zeta = (i + zoff) * a.delta - d.z0 - t;
    const double ez2 = zeta * zeta * d.inv2sz2;
    double acc = 0.0;
    for (int j = threadIdx.x; j < a.nx; j += blockDim.x) {
        const double xx = (j - 0.5 * (a.nx - 1)) * a.delta - d.x0;
        const double e = ez2 + xx * xx * d.inv2sx2;
        if (e <= 746.0) acc += lez[(size_t)j * a.nz + i] * exp(-e);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        col[i] = red[0];
        col[a.nz + i] = (double)slice_of(d, zeta);
    }
}

// Initial fields: E_x(j, i) = g(zeta_e) tr(j), B_y(j, i) = g(zeta_b) tr(j) with
// g = alpha w_s exp(-zeta^2 / 2 sigma_z^2); col[i] = exp(-zeta^2 / 2 sigma_z^2)
// sum_j lambda tr(j) and the column's slice in col[nz + i].
__global__ __launch_bounds__(256) void k_adj_init_cols(AdjArgs a, const double *lam, double t, double zoff, int i0,
                                                       double *col)
{
    __shared__ double red[256];
    const int i = i0 + blockIdx.x;
    const Driver &d = a.drv;
    double acc = 0.0;
    for (int j = threadIdx.x; j < a.nx; j += blockDim.x) {
        const double xh = (j + 0.5 - 0.5 * (a.nx - 1)) * a.delta - d.x0;
        const double tr = -d.sigma_x * sqrt(M_PI / 2.0) * erf(xh / (sqrt(2.0) * d.sigma_x));
        acc += lam[(size_t)j * a.nz + i] * tr;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double zeta = (i + zoff) * a.delta - d.z0 - t;
        col[i] = red[0] * exp(-zeta * zeta * d.inv2sz2);
        col[a.nz + i] = (double)slice_of(d, zeta);
    }
}

// grad[s] += scale * alpha * sum of col[i] over the window's columns of slice
// s. zeta grows with the column and slice_of does not decrease with zeta on
// the slice range (columns outside it hold -1), so the columns of one slice
// form one run: the thread at a run's first column adds the run in column
// order, starting from zero, and only it writes grad[s].
__global__ __launch_bounds__(256) void k_adj_slices(AdjArgs a, const double *col, int i0, int i1, double scale)
{
    const int i = i0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= i1) return;
    const double *ks = col + a.nz;
    const int s = (int)ks[i];
    if (s < 0 || (i > i0 && (int)ks[i - 1] == s)) return;
    double acc = 0.0;
    for (int c = i; c < i1 && (int)ks[c] == s; ++c) acc += col[c];
    a.grad[s] += scale * a.drv.alpha * acc;
}

}  // namespace lbw
