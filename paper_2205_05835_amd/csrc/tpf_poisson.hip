// Variable-density pressure Poisson solve, matrix free:
//     D(beta G p) = D f* - mean(D f*),   mean(p) = 0,   beta_a = 1 / A_a rho
// Conjugate gradients on the SPD form  A = -D(beta G .)  (zero-mean subspace),
// preconditioned by one geometric multigrid V-cycle: cell-centred coarsening
// by 2, rediscretised coarse operators with face-averaged beta, two damped
// Jacobi sweeps before and after the coarse correction, averaging
// restriction, piecewise-constant prolongation, fixed Jacobi sweeps on the
// coarsest grid in one workgroup.  Every piece is a fixed linear symmetric
// operator, so the V-cycle is a valid CG preconditioner.
//
// Fine level: beta is recomputed from phi inside every kernel (one field read
// instead of one per axis).  The kernels are fused along the data flow of one
// PCG iteration:
//   apply     p = z + beta p_old, q = A p, <p,q>
//   first     x += alpha p, r -= alpha q, <r,r>, z1 = omega r / d
//   sweep     z2 = z1 + omega (r - A z1) / d
//   restrict  r_c = mean over children of (r - A z2)     (coalesced, one
//             thread per fine cell, 2x2x2 sums in registers and LDS)
//   prolong   z3 = Z + omega (r - A Z) / d, Z = z2 + P z_c formed on the fly
//   sweep+dot z4 = z3 + omega (r - A z3) / d, <r, z4>
// Coarse levels use the same kernels with stored face coefficients.
//
// Mixed precision: the outer loop forms the residual in FP64 (FP64 beta from
// phi, FP64 right-hand side and iterate) and solves for the correction with
// the FP32 multigrid-PCG (defect correction).
//
// Scalars (alpha, beta, norms, the done flag) stay on the device; every
// solver kernel returns immediately once done is set, so the host queues
// several iterations between convergence checks.  Block partial sums go to
// two regions (offset 0 and offset max_blocks) summed by one finalize kernel.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <cmath>
#include <limits>
#include <type_traits>
#include <vector>

#include <cstdio>
#include <string>

#include "tpf_internal.hpp"

namespace tpf {

template <typename T>
static inline T* tp(void* p) { return static_cast<T*>(p); }

// 2 / s and 1 / s: correctly rounded in FP64 (parity path), hardware
// reciprocal in FP32 (inner solver of the mixed path)
__device__ __forceinline__ double two_over(double s) { return 2.0 / s; }
__device__ __forceinline__ float two_over(float s) { return 2.0f * __builtin_amdgcn_rcpf(s); }
// FP64: hardware reciprocal refined by two Newton steps (error within one
// ulp of 1/s, far cheaper than the IEEE divide sequence)
__device__ __forceinline__ double recip(double s) {
    double y = __builtin_amdgcn_rcp(s);
    double e = fma(-s, y, 1.0);
    y = fma(y, e, y);
    e = fma(-s, y, 1.0);
    return fma(y, e, y);
}
__device__ __forceinline__ float recip(float s) { return __builtin_amdgcn_rcpf(s); }

// block sums of two values to region 0 and region 1 (stride apart)
__device__ __forceinline__ void block_partials_2r(double (&v)[2], double* partials, long stride) {
    block_sum<2>(v);
    if (thread_linear() == 0) {
        const int b = block_linear();
        partials[b] = v[0];
        partials[stride + b] = v[1];
    }
}
__device__ __forceinline__ void block_partials_3r(double (&v)[3], double* partials, long stride) {
    block_sum<3>(v);
    if (thread_linear() == 0) {
        const int b = block_linear();
        partials[b] = v[0];
        partials[stride + b] = v[1];
        partials[2 * stride + b] = v[2];
    }
}

// The rounding level of an explicitly evaluated residual f - A x: each cell's
// value is a sum of face fluxes beta (x_nb - x_c) / h^2 that can be much
// larger than the result (a smooth pressure with a large jump, a density
// ratio of 1000), and FP64 evaluates it to within a few ulps of the sum of
// their magnitudes.  A solve whose explicit residual reaches
// RESID_FLOOR_ULPS u |A||x| (u = 2^-53, norms over all cells) is as
// converged as FP64 can tell.
constexpr double RESID_FLOOR_ULPS = 16.0;
template <typename S, int DIM, typename Fx>
__device__ __forceinline__ double abs_flux_sum(const S* bl, const S* bh, Fx x, S xc, S ih2) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a)
        s += fabs((double)bl[a] * (double)(xc - x(a, -1))) + fabs((double)bh[a] * (double)(x(a, 1) - xc));
    return s * (double)ih2;
}

// ---------------------------------------------------------------- coefficients
// Fine level: beta on the faces of a cell from the density law of phi.  Both
// policies return the half density h = rho / 2, and a face between cells
// lo < hi is always 1 / (h(lo) + h(hi)) in that operand order, so both cells
// of a face see bit-identical coefficients (symmetric A).  CoefPhi evaluates
// the law from phi; CoefRho reads h precomputed once per solve.  A face on a
// free-slip wall (the cell's wall bits) has coefficient 0: no flux through
// the wall, and the wrapped neighbour read there drops out.
template <typename T, typename S, bool W = false>
struct CoefPhi {
    static constexpr bool kWalls = W;     // cells carry wall bits (boxes with walls)
    const T* __restrict__ phi;
    S h2, dh;          // rho2 / 2, (rho1 - rho2) / 2
    S lo, hi;          // clamp bounds of phi: [0, 1], or +-inf when not clamping
    // the clamp in the storage precision T: the bounds (0, 1 or infinities)
    // and the conversion to S are exact, so this equals clamping in S
    __device__ __forceinline__ S hr(unsigned c) const {
        return h2 + dh * S(med3(ld(phi, c), T(lo), T(hi)));
    }
    template <int DIM>
    __device__ __forceinline__ void faces(const Cell& C, S* bl, S* bh) const {
        const S hc = hr(C.id);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            bl[a] = recip(hr(C.nb(a, -1)) + hc);
            bh[a] = recip(hc + hr(C.nb(a, 1)));
            if constexpr (W) {
                bl[a] = C.wall(a, -1) ? S(0) : bl[a];
                bh[a] = C.wall(a, 1) ? S(0) : bh[a];
            }
        }
    }
};

template <typename S, bool W = false>
struct CoefRho {
    static constexpr bool kWalls = W;
    const S* __restrict__ h;
    __device__ __forceinline__ S hr(unsigned c) const { return ld(h, c); }
    template <int DIM>
    __device__ __forceinline__ void faces(const Cell& C, S* bl, S* bh) const {
        const S hc = hr(C.id);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            bl[a] = recip(hr(C.nb(a, -1)) + hc);
            bh[a] = recip(hc + hr(C.nb(a, 1)));
            if constexpr (W) {
                bl[a] = C.wall(a, -1) ? S(0) : bl[a];
                bh[a] = C.wall(a, 1) ? S(0) : bh[a];
            }
        }
    }
};

// h = rho(phi) / 2 for the fine level, once per solve
template <typename T, typename S, bool W>
__global__ __launch_bounds__(BLOCK) void k_half_rho(long N, CoefPhi<T, S, W> cf, S* __restrict__ h) {
    // four consecutive cells per thread and pass, their loads issued together
    const long n4 = N / 4, t0 = (long)blockIdx.x * BLOCK + threadIdx.x, stride = (long)gridDim.x * BLOCK;
    for (long q = t0; q < n4; q += stride) {
        S v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = cf.hr((unsigned)(4 * q + u));
#pragma unroll
        for (int u = 0; u < 4; ++u) h[4 * q + u] = v[u];
    }
    for (long c = 4 * n4 + t0; c < N; c += stride) h[c] = cf.hr((unsigned)c);
}

template <typename S>
struct CoefStored {
    static constexpr bool kWalls = false;   // wall faces hold stored zeros
    const S* __restrict__ b0;
    const S* __restrict__ b1;
    const S* __restrict__ b2;
    template <int DIM>
    __device__ __forceinline__ void faces(const Cell& C, S* bl, S* bh) const {
        const S* b[3] = {b0, b1, b2};
        const unsigned c = C.id;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            bl[a] = ld(b[a], c);
            bh[a] = ld(b[a], C.nb(a, 1));
        }
    }
};

// (A x)[c] given the face coefficients; x(a, s) returns x at c + s e_a.  Also
// the diagonal d[c].
template <typename S, int DIM, typename Fx>
__device__ __forceinline__ S apply_at(const S* bl, const S* bh, Fx x, S xc, S ih2, S& diag) {
    S acc = S(0), dg = S(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        acc += bl[a] * (xc - x(a, -1)) - bh[a] * (x(a, 1) - xc);
        dg += bl[a] + bh[a];
    }
    diag = dg * ih2;
    return acc * ih2;
}

// ---------------------------------------------------------------- coefficients setup
// stored coefficients of level 1: mean of the fine face coefficients (same law
// as CoefPhi) over the fine faces covering each coarse face
template <typename Coef, typename S, int DIM>
__global__ __launch_bounds__(BLOCK) void k_beta_from_phi(Dims fd, Dims cd, Coef cf, S* b0, S* b1, S* b2) {
    Cell C;
    if (!cell_of_thread<Coef::kWalls>(cd, C)) return;
    S* b[3] = {b0, b1, b2};
    const int i0 = 2 * C.i, j0 = 2 * C.j, k0 = DIM == 3 ? 2 * C.k : 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        S s = S(0);
        for (int t = 0; t < (1 << (DIM - 1)); ++t) {
            int o[3] = {0, 0, 0};
            int q = 0;
            for (int e = 0; e < DIM; ++e)
                if (e != a) o[e] = (t >> q++) & 1;
            const Cell F = Coef::kWalls ? make_cell_w(fd, i0 + o[0], j0 + o[1], k0 + o[2])
                                        : make_cell(fd, i0 + o[0], j0 + o[1], k0 + o[2]);
            const S f = recip(cf.hr(F.nb(a, -1)) + cf.hr(F.id));
            s += F.wall(a, -1) ? S(0) : f;
        }
        b[a][C.id] = s * S(1.0 / (1 << (DIM - 1)));
    }
}

template <typename S, int DIM>
__global__ __launch_bounds__(BLOCK) void k_beta_coarsen(Dims fd, Dims cd, CoefStored<S> f, S* b0,
                                                        S* b1, S* b2) {
    Cell C;
    if (!cell_of_thread(cd, C)) return;
    const S* fb[3] = {f.b0, f.b1, f.b2};
    S* b[3] = {b0, b1, b2};
    const int i0 = 2 * C.i, j0 = 2 * C.j, k0 = DIM == 3 ? 2 * C.k : 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        S s = S(0);
        for (int t = 0; t < (1 << (DIM - 1)); ++t) {
            int o[3] = {0, 0, 0};
            int q = 0;
            for (int e = 0; e < DIM; ++e)
                if (e != a) o[e] = (t >> q++) & 1;
            const long fc = ((long)(k0 + o[2]) * fd.ny + (j0 + o[1])) * fd.nx + (i0 + o[0]);
            const long fmax = (long)fd.nx * fd.ny * fd.nz - 1;
            s += fb[a][fc < fmax ? fc : fmax];
        }
        b[a][C.id] = s * S(1.0 / (1 << (DIM - 1)));
    }
}

// ---------------------------------------------------------------- residuals
// r = -(b - mean) - A x in precision S (x and b FP64), stored as R;
// partials: |f|^2 -> region 0, |r|^2 -> region 1, and with FL the sum of
// squares of |A||x| (the rounding floor of the residual) -> region 2
template <typename Coef, typename S, typename R, int DIM, bool FL = true>
__global__ __launch_bounds__(BLOCK) void k_resid(Dims d, S ih2, Coef cf,
                                                 const double* __restrict__ b,
                                                 const double* __restrict__ x,
                                                 R* __restrict__ r,
                                                 const SolverScalars* __restrict__ sc,
                                                 double* __restrict__ partials, long stride) {
    Cell C;
    double v[3] = {0.0, 0.0, 0.0};
    if (cell_of_thread<Coef::kWalls>(d, C)) {
        S bl[3], bh[3], dg;
        cf.template faces<DIM>(C, bl, bh);
        const unsigned c = C.id;
        auto X = [&](int a, int s) { return S(ld(x, C.nb(a, s))); };
        const double f = -(ld(b, c) - sc->mean);
        const S xc = S(ld(x, c));
        const double rc = f - (double)apply_at<S, DIM>(bl, bh, X, xc, ih2, dg);
        st(r, c, R(rc));
        v[0] = f * f;
        v[1] = rc * rc;
        if (FL) {
            const double ax = abs_flux_sum<S, DIM>(bl, bh, X, xc, ih2);
            v[2] = ax * ax;
        }
    }
    block_partials_3r(v, partials, stride);
}

// ---------------------------------------------------------------- smoothing
// z = omega r / d  (first sweep from a zero guess)
template <typename Coef, typename S, int DIM>
__global__ __launch_bounds__(BLOCK) void k_jac_first(Dims d, S ih2, S omega, Coef cf,
                                                     const S* __restrict__ r, S* __restrict__ z,
                                                     const SolverScalars* __restrict__ sc) {
    if (sc->done) return;
    Cell C;
    if (!cell_of_thread<Coef::kWalls>(d, C)) return;
    S bl[3], bh[3], dg = S(0);
    cf.template faces<DIM>(C, bl, bh);
#pragma unroll
    for (int a = 0; a < DIM; ++a) dg += bl[a] + bh[a];
    const unsigned c = C.id;
    st(z, c, omega * ld(r, c) * recip(dg * ih2));
}

// PCG update fused with the first smoothing sweep of the V-cycle:
//   x += alpha p, r -= alpha q, <r,r> (region 0), z = omega r / d
// (XZ: x is zero before this update and not read)
template <typename Coef, typename S, typename X, int DIM, bool XZ = false>
__global__ __launch_bounds__(BLOCK) void k_jac_first_update(Dims d, S ih2, S omega, Coef cf,
                                                            X* __restrict__ x, S* __restrict__ r,
                                                            const S* __restrict__ p,
                                                            const S* __restrict__ q,
                                                            S* __restrict__ z,
                                                            const SolverScalars* __restrict__ sc,
                                                            double* __restrict__ partials) {
    if (sc->done) return;
    Cell C;
    double v[1] = {0.0};
    if (cell_of_thread<Coef::kWalls>(d, C)) {
        const unsigned c = C.id;
        const double alpha = sc->alpha;
        st(x, c, X((double)(XZ ? X(0) : ld(x, c)) + alpha * (double)ld(p, c)));
        const S rn = S((double)ld(r, c) - alpha * (double)ld(q, c));
        st(r, c, rn);
        v[0] = (double)rn * (double)rn;
        S bl[3], bh[3], dg = S(0);
        cf.template faces<DIM>(C, bl, bh);
#pragma unroll
        for (int a = 0; a < DIM; ++a) dg += bl[a] + bh[a];
        st(z, c, omega * rn * recip(dg * ih2));
    }
    block_partials<1>(v, partials);
}

template <typename S>
struct Vec2;
template <>
struct Vec2<float> { using type = float2; };
template <>
struct Vec2<double> { using type = double2; };

// zt = z + omega (r - A z) / d; DOT = 1 also emits <r, zt> to region 1 and
// <q, zt> to region 2 (stride apart) for the flexible-CG update.
template <typename Coef, typename S, int DIM, int DOT>
__global__ __launch_bounds__(BLOCK) void k_jac(Dims d, S ih2, S omega, Coef cf,
                                               const S* __restrict__ r, const S* __restrict__ z,
                                               S* __restrict__ zt, const S* __restrict__ qv,
                                               const SolverScalars* __restrict__ sc,
                                               double* __restrict__ partials, long stride) {
    if (sc->done) return;
    Cell C;
    double v[2] = {0.0, 0.0};
    if (cell_of_thread<Coef::kWalls>(d, C)) {
        auto Z = [&](int a, int s) -> S { return ld(z, C.nb(a, s)); };
        S bl[3], bh[3], dg;
        cf.template faces<DIM>(C, bl, bh);
        const unsigned c = C.id;
        const S zcen = ld(z, c);
        const S az = apply_at<S, DIM>(bl, bh, Z, zcen, ih2, dg);
        const S rc = ld(r, c);
        const S out = zcen + omega * (rc - az) * recip(dg);
        st(zt, c, out);
        if (DOT) {
            v[0] = (double)rc * (double)out;
            v[1] = (double)ld(qv, c) * (double)out;
        }
    }
    if (DOT) block_partials_2r(v, partials, stride);
}

// 1 / d of a stored-coefficient level (d = ih2 times the sum of the face
// coefficients, summed as in k_jac_first), once per solve
template <typename S, int DIM>
__global__ __launch_bounds__(BLOCK) void k_dinv(Dims d, S ih2, CoefStored<S> cf, S* __restrict__ dinv) {
    Cell C;
    if (!cell_of_thread<false>(d, C)) return;
    S bl[3], bh[3], dg = S(0);
    cf.template faces<DIM>(C, bl, bh);
#pragma unroll
    for (int a = 0; a < DIM; ++a) dg += bl[a] + bh[a];
    st(dinv, C.id, recip(dg * ih2));
}

// The first two pre-smoothing sweeps of a stored-coefficient level in one
// pass: the first sweep from zero is pointwise, z1 = w1 r / d, so the second,
// zt = z1 + w2 (r - A z1) / d, forms z1 at its stencil points from r and the
// stored 1 / d.  The same arithmetic as k_jac_first then k_jac (bitwise: z1
// is rounded as when it is stored, its products are not contracted into the
// stencil's differences), and z1 never goes to memory.
template <typename S, int DIM>
__global__ __launch_bounds__(BLOCK) void k_jac2_first(Dims d, S ih2, S w1, S w2, CoefStored<S> cf,
                                                      const S* __restrict__ r, const S* __restrict__ dinv,
                                                      S* __restrict__ zt, const SolverScalars* __restrict__ sc) {
    if (sc->done) return;
    Cell C;
    if (!cell_of_thread<false>(d, C)) return;
    auto z1 = [&](unsigned n) {
#pragma clang fp contract(off)
        return w1 * ld(r, n) * ld(dinv, n);
    };
    S bl[3], bh[3], dg;
    cf.template faces<DIM>(C, bl, bh);
    const unsigned c = C.id;
    const S zc = z1(c);
    auto Z = [&](int a, int s) -> S { return z1(C.nb(a, s)); };
    const S az = apply_at<S, DIM>(bl, bh, Z, zc, ih2, dg);
    st(zt, c, zc + w2 * (ld(r, c) - az) * recip(dg));
}

// Cell-centred multilinear interpolation of a coarse field at fine cell
// (i, j, k): along each axis the fine cell 2I + s takes 3/4 of coarse cell I
// and 1/4 of the coarse neighbour on its own side (I - 1 for s = 0, I + 1 for
// s = 1), periodic; the weights multiply across axes.
template <typename S, int DIM>
__device__ __forceinline__ S prolong_at(const Dims& cd, const S* zc, int i, int j, int k) {
    const int I = i >> 1, J = j >> 1, K = DIM == 3 ? k >> 1 : 0;
    const int I2 = wrapc(I + ((i & 1) ? 1 : -1), cd.nx);
    const int J2 = wrapc(J + ((j & 1) ? 1 : -1), cd.ny);
    const int K2 = DIM == 3 ? wrapc(K + ((k & 1) ? 1 : -1), cd.nz) : 0;
    auto at = [&](int a, int b, int e) { return zc[(e * cd.ny + b) * cd.nx + a]; };
    const S w1 = S(0.75), w2 = S(0.25);
    const S s0 = w1 * (w1 * at(I, J, K) + w2 * at(I2, J, K)) + w2 * (w1 * at(I, J2, K) + w2 * at(I2, J2, K));
    if (DIM == 2) return s0;
    const S s1 = w1 * (w1 * at(I, J, K2) + w2 * at(I2, J, K2)) + w2 * (w1 * at(I, J2, K2) + w2 * at(I2, J2, K2));
    return w1 * s0 + w2 * s1;
}

// z += P zc (the coarse-grid correction, interpolated).  One thread per
// coarse cell writes its 2^DIM children: the 3^DIM coarse values around the
// cell are read once and interpolated axis by axis (x, then y, then z), and
// each fine row pair (2I, 2I + 1) is one 2-element access (coalesced across
// the wave).
template <typename S, int DIM>
__global__ __launch_bounds__(BLOCK) void k_prolong(Dims fd, Dims cd, const S* __restrict__ zc,
                                                   S* __restrict__ z, const SolverScalars* __restrict__ sc) {
#pragma clang fp contract(off)     // the same roundings as k_cup's prolongation
    if (sc->done) return;
    Cell Q;
    if (!cell_of_thread(cd, Q)) return;
    using S2 = typename Vec2<S>::type;
    constexpr int NZ = DIM == 3 ? 3 : 1;
    const S w1 = S(0.75), w2 = S(0.25);
    // x pass: for each coarse row (J + dj, K + dk), the values at the two
    // fine x positions 2I and 2I + 1
    S xl[NZ][3], xh[NZ][3];
#pragma unroll
    for (int dk = 0; dk < NZ; ++dk)
#pragma unroll
        for (int dj = 0; dj < 3; ++dj) {
            unsigned q = Q.id;
            if (DIM == 3 && dk != 1) q += (unsigned)Q.o[2][dk > 1];
            if (dj != 1) q += (unsigned)Q.o[1][dj > 1];
            const int row = (int)q - Q.i;       // first cell of that coarse row
            const S cm = ld(zc, (unsigned)(row + (Q.i == 0 ? cd.nx - 1 : Q.i - 1)));
            const S c0 = ld(zc, q);
            const S cp = ld(zc, (unsigned)(row + (Q.i == cd.nx - 1 ? 0 : Q.i + 1)));
            xl[dk][dj] = w1 * c0 + w2 * cm;
            xh[dk][dj] = w1 * c0 + w2 * cp;
        }
    const int fi = 2 * Q.i;
#pragma unroll
    for (int sz = 0; sz < (DIM == 3 ? 2 : 1); ++sz)
#pragma unroll
        for (int sy = 0; sy < 2; ++sy) {
            // y pass (rows J and J -+ 1), then z pass (planes K and K -+ 1)
            auto ypass = [&](int dk, S& lo, S& hi) {
                const int dj = sy ? 2 : 0;
                lo = w1 * xl[dk][1] + w2 * xl[dk][dj];
                hi = w1 * xh[dk][1] + w2 * xh[dk][dj];
            };
            S lo, hi;
            if (DIM == 3) {
                S l0, h0, l1, h1;
                ypass(1, l0, h0);
                ypass(sz ? 2 : 0, l1, h1);
                lo = w1 * l0 + w2 * l1;
                hi = w1 * h0 + w2 * h1;
            } else {
                ypass(0, lo, hi);
            }
            const int fj = 2 * Q.j + sy, fk = DIM == 3 ? 2 * Q.k + sz : 0;
            const unsigned f = (unsigned)((fk * fd.ny + fj) * fd.nx + fi);
            S2* p = reinterpret_cast<S2*>(reinterpret_cast<char*>(z) + (unsigned)(f * (unsigned)sizeof(S)));
            S2 v = *p;
            v.x += lo;
            v.y += hi;
            *p = v;
        }
}

// coarse rhs = mean over the 2^DIM children of (r - A z).  One thread per
// fine cell (coalesced); block 64 x 2 x 2 (3D) or 64 x 4 (2D); x pairs summed
// with a lane shuffle, y/z pairs through LDS.
template <typename Coef, typename S, int DIM>
__global__ __launch_bounds__(BLOCK) void k_restrict(Dims fd, Dims cd, S ih2, S rw, Coef cf,
                                                    const S* __restrict__ r,
                                                    const S* __restrict__ z,
                                                    S* __restrict__ rc,
                                                    const SolverScalars* __restrict__ sc) {
    if (sc->done) return;
    constexpr int TY = DIM == 3 ? 2 : 4, TZ = DIM == 3 ? 2 : 1;
    __shared__ S sh[TZ][TY][BX];
    const int tx = threadIdx.x, ty = threadIdx.y, tz = threadIdx.z;
    int bx, by, bz;
    const bool tile = block_tile(fd.xcd, (fd.nx + BX - 1) / BX, (fd.ny + TY - 1) / TY, (fd.nz + TZ - 1) / TZ, bx,
                                 by, bz);
    const int fi = bx * BX + tx, fj = by * TY + ty, fk = bz * TZ + tz;
    const bool in = tile && fi < fd.nx && fj < fd.ny && fk < fd.nz;
    const Cell C = Coef::kWalls ? make_cell_w(fd, in ? fi : 0, in ? fj : 0, in ? fk : 0)
                                : make_cell(fd, in ? fi : 0, in ? fj : 0, in ? fk : 0);
    S res = S(0);
    if (in) {
        S bl[3], bh[3], dg;
        cf.template faces<DIM>(C, bl, bh);
        auto Z = [&](int a, int s) { return ld(z, C.nb(a, s)); };
        const unsigned c = C.id;
        res = ld(r, c) - apply_at<S, DIM>(bl, bh, Z, ld(z, c), ih2, dg);
    }
    res += __shfl_xor(res, 1, 64);
    sh[tz][ty][tx] = res;
    __syncthreads();
    if (in && (tx & 1) == 0 && (ty & 1) == 0 && tz == 0) {
        S s = sh[0][ty][tx] + sh[0][ty + 1][tx];
        if constexpr (DIM == 3) s += sh[1][ty][tx] + sh[1][ty + 1][tx];
        const long cc = ((long)(C.k >> 1) * cd.ny + (C.j >> 1)) * cd.nx + (C.i >> 1);
        const long cmax = (long)cd.nx * cd.ny * cd.nz - 1;
        rc[cc < cmax ? cc : cmax] = s * rw;
    }
}

// coarsest grid: `sweeps` damped Jacobi sweeps from zero in one workgroup;
// result in z
template <typename S, int DIM>
__global__ __launch_bounds__(1024) void k_coarse(Dims d, S ih2, S omega, int sweeps,
                                                 CoefStored<S> cf, const S* __restrict__ r, S* z,
                                                 S* zt, const SolverScalars* __restrict__ sc) {
    if (sc->done) return;
    const long N = (long)d.nx * d.ny * d.nz;
    for (long q = threadIdx.x; q < N; q += blockDim.x) z[q] = S(0);
    __syncthreads();
    S* src = z;
    S* dst = zt;
    for (int s = 0; s < sweeps; ++s) {
        for (long q = threadIdx.x; q < N; q += blockDim.x) {
            const Cell C = make_cell(d, (int)(q % d.nx), (int)((q / d.nx) % d.ny),
                                     (int)(q / ((long)d.nx * d.ny)));
            S bl[3], bh[3], dg;
            cf.template faces<DIM>(C, bl, bh);
            const S* xs = src;
            auto X = [&](int a, int t) { return xs[C.nb(a, t)]; };
            const S az = apply_at<S, DIM>(bl, bh, X, src[q], ih2, dg);
            dst[q] = src[q] + omega * (r[q] - az) * recip(dg);
        }
        __syncthreads();
        S* t = src;
        src = dst;
        dst = t;
    }
    if (src != z) {
        for (long q = threadIdx.x; q < N; q += blockDim.x) z[q] = src[q];
    }
}

// ---------------------------------------------------------------- LDS tail
// The last levels of the V-cycle (every level from `first` down, at most
// TAIL_MAX_LEVELS, all of them together small enough for LDS) run in one
// 1024-thread workgroup: r, z and zt of every tail level live in LDS, the
// face coefficients stay in global memory (L2).  The operations and their
// order are those of the multi-kernel levels above (two damped Jacobi sweeps
// before and after, averaging restriction, multilinear prolongation, fixed
// Jacobi sweeps on the coarsest grid), so the preconditioner remains the same
// linear operator; only launches are saved.
constexpr int TAIL_MAX_LEVELS = 8;
constexpr size_t TAIL_LDS_BYTES = 64 * 1024;

struct TailDesc {
    int nlev;
    int n[TAIL_MAX_LEVELS][3];
    int off[TAIL_MAX_LEVELS];          // element offset of level l's r; z, zt follow
    double ih2[TAIL_MAX_LEVELS];
    const void* beta[TAIL_MAX_LEVELS][3];
    int lg[TAIL_MAX_LEVELS][2];         // log2 nx, log2 (nx ny) when both are powers of two, else -1
    double rw;                          // restriction weight
};

template <typename S, int DIM>
__global__ __launch_bounds__(1024) void k_tail(TailDesc D, S w1, S w2, S omega_c, int sweeps,
                                               const S* __restrict__ rin, S* __restrict__ zout,
                                               const SolverScalars* __restrict__ sc) {
    if (sc->done) return;
    extern __shared__ __align__(16) unsigned char tail_smem[];
    S* L = reinterpret_cast<S*>(tail_smem);
    const int t = threadIdx.x, T = blockDim.x;
    auto dims = [&](int l) { return Dims{D.n[l][0], D.n[l][1], D.n[l][2], 0, 0}; };
    auto ncell = [&](int l) { return D.n[l][0] * D.n[l][1] * D.n[l][2]; };
    // a level's sizes and index shifts, read from the descriptor once per pass
    // (indexed by the level, the descriptor lives in kernel-argument memory)
    struct Lev {
        Dims d;
        int lx, lxy;
    };
    auto lev = [&](int l) { return Lev{dims(l), D.lg[l][0], D.lg[l][1]}; };
    // (i, j, k) of cell q: shifts and masks when nx and ny are powers of two
    // (lx >= 0, the usual case), else divisions
    auto ijk = [&](const Lev& V, int q, int& i, int& j, int& k) {
        if (V.lx >= 0) {
            i = q & (V.d.nx - 1);
            j = (q >> V.lx) & (V.d.ny - 1);
            k = q >> V.lxy;
        } else {
            i = q % V.d.nx;
            j = (q / V.d.nx) % V.d.ny;
            k = q / (V.d.nx * V.d.ny);
        }
    };
    auto cell = [&](const Lev& V, int q) {
        int i, j, k;
        ijk(V, q, i, j, k);
        return make_cell(V.d, i, j, k);
    };
    auto coef = [&](int l) {
        return CoefStored<S>{static_cast<const S*>(D.beta[l][0]), static_cast<const S*>(D.beta[l][1]),
                             static_cast<const S*>(D.beta[l][2])};
    };
    // one damped Jacobi sweep out = X + w (r - A X) / d, X(a, s) from get
    // (1 / d by the reciprocal of the separate sweep kernels)
    auto sweep = [&](int l, S w, auto get, S* out) {
        const Lev V = lev(l);
        const int N = ncell(l);
        const S* r = L + D.off[l];
        const S ih2 = S(D.ih2[l]);
        const CoefStored<S> cf = coef(l);
        for (int q = t; q < N; q += T) {
            const Cell C = cell(V, q);
            S bl[3], bh[3], dg;
            cf.template faces<DIM>(C, bl, bh);
            auto X = [&](int a, int s) { return get(C, a, s); };
            const S xc = get(C, 0, 0);
            const S az = apply_at<S, DIM>(bl, bh, X, xc, ih2, dg);
            out[q] = xc + w * (r[q] - az) * recip(dg);
        }
        __syncthreads();
    };
    {
        const int N0 = ncell(0);
        for (int q = t; q < N0; q += T) L[D.off[0] + q] = rin[q];
        __syncthreads();
    }
    // ---- down
    for (int l = 0; l + 1 < D.nlev; ++l) {
        const int N = ncell(l);
        S* r = L + D.off[l];
        S* z = r + N;
        S* zt = z + N;
        const S ih2 = S(D.ih2[l]);
        const CoefStored<S> cf = coef(l);
        const Lev V = lev(l);
        for (int q = t; q < N; q += T) {            // z = omega r / d
            const Cell C = cell(V, q);
            S bl[3], bh[3], dg = S(0);
            cf.template faces<DIM>(C, bl, bh);
            for (int a = 0; a < DIM; ++a) dg += bl[a] + bh[a];
            z[q] = w1 * r[q] * recip(dg * ih2);
        }
        __syncthreads();
        sweep(l, w2, [&](const Cell& C, int a, int s) { return z[s == 0 ? C.id : C.nb(a, s)]; }, zt);
        // restriction of r - A zt into the next level's r
        const int Nc = ncell(l + 1);
        S* rc = L + D.off[l + 1];
        const Dims df = V.d;
        const Lev VC = lev(l + 1);
        for (int Q = t; Q < Nc; Q += T) {
            int I, J, K;
            ijk(VC, Q, I, J, K);
            S s = S(0);
            for (int dk = 0; dk < (DIM == 3 ? 2 : 1); ++dk)
                for (int dj = 0; dj < 2; ++dj)
                    for (int di = 0; di < 2; ++di) {
                        const Cell C = make_cell(df, 2 * I + di, 2 * J + dj, DIM == 3 ? 2 * K + dk : 0);
                        S bl[3], bh[3], dg;
                        cf.template faces<DIM>(C, bl, bh);
                        auto X = [&](int a, int s2) { return zt[C.nb(a, s2)]; };
                        s += r[C.id] - apply_at<S, DIM>(bl, bh, X, zt[C.id], ih2, dg);
                    }
            rc[Q] = s * S(D.rw);
        }
        __syncthreads();
    }
    // ---- coarsest: fixed Jacobi sweeps from zero, result in zt
    {
        const int l = D.nlev - 1;
        const int N = ncell(l);
        S* r = L + D.off[l];
        if (N <= 64) {
            // one cell per lane of the first wave: the sweeps read the
            // neighbours' values by lane shuffles and need no block barrier
            // (the same arithmetic as the block-wide sweeps below)
            if (t < 64) {
                const int q = t < N ? t : 0;
                const Cell C = cell(lev(l), q);
                const CoefStored<S> cf = coef(l);
                const S ih2 = S(D.ih2[l]);
                S bl[3], bh[3];
                cf.template faces<DIM>(C, bl, bh);
                int lm[3] = {0, 0, 0}, lp[3] = {0, 0, 0};
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    lm[a] = (int)C.nb(a, -1);
                    lp[a] = (int)C.nb(a, 1);
                }
                const S rq = r[q];
                S x = S(0);
                for (int s = 0; s < sweeps; ++s) {
                    S xm[3], xp[3];
#pragma unroll
                    for (int a = 0; a < DIM; ++a) {
                        xm[a] = __shfl(x, lm[a], 64);
                        xp[a] = __shfl(x, lp[a], 64);
                    }
                    auto X = [&](int a, int s2) { return s2 < 0 ? xm[a] : xp[a]; };
                    S dg;
                    const S az = apply_at<S, DIM>(bl, bh, X, x, ih2, dg);
                    x = x + omega_c * (rq - az) * recip(dg);
                }
                if (t < N) r[2 * N + t] = x;
            }
            __syncthreads();
        } else {
            S* src = r + 2 * N;   // zt
            S* dst = r + N;       // z
            for (int q = t; q < N; q += T) src[q] = S(0);
            __syncthreads();
            for (int s = 0; s < sweeps; ++s) {
                const S* in = src;
                sweep(l, omega_c, [&](const Cell& C, int a, int s2) { return in[s2 == 0 ? C.id : C.nb(a, s2)]; }, dst);
                S* tmp = src;
                src = dst;
                dst = tmp;
            }
            if (src != r + 2 * N) {
                for (int q = t; q < N; q += T) r[2 * N + q] = src[q];
                __syncthreads();
            }
        }
    }
    // ---- up
    for (int l = D.nlev - 2; l >= 0; --l) {
        const int N = ncell(l);
        S* r = L + D.off[l];
        S* z = r + N;
        S* zt = z + N;
        const Dims dc = dims(l + 1);
        const S* zc = L + D.off[l + 1] + 2 * ncell(l + 1);
        const Lev V = lev(l);
        // zt += P zc, then two sweeps zt -> z -> zt
        for (int q = t; q < N; q += T) {
            int i, j, k;
            ijk(V, q, i, j, k);
            zt[q] += prolong_at<S, DIM>(dc, zc, i, j, k);
        }
        __syncthreads();
        sweep(l, w2, [&](const Cell& C, int a, int s) { return zt[s == 0 ? C.id : C.nb(a, s)]; }, z);
        sweep(l, w1, [&](const Cell& C, int a, int s) { return z[s == 0 ? C.id : C.nb(a, s)]; }, zt);
    }
    {
        const int N0 = ncell(0);
        const S* zt0 = L + D.off[0] + 2 * N0;
        for (int q = t; q < N0; q += T) zout[q] = zt0[q];
    }
}

// ---------------------------------------------------------------- fused coarse levels (3D)
// On a stored-coefficient level of a 3D V-cycle, one launch per direction
// replaces the six separate ones: `k_cdown` does the first sweep from zero,
// the second sweep and the restriction of the residual; `k_cup` the
// prolongation and the two post-smoothing sweeps.  Each block owns a CT^3
// tile and recomputes on a halo what its stencils need (the first sweep on
// the tile plus two cells, the second on the tile plus one), from LDS copies
// of r and of the face coefficients, so no intermediate sweep goes to memory.
// The per-cell arithmetic is that of k_jac_first, k_jac, k_restrict and
// k_prolong, in the same order (the prolongation with contraction off in
// both), so the results are bitwise those of the separate kernels.  Only
// small levels take this path (at 256^3: 64^3 and 32^3), where the separate
// kernels are bound by launch latency, not bandwidth.
// The tile edge TE is 8, or 4 on a level whose 8^3 tiles would not give
// every compute unit a block (at 256^3: 32^3, 64 tiles of 8^3).
template <int TE>
struct CTile {
    static_assert(TE % 2 == 0, "restriction pairs stay in the tile");
    static constexpr int CT = TE;              // tile edge
    static constexpr int CH2 = CT + 4;         // tile plus two cells on each side
    static constexpr int CH1 = CT + 2;         // tile plus one
    static constexpr int CB = CT + 5;          // coefficient region: the faces of the CH2 cells
    static constexpr int CC = CT / 2 + 4;      // coarse region of k_cup: the coarse cells the CH2 cells interpolate from
    static constexpr int CNB = CB * CB * CB, CN2 = CH2 * CH2 * CH2, CN1 = CH1 * CH1 * CH1, CNT = CT * CT * CT;
    static constexpr int CNC = CC * CC * CC;
};
#define TPF_CTILE(TE)                                                                            \
    constexpr int CT = CTile<TE>::CT, CH2 = CTile<TE>::CH2, CH1 = CTile<TE>::CH1, CB = CTile<TE>::CB; \
    constexpr int CC = CTile<TE>::CC, CNB = CTile<TE>::CNB, CN2 = CTile<TE>::CN2, CN1 = CTile<TE>::CN1; \
    constexpr int CNT = CTile<TE>::CNT, CNC = CTile<TE>::CNC;                                     \
    (void)CT; (void)CH2; (void)CH1; (void)CB; (void)CC; (void)CNB; (void)CN2; (void)CN1; (void)CNT; (void)CNC
// Levels up to this size take the fused kernels.  Measured per V-cycle at
// 256^3: 64^3 18 us fused against 28 us in six launches, 32^3 15 against
// 28 us; at 128^3 (4096 tiles, each recomputing a halo of 3.4 times its
// cells) 88 us fused against 53 us for the separate, bandwidth-bound kernels.
constexpr long CFUSE_MAX_CELLS = 1L << 19;

template <int E>
__device__ __forceinline__ void cdec(int e, int& x, int& y, int& z) {
    z = e / (E * E);
    const int q = e - z * (E * E);
    y = q / E;
    x = q - y * E;
}

// global element offsets of the local positions along each axis: position p
// of axis a is global index origin[a] + p (periodic), times the axis stride
template <int NP>
__device__ __forceinline__ void coarse_offsets(const Dims& d, int o0, int o1, int o2, int (*g)[NP]) {
    const int t = threadIdx.x;
    if (t < 3 * NP) {
        const int a = t / NP, p = t - a * NP;
        const int n = a == 0 ? d.nx : a == 1 ? d.ny : d.nz;
        int v = ((a == 0 ? o0 : a == 1 ? o1 : o2) + p) % n;
        v += v < 0 ? n : 0;
        g[a][p] = a == 0 ? v : a == 1 ? v * d.nx : v * d.nx * d.ny;
    }
}

// face coefficients of the cell at position b of the coefficient region
template <int TE, typename S>
__device__ __forceinline__ void cfaces(const S* sb, int b, S* bl, S* bh) {
    TPF_CTILE(TE);
    bl[0] = sb[b];
    bh[0] = sb[b + 1];
    bl[1] = sb[CNB + b];
    bh[1] = sb[CNB + b + CB];
    bl[2] = sb[2 * CNB + b];
    bh[2] = sb[2 * CNB + b + CB * CB];
}

template <typename S, int TE>
__global__ __launch_bounds__(BLOCK) void k_cdown(Dims d, Dims cd, S ih2, S w1, S w2, S rw, CoefStored<S> cf,
                                                 const S* __restrict__ r, S* __restrict__ zt,
                                                 S* __restrict__ rc, const SolverScalars* __restrict__ sc) {
    TPF_CTILE(TE);
    if (sc->done) return;
    // sb: the three coefficient arrays on the CB^3 region, then r on the CH2^3
    // region (both with origin tile - 2); sz: z on CH2^3, later the residual
    // on the tile; szt: zt on CH1^3 (origin tile - 1)
    __shared__ S sb[3 * CNB + CN2];
    __shared__ S sz[CN2];
    __shared__ S szt[CN1];
    __shared__ int gof[3][CB];
    int bx, by, bz;
    if (!block_tile(d.xcd, (d.nx + CT - 1) / CT, (d.ny + CT - 1) / CT, (d.nz + CT - 1) / CT, bx, by, bz)) return;
    const int t = threadIdx.x;
    const int i0 = bx * CT, j0 = by * CT, k0 = bz * CT;
    coarse_offsets<CB>(d, i0 - 2, j0 - 2, k0 - 2, gof);
    __syncthreads();
    {
        // every load of the block in flight before the first store
        constexpr int NE = 3 * CNB + CN2, U = (NE + BLOCK - 1) / BLOCK;
        S v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = t + u * BLOCK;
            int x, y, z, src;
            if (e < 3 * CNB) {
                src = e / CNB;
                cdec<CB>(e - src * CNB, x, y, z);
            } else {
                src = 3;
                cdec<CH2>(min(e - 3 * CNB, CN2 - 1), x, y, z);
            }
            const unsigned g = (unsigned)(gof[2][z] + gof[1][y] + gof[0][x]);
            const S* p = src == 0 ? cf.b0 : src == 1 ? cf.b1 : src == 2 ? cf.b2 : r;
            v[u] = e < NE ? ld(p, g) : S(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = t + u * BLOCK;
            if (e < NE) sb[e] = v[u];
        }
    }
    __syncthreads();
    const S* sr = sb + 3 * CNB;
    // first sweep from zero on the tile plus two: z = w1 r / d
    for (int e = t; e < CN2; e += BLOCK) {
        int x, y, z;
        cdec<CH2>(e, x, y, z);
        S bl[3], bh[3], dg = S(0);
        cfaces<TE>(sb, (z * CB + y) * CB + x, bl, bh);
#pragma unroll
        for (int a = 0; a < 3; ++a) dg += bl[a] + bh[a];
        sz[e] = w1 * sr[e] * recip(dg * ih2);
    }
    __syncthreads();
    // second sweep on the tile plus one: zt = z + w2 (r - A z) / d
    for (int e = t; e < CN1; e += BLOCK) {
        int x, y, z;
        cdec<CH1>(e, x, y, z);
        const int p = ((z + 1) * CH2 + y + 1) * CH2 + x + 1;
        S bl[3], bh[3], dg;
        cfaces<TE>(sb, ((z + 1) * CB + y + 1) * CB + x + 1, bl, bh);
        auto Z = [&](int a, int s) {
            const int o = a == 0 ? 1 : a == 1 ? CH2 : CH2 * CH2;
            return sz[s > 0 ? p + o : p - o];
        };
        const S zcen = sz[p];
        const S az = apply_at<S, 3>(bl, bh, Z, zcen, ih2, dg);
        const S rv = sr[p];
        szt[e] = zcen + w2 * (rv - az) * recip(dg);
    }
    __syncthreads();
    // residual on the tile (into sz) and zt of the tile to memory
    for (int e = t; e < CNT; e += BLOCK) {
        int x, y, z;
        cdec<CT>(e, x, y, z);
        const int q = ((z + 1) * CH1 + y + 1) * CH1 + x + 1;
        S bl[3], bh[3], dg;
        cfaces<TE>(sb, ((z + 2) * CB + y + 2) * CB + x + 2, bl, bh);
        auto X = [&](int a, int s) {
            const int o = a == 0 ? 1 : a == 1 ? CH1 : CH1 * CH1;
            return szt[s > 0 ? q + o : q - o];
        };
        const S ztc = szt[q];
        sz[e] = sr[((z + 2) * CH2 + y + 2) * CH2 + x + 2] - apply_at<S, 3>(bl, bh, X, ztc, ih2, dg);
        const int gi = i0 + x, gj = j0 + y, gk = k0 + z;
        if (gi < d.nx && gj < d.ny && gk < d.nz) st(zt, (unsigned)((gk * d.ny + gj) * d.nx + gi), ztc);
    }
    __syncthreads();
    // restriction: the mean of the 8 children, summed as k_restrict does
    // (x pairs, then the y pair of each z plane, then the two planes)
    constexpr int H = CT / 2;
    if (t < H * H * H) {
        int X, Y, Z;
        cdec<H>(t, X, Y, Z);
        auto pr = [&](int dy, int dz) {
            const int b = ((2 * Z + dz) * CT + 2 * Y + dy) * CT + 2 * X;
            return sz[b] + sz[b + 1];
        };
        S s = pr(0, 0) + pr(1, 0);
        s += pr(0, 1) + pr(1, 1);
        const int I = i0 / 2 + X, J = j0 / 2 + Y, K = k0 / 2 + Z;
        if (I < cd.nx && J < cd.ny && K < cd.nz) st(rc, (unsigned)((K * cd.ny + J) * cd.nx + I), s * rw);
    }
}

// the prolongation step of k_prolong for fine position (x, y, z) of the CH2
// region from the CC^3 coarse region; contraction off, as there
template <int TE, typename S>
__device__ __forceinline__ S cprolong(const S* szc, int x, int y, int z) {
#pragma clang fp contract(off)
    TPF_CTILE(TE);
    const int I = 1 + (x >> 1), J = 1 + (y >> 1), K = 1 + (z >> 1);
    const int I2 = I + ((x & 1) ? 1 : -1), J2 = J + ((y & 1) ? 1 : -1), K2 = K + ((z & 1) ? 1 : -1);
    auto at = [&](int a, int b, int e) { return szc[(e * CC + b) * CC + a]; };
    const S w1 = S(0.75), w2 = S(0.25);
    auto xrow = [&](int b, int e) { return w1 * at(I, b, e) + w2 * at(I2, b, e); };
    auto yz = [&](int e) { return w1 * xrow(J, e) + w2 * xrow(J2, e); };
    return w1 * yz(K) + w2 * yz(K2);
}

template <typename S, int TE>
__global__ __launch_bounds__(BLOCK) void k_cup(Dims d, Dims cd, S ih2, S w1, S w2, CoefStored<S> cf,
                                               const S* __restrict__ r, const S* __restrict__ zc,
                                               const S* __restrict__ zt, S* __restrict__ zout,
                                               const SolverScalars* __restrict__ sc) {
    TPF_CTILE(TE);
    if (sc->done) return;
    // sb: coefficients on CB^3, then zt on CH2^3 (origin tile - 2), r on CH1^3
    // (origin tile - 1) and the coarse correction on CC^3 (origin tile/2 - 2)
    constexpr int OZT = 3 * CNB, OR = OZT + CN2, OC = OR + CN1, NE = OC + CNC;
    __shared__ S sb[NE];
    __shared__ S sz[CN1];
    __shared__ int gof[3][CB];
    __shared__ int cof[3][CC];
    int bx, by, bz;
    if (!block_tile(d.xcd, (d.nx + CT - 1) / CT, (d.ny + CT - 1) / CT, (d.nz + CT - 1) / CT, bx, by, bz)) return;
    const int t = threadIdx.x;
    const int i0 = bx * CT, j0 = by * CT, k0 = bz * CT;
    coarse_offsets<CB>(d, i0 - 2, j0 - 2, k0 - 2, gof);
    coarse_offsets<CC>(cd, i0 / 2 - 2, j0 / 2 - 2, k0 / 2 - 2, cof);
    __syncthreads();
    {
        constexpr int U = (NE + BLOCK - 1) / BLOCK;
        S v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = t + u * BLOCK;
            int x, y, z, src;
            unsigned g;
            if (e < OZT) {
                src = e / CNB;
                cdec<CB>(e - src * CNB, x, y, z);
                g = (unsigned)(gof[2][z] + gof[1][y] + gof[0][x]);
            } else if (e < OR) {
                src = 3;
                cdec<CH2>(e - OZT, x, y, z);
                g = (unsigned)(gof[2][z] + gof[1][y] + gof[0][x]);
            } else if (e < OC) {
                src = 4;
                cdec<CH1>(e - OR, x, y, z);
                g = (unsigned)(gof[2][z + 1] + gof[1][y + 1] + gof[0][x + 1]);
            } else {
                src = 5;
                cdec<CC>(min(e - OC, CNC - 1), x, y, z);
                g = (unsigned)(cof[2][z] + cof[1][y] + cof[0][x]);
            }
            const S* p = src == 0 ? cf.b0 : src == 1 ? cf.b1 : src == 2 ? cf.b2 : src == 3 ? zt : src == 4 ? r : zc;
            v[u] = e < NE ? ld(p, g) : S(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = t + u * BLOCK;
            if (e < NE) sb[e] = v[u];
        }
    }
    __syncthreads();
    S* szt = sb + OZT;
    const S* sr = sb + OR;
    const S* szc = sb + OC;
    // zt += P zc on the tile plus two
    for (int e = t; e < CN2; e += BLOCK) {
        int x, y, z;
        cdec<CH2>(e, x, y, z);
        szt[e] = szt[e] + cprolong<TE>(szc, x, y, z);
    }
    __syncthreads();
    // first post-sweep on the tile plus one: z = zt + w2 (r - A zt) / d
    for (int e = t; e < CN1; e += BLOCK) {
        int x, y, z;
        cdec<CH1>(e, x, y, z);
        const int p = ((z + 1) * CH2 + y + 1) * CH2 + x + 1;
        S bl[3], bh[3], dg;
        cfaces<TE>(sb, ((z + 1) * CB + y + 1) * CB + x + 1, bl, bh);
        auto X = [&](int a, int s) {
            const int o = a == 0 ? 1 : a == 1 ? CH2 : CH2 * CH2;
            return szt[s > 0 ? p + o : p - o];
        };
        const S xc = szt[p];
        const S az = apply_at<S, 3>(bl, bh, X, xc, ih2, dg);
        const S rv = sr[e];
        sz[e] = xc + w2 * (rv - az) * recip(dg);
    }
    __syncthreads();
    // second post-sweep on the tile: out = z + w1 (r - A z) / d
    for (int e = t; e < CNT; e += BLOCK) {
        int x, y, z;
        cdec<CT>(e, x, y, z);
        const int q = ((z + 1) * CH1 + y + 1) * CH1 + x + 1;
        S bl[3], bh[3], dg;
        cfaces<TE>(sb, ((z + 2) * CB + y + 2) * CB + x + 2, bl, bh);
        auto X = [&](int a, int s) {
            const int o = a == 0 ? 1 : a == 1 ? CH1 : CH1 * CH1;
            return sz[s > 0 ? q + o : q - o];
        };
        const S xc = sz[q];
        const S az = apply_at<S, 3>(bl, bh, X, xc, ih2, dg);
        const S rv = sr[q];
        const int gi = i0 + x, gj = j0 + y, gk = k0 + z;
        if (gi < d.nx && gj < d.ny && gk < d.nz)
            st(zout, (unsigned)((gk * d.ny + gj) * d.nx + gi), xc + w1 * (rv - az) * recip(dg));
    }
}

// ---------------------------------------------------------------- CG apply
// p = z + beta p_old (first: p = z) at the stencil points, q = A p, <p, q>
template <typename Coef, typename S, int DIM>
__global__ __launch_bounds__(BLOCK) void k_apply(Dims d, S ih2, Coef cf, int first,
                                                 const S* __restrict__ z,
                                                 const S* __restrict__ pold,
                                                 S* __restrict__ pnew, S* __restrict__ q,
                                                 const SolverScalars* __restrict__ sc,
                                                 double* __restrict__ partials) {
    if (sc->done) return;
    Cell C;
    double v[1] = {0.0};
    if (cell_of_thread<Coef::kWalls>(d, C)) {
        const S beta = first ? S(0) : S(sc->beta);
        auto Pn = [&](unsigned t) -> S { return first ? ld(z, t) : ld(z, t) + beta * ld(pold, t); };
        auto Pa = [&](int a, int s) { return Pn(C.nb(a, s)); };
        S bl[3], bh[3], dg;
        cf.template faces<DIM>(C, bl, bh);
        const unsigned c = C.id;
        const S pc = Pn(c);
        const S aq = apply_at<S, DIM>(bl, bh, Pa, pc, ih2, dg);
        st(pnew, c, pc);
        st(q, c, aq);
        v[0] = (double)pc * (double)aq;
    }
    block_partials<1>(v, partials);
}

// ---------------------------------------------------------------- small vector kernels
constexpr int VBLOCKS = 1024;   // grid-stride vector kernels

// x += e (the FP32 correction of a defect-correction pass)
__global__ __launch_bounds__(BLOCK) void k_correct(long N, double* __restrict__ x,
                                                   const float* __restrict__ e) {
    for (long c = (long)blockIdx.x * BLOCK + threadIdx.x; c < N; c += (long)gridDim.x * BLOCK)
        x[c] += (double)e[c];
}

__global__ __launch_bounds__(BLOCK) void k_sum(long N, const double* __restrict__ x,
                                               double* __restrict__ partials) {
    double v[1] = {0.0};
    for (long c = (long)blockIdx.x * BLOCK + threadIdx.x; c < N; c += (long)gridDim.x * BLOCK)
        v[0] += x[c];
    block_partials<1>(v, partials);
}

__global__ __launch_bounds__(BLOCK) void k_sub_mean(long N, double* __restrict__ x,
                                                    const SolverScalars* __restrict__ sc) {
    const double m = sc->sum / (double)N;
    for (long c = (long)blockIdx.x * BLOCK + threadIdx.x; c < N; c += (long)gridDim.x * BLOCK)
        x[c] -= m;
}

// ---------------------------------------------------------------- finalize
// One 1024-thread block sums region 0 (nb0 partials) and region 1 (nb1
// partials at partials + stride) in a fixed order and applies op.
constexpr int FIN_THREADS = 1024;

__global__ __launch_bounds__(FIN_THREADS) void k_finalize(int nb0, int nb1, int nb2, long stride, int op,
                                                          double arg, long N,
                                                          const double* __restrict__ partials,
                                                          SolverScalars* sc) {
    const bool skip = (op == FIN_ALPHA || op == FIN_BETA || op == FIN_RZ0) && sc->done;
    if (skip) return;
    __shared__ double red[3][FIN_THREADS / 64];
    const int t = threadIdx.x;
    double v[3];
    for (int q = 0; q < 3; ++q) {
        const int nb = q == 0 ? nb0 : (q == 1 ? nb1 : nb2);
        const double* p = partials + q * stride;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int b = t;
        for (; b + 3 * FIN_THREADS < nb; b += 4 * FIN_THREADS) {
            a0 += p[b];
            a1 += p[b + FIN_THREADS];
            a2 += p[b + 2 * FIN_THREADS];
            a3 += p[b + 3 * FIN_THREADS];
        }
        for (; b < nb; b += FIN_THREADS) a0 += p[b];
        v[q] = (a0 + a1) + (a2 + a3);
    }
    for (int q = 0; q < 3; ++q)
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_down(v[q], o, 64);
    if ((t & 63) == 0)
        for (int q = 0; q < 3; ++q) red[q][t >> 6] = v[q];
    __syncthreads();
    if (t != 0) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int w = 0; w < FIN_THREADS / 64; ++w) {
        s0 += red[0][w];
        s1 += red[1][w];
        s2 += red[2][w];
    }
    switch (op) {
    case FIN_MEAN:    // region 0: sum b
        sc->mean = s0 / (double)N;
        break;
    case FIN_INIT:    // region 0: |f|^2, region 1: |r|^2, region 2: | |A||x| |^2
        sc->ff = s0;
        sc->rr = s1;
        sc->tol2 = arg;
        sc->iters = 0;
        sc->floor2 = (RESID_FLOOR_ULPS * 0x1p-53) * (RESID_FLOOR_ULPS * 0x1p-53) * s2;
        sc->done = (s0 == 0.0 || s1 <= arg * s0 || (arg > 0.0 && s1 <= sc->floor2)) ? 1 : 0;
        break;
    case FIN_RZ0:     // region 1: <r, z>
        sc->rz = s1;
        if (!(s1 > 0.0)) sc->done = 1;
        break;
    case FIN_ALPHA:   // region 0: <p, A p>
        sc->pq = s0;
        sc->alpha = (s0 > 0.0) ? sc->rz / s0 : 0.0;
        if (!(s0 > 0.0)) sc->done = 1;
        break;
    case FIN_BETA:    // region 0: |r|^2, region 1: <r, z>, region 2: <A p, z>
        // flexible CG: the new direction z + beta p is made A-orthogonal to
        // p (the preconditioner need not be symmetric)
        sc->rr = s0;
        sc->beta = (sc->pq > 0.0) ? -s2 / sc->pq : 0.0;
        sc->rz = s1;
        sc->iters += 1;
        if (s0 <= sc->tol2 * sc->ff || !(s1 > 0.0)) sc->done = 1;
        break;
    case FIN_SUM:     // region 0: sum x
        sc->sum = s0;
        break;
    default:
        break;
    }
}

// start an inner solve for the current residual: ff = rr, new tolerance
__global__ void k_inner_setup(SolverScalars* sc, double tol2) {
    if (threadIdx.x != 0) return;
    sc->ff = sc->rr;
    sc->tol2 = tol2;
    sc->done = sc->rr > 0.0 ? 0 : 1;
}

// The first inner solve's set-up without a host round trip: the inner
// tolerance from the outer residual just finalized, by the rule of the mixed
// solve (0.9 of the reduction the outer tolerance needs, INNER_MARGIN, clamped to [rin, 0.1];
// 0 in the fixed-iteration mode).  An outer residual that already meets the
// tolerance, or is not finite, leaves the inner solve done before it starts,
// with iters = -1 and the outer ||f||^2, ||r||^2 kept for the host.
__global__ void k_inner_setup_first(SolverScalars* sc, double rtol, double rin, int fixed) {
    if (threadIdx.x != 0) return;
    const double ff = sc->ff, rr = sc->rr;
    if (sc->done || !isfinite(ff) || !isfinite(rr)) {
        sc->done = 1;
        sc->iters = -1;
        return;
    }
    const double tin = fixed ? 0.0 : fmin(0.1, fmax(rin, INNER_MARGIN * rtol * sqrt(ff / rr)));
    sc->ff = rr;
    sc->tol2 = tin * tin;
    sc->done = rr > 0.0 ? 0 : 1;
}

// copy of the solver scalars into pinned host memory, the token last
__global__ void k_publish(const SolverScalars* __restrict__ sc, PubScalars* out, int token) {
    if (threadIdx.x != 0) return;
    out->s = *sc;
    __threadfence_system();
    *reinterpret_cast<volatile int*>(&out->token) = token;
}

__global__ void k_publish_flag(const int* __restrict__ flags, PubScalars* out, int token) {
    if (threadIdx.x != 0) return;
    out->flag = flags[0];
    __threadfence_system();
    *reinterpret_cast<volatile int*>(&out->token) = token;
}

// spin until the pinned buffer carries `token` (false: the stream drained
// without it, or *err holds the stream's error)
static bool wait_token(tpf_ctx* c, int token, hipError_t* err) {
    const volatile int* tk = &c->pub->token;
    *err = hipSuccess;
    for (long spin = 1;; ++spin) {
        if (*tk == token) break;
        if ((spin & 1023) == 0) {
            const hipError_t e = hipStreamQuery(c->stream);
            if (e == hipSuccess) return *tk == token;
            if (e != hipErrorNotReady) {
                *err = e;
                return false;
            }
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return true;
}

// nbytes (a multiple of 4, at most sizeof(SolverScalars)) of device memory
// into the pinned buffer, the token last
__global__ void k_publish_words(const unsigned* __restrict__ src, int nwords, PubScalars* out, int token) {
    if (threadIdx.x != 0) return;
    unsigned* dst = reinterpret_cast<unsigned*>(&out->s);
    for (int i = 0; i < nwords; ++i) dst[i] = src[i];
    __threadfence_system();
    *reinterpret_cast<volatile int*>(&out->token) = token;
}

hipError_t fetch_bytes(tpf_ctx* c, const void* dev, size_t nbytes, void* host) {
    if (c->pub && nbytes % 4 == 0 && nbytes <= sizeof(SolverScalars)) {
        const int token = ++c->pub_token;
        k_publish_words<<<1, 64, 0, c->stream>>>(static_cast<const unsigned*>(dev), (int)(nbytes / 4), c->pub_dev,
                                                 token);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (wait_token(c, token, &e)) {
            std::memcpy(host, const_cast<const SolverScalars*>(&c->pub->s), nbytes);
            return hipSuccess;
        }
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipMemcpyAsync(host, dev, nbytes, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e;
}

hipError_t fetch_flag(tpf_ctx* c, int* flag) {
    if (c->pub) {
        const int token = ++c->pub_token;
        k_publish_flag<<<1, 64, 0, c->stream>>>(c->flags, c->pub_dev, token);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (wait_token(c, token, &e)) {
            *flag = *const_cast<const volatile int*>(&c->pub->flag);
            return hipSuccess;
        }
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipMemcpyAsync(flag, c->flags, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e;
}

// The solver scalars as they stand after the work queued so far.  With the
// pinned buffer a kernel publishes them and the host spins on the token (a
// stream synchronisation would add a copy kernel and a host wake-up, ≈ 50 us
// of idle GPU per read); while spinning it asks the stream every 1024 polls,
// so that a failed launch ends the wait with its error.
hipError_t fetch_scalars(tpf_ctx* c, SolverScalars* out) {
    if (c->pub) {
        const int token = ++c->pub_token;
        k_publish<<<1, 64, 0, c->stream>>>(c->scal, c->pub_dev, token);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (wait_token(c, token, &e)) {
            std::memcpy(out, const_cast<const SolverScalars*>(&c->pub->s), sizeof(SolverScalars));
            return hipSuccess;
        }
        if (e != hipSuccess) return e;
        // the stream drained without the token showing: read it the plain way
    }
    hipError_t e = hipMemcpyAsync(out, c->scal, sizeof(SolverScalars), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e;
}

static hipError_t finalize3(tpf_ctx* c, int nb0, int nb1, int nb2, int op, double arg) {
    prof_begin(c, PC_FINALIZE, (double)(nb0 + nb1 + nb2) * 8);
    k_finalize<<<1, FIN_THREADS, 0, c->stream>>>(nb0, nb1, nb2, c->max_blocks, op, arg, c->N,
                                                 c->partials, c->scal);
    prof_end(c);
    return hipGetLastError();
}
static hipError_t finalize2(tpf_ctx* c, int nb0, int nb1, int op, double arg) {
    return finalize3(c, nb0, nb1, 0, op, arg);
}

hipError_t launch_finalize(tpf_ctx* c, int nblocks, int nv, int op) {
    return finalize2(c, nblocks, nv > 1 ? nblocks : 0, op, 0.0);
}

// ================================================================== 3D level 0, z-marching
// Block 64 x 4 threads over (x, y); each thread walks kz consecutive z planes
// of its column.  z-neighbours come from a rolling register window, x
// neighbours from the adjacent lanes of the wave (a wave is 64 consecutive x
// cells; the two edge lanes load theirs), y neighbours from loads that mostly
// hit the rows the block's other waves just read.  Each field is thus read
// about once from L2 per sweep instead of once per stencil point.

struct Col : ColIndex {
    bool valid;               // lane owns a real column
    bool sxm, sxp;            // x neighbour held by the adjacent lane
    int kslab;                // index of this block's slab of kz planes
    unsigned wxy;             // column next to a wall: 1 x-, 2 x+, 4 y-, 8 y+
    bool wz;                  // walls at both ends of z
    __device__ __forceinline__ void init(const Dims& d, int kz) {
        const int tx = threadIdx.x;
        int bx = 0, by = 0;
        const bool tile = block_tile(d.xcd, (d.nx + BX - 1) / BX, (d.ny + BY - 1) / BY, d.nz / kz, bx, by, kslab);
        const int i0 = bx * BX + tx, j0 = by * BY + threadIdx.y;
        if (!tile) kslab = d.nz / kz;      // empty range: the block only joins its reductions
        valid = tile && i0 < d.nx && j0 < d.ny;
        // inactive lanes take column (0, 0), so every offset stays in the grid
        set(d.nx, d.ny, d.nz, valid ? i0 : 0, valid ? j0 : 0);
        sxm = tx > 0 && i > 0;
        sxp = tx < BX - 1 && i < nx - 1;
        wxy = 0u;
        if (d.walls & 1) wxy |= (i == 0 ? 1u : 0u) | (i == nx - 1 ? 2u : 0u);
        if (d.walls & 2) wxy |= (j == 0 ? 4u : 0u) | (j == ny - 1 ? 8u : 0u);
        wz = (d.walls & 4) != 0;
    }
};

// value of the lane on the left / right (lanes 0 / 63 get their own back)
template <typename V>
__device__ __forceinline__ V lane_m(V v) { return __shfl_up(v, 1, 64); }
template <typename V>
__device__ __forceinline__ V lane_p(V v) { return __shfl_down(v, 1, 64); }

// Coefficients and stencil of one cell from the rolling/neighbour values:
// rho at c and its six neighbours, field at c and its six neighbours.
template <typename S>
struct Nbr7 {
    S c, xm, xp, ym, yp, zm, zp;
    unsigned wm;    // faces on a free-slip wall: 1 x-, 2 x+, 4 y-, 8 y+, 16 z-, 32 z+ (coefficient 0)
};

template <typename S>
__device__ __forceinline__ void faces7(const Nbr7<S>& rho, S* bl, S* bh) {
    bl[0] = (rho.wm & 1u) ? S(0) : recip(rho.xm + rho.c);
    bh[0] = (rho.wm & 2u) ? S(0) : recip(rho.c + rho.xp);
    bl[1] = (rho.wm & 4u) ? S(0) : recip(rho.ym + rho.c);
    bh[1] = (rho.wm & 8u) ? S(0) : recip(rho.c + rho.yp);
    bl[2] = (rho.wm & 16u) ? S(0) : recip(rho.zm + rho.c);
    bh[2] = (rho.wm & 32u) ? S(0) : recip(rho.c + rho.zp);
}

template <typename S>
__device__ __forceinline__ S apply7(const S* bl, const S* bh, const Nbr7<S>& x, S ih2, S& diag) {
    const S acc = bl[0] * (x.c - x.xm) - bh[0] * (x.xp - x.c) + bl[1] * (x.c - x.ym) -
                  bh[1] * (x.yp - x.c) + bl[2] * (x.c - x.zm) - bh[2] * (x.zp - x.c);
    diag = (bl[0] + bh[0] + bl[1] + bh[1] + bl[2] + bh[2]) * ih2;
    return acc * ih2;
}

// Marches the half density and one field along the column through the KZ
// planes of the block's slab (KZ a compile-time constant, the loop fully
// unrolled): with a lookahead of LA planes, the column values of planes up to
// k+LA+1 and the in-plane neighbours and per-cell operands (pre) of planes up
// to k+LA are in flight while plane k is computed.  Unrolling gives every plane's operands their own
// registers, so no loaded value is copied before it is used and the memory
// waits are partial (only for the plane being computed), never a drain.
// fld(idx, i, j, k) loads the field's raw operands at a cell (type V);
// comb(V) forms the field value where it is used; pre(c) loads the per-cell
// operands of the body; body(k, c, rho7, f7, e) computes one plane.
template <typename S, typename V>
struct SideV {           // plane neighbours that need loads
    S hxm, hxp, hym, hyp;
    V fxm, fxp, fym, fyp;
};

#ifndef TPF_MARCH_LOOKAHEAD
#define TPF_MARCH_LOOKAHEAD 2
#endif
template <int KZ, typename Coef, typename S, bool WITH_FIELD, typename F, typename Cmb, typename Pre,
          typename Body>
__device__ __forceinline__ void march(const Col& q, const Coef& cf, int k0, F fld, Cmb comb, Pre pre,
                                      Body body) {
    constexpr int LA = TPF_MARCH_LOOKAHEAD;     // planes of lookahead (1 or 2)
    using V = decltype(fld(0u, 0, 0, 0));
    using E = decltype(pre(0u));
    auto side = [&](int k) {
        SideV<S, V> s;
        const unsigned c = q.at(k);
        s.hxm = q.sxm ? S(0) : cf.hr(c + q.oxm);
        s.hxp = q.sxp ? S(0) : cf.hr(c + q.oxp);
        s.hym = cf.hr(c + q.oym);
        s.hyp = cf.hr(c + q.oyp);
        if (WITH_FIELD) {
            s.fxm = q.sxm ? V{} : fld(c + q.oxm, q.im, q.j, k);
            s.fxp = q.sxp ? V{} : fld(c + q.oxp, q.ip, q.j, k);
            s.fym = fld(c + q.oym, q.i, q.jm, k);
            s.fyp = fld(c + q.oyp, q.i, q.jp, k);
        } else {
            s.fxm = s.fxp = s.fym = s.fyp = V{};
        }
        return s;
    };
    auto hcol = [&](int k) { return cf.hr(q.at(q.kwrap(k))); };
    auto fcol = [&](int k) {
        const int kk = q.kwrap(k);
        return WITH_FIELD ? fld(q.at(kk), q.i, q.j, kk) : V{};
    };
    // h[m], f[m]: column of plane k0 - 1 + m
    S h[KZ + 2];
    V f[KZ + 2];
    SideV<S, V> sd[KZ];
    E e[KZ];
#pragma unroll
    for (int m = 0; m < LA + 2 && m < KZ + 2; ++m) {
        h[m] = hcol(k0 - 1 + m);
        f[m] = fcol(k0 - 1 + m);
    }
#pragma unroll
    for (int t = 0; t < LA && t < KZ; ++t) {
        sd[t] = side(k0 + t);
        e[t] = pre(q.at(k0 + t));
    }
#pragma unroll
    for (int t = 0; t < KZ; ++t) {
        if (t + LA < KZ) {           // loads of plane k+LA and of the column of k+LA+1
            sd[t + LA] = side(k0 + t + LA);
            e[t + LA] = pre(q.at(k0 + t + LA));
            h[t + LA + 2] = hcol(k0 + t + LA + 1);
            f[t + LA + 2] = fcol(k0 + t + LA + 1);
        }
        const S hc = h[t + 1];
        const S lhm = lane_m(hc), lhp = lane_p(hc);
        Nbr7<S> R, X;
        if constexpr (Coef::kWalls)
            R.wm = q.wxy | (q.wz && k0 + t == 0 ? 16u : 0u) | (q.wz && k0 + t == q.nz - 1 ? 32u : 0u);
        else
            R.wm = 0u;
        X.wm = 0u;
        R.c = hc;
        R.zm = h[t];
        R.zp = h[t + 2];
        R.xm = q.sxm ? lhm : sd[t].hxm;
        R.xp = q.sxp ? lhp : sd[t].hxp;
        R.ym = sd[t].hym;
        R.yp = sd[t].hyp;
        if (WITH_FIELD) {
            const S fc = comb(f[t + 1]);
            const S lfm = lane_m(fc), lfp = lane_p(fc);
            X.c = fc;
            X.zm = comb(f[t]);
            X.zp = comb(f[t + 2]);
            X.xm = q.sxm ? lfm : comb(sd[t].fxm);
            X.xp = q.sxp ? lfp : comb(sd[t].fxp);
            X.ym = comb(sd[t].fym);
            X.yp = comb(sd[t].fyp);
        }
        body(k0 + t, q.at(k0 + t), R, X, e[t]);
    }
}

// Run march<KZ> for the block's slab with KZ = kz (8 or 16); padding blocks
// of the XCD tiling (empty slab) do nothing.
template <typename Coef, typename S, bool WITH_FIELD, typename F, typename Cmb, typename Pre, typename Body>
__device__ __forceinline__ void march_kz(const Col& q, const Coef& cf, int kz, F fld, Cmb comb, Pre pre,
                                         Body body) {
    const int k0 = q.kslab * kz;
    if (k0 >= q.nz) return;
    if (kz == 16) march<16, Coef, S, WITH_FIELD>(q, cf, k0, fld, comb, pre, body);
    else march<8, Coef, S, WITH_FIELD>(q, cf, k0, fld, comb, pre, body);
}

template <typename S>
struct Ident {
    __device__ __forceinline__ S operator()(S v) const { return v; }
};
template <typename S>
struct Pair {
    S a, b;
};

struct NoPre {};

// sweep zt = z + omega (r - A z)/d; MODE 2 also emits <r, zt> to region 1
// and <q, zt> to region 2 (stride apart) for the flexible-CG update
template <typename Coef, typename S, int MODE>
__global__ __launch_bounds__(BLOCK) void k_fz_jac(Dims d, int kz, S ih2, S omega, Coef cf,
                                                  const S* __restrict__ r,
                                                  const S* __restrict__ z, S* __restrict__ zt,
                                                  const S* __restrict__ qv,
                                                  const SolverScalars* __restrict__ sc,
                                                  double* __restrict__ partials, long stride) {
    if (sc->done) return;
    Col q;
    q.init(d, kz);
    auto fld = [&](unsigned idx, int, int, int) -> S { return ld(z, idx); };
    auto pre = [&](unsigned c) -> Pair<S> { return Pair<S>{ld(r, c), MODE == 2 ? ld(qv, c) : S(0)}; };
    double v[2] = {0.0, 0.0};
    march_kz<Coef, S, true>(q, cf, kz, fld, Ident<S>{}, pre,
                         [&](int, unsigned c, const Nbr7<S>& R, const Nbr7<S>& X, const Pair<S>& e) {
        S bl[3], bh[3], dg;
        faces7(R, bl, bh);
        const S az = apply7(bl, bh, X, ih2, dg);
        if (q.valid) {
            const S out = X.c + omega * (e.a - az) * recip(dg);
            stn(zt, c, out);
            if (MODE == 2) {
                v[0] += (double)e.a * (double)out;
                v[1] += (double)e.b * (double)out;
            }
        }
    });
    if (MODE == 2) block_partials_2r(v, partials, stride);
}

// first sweep from zero: z = omega r / d; UPD: first the PCG update
// x += alpha p, r -= alpha q with <r, r> to the partials (UPD 2: x is zero
// before this update, the first of a solve from a zero guess, and not read)
template <typename S, typename X>
struct FirstPre {
    S r, q, p;
    X x;
};

template <typename Coef, typename S, typename X, int UPD>
__global__ __launch_bounds__(BLOCK) void k_fz_first(Dims d, int kz, S ih2, S omega, Coef cf,
                                                    X* __restrict__ x, S* __restrict__ r,
                                                    const S* __restrict__ p,
                                                    const S* __restrict__ qv, S* __restrict__ z,
                                                    const SolverScalars* __restrict__ sc,
                                                    double* __restrict__ partials) {
    if (sc->done) return;
    Col q;
    q.init(d, kz);
    const double alpha = UPD ? sc->alpha : 0.0;
    auto none = [](unsigned, int, int, int) { return S(0); };
    auto pre = [&](unsigned c) {
        FirstPre<S, X> e;
        e.r = ld(r, c);
        if (UPD) {
            e.q = ld(qv, c);
            e.p = ld(p, c);
            e.x = UPD == 2 ? X(0) : ld(x, c);
        } else {
            e.q = e.p = S(0);
            e.x = X(0);
        }
        return e;
    };
    double acc = 0.0;
    march_kz<Coef, S, false>(q, cf, kz, none, Ident<S>{}, pre,
                          [&](int, unsigned c, const Nbr7<S>& R, const Nbr7<S>&, const FirstPre<S, X>& e) {
        S bl[3], bh[3];
        faces7(R, bl, bh);
        const S dg = (bl[0] + bh[0] + bl[1] + bh[1] + bl[2] + bh[2]) * ih2;
        if (q.valid) {
            S rn = e.r;
            if (UPD) {
                stn(x, c, X((double)e.x + alpha * (double)e.p));
                rn = S((double)rn - alpha * (double)e.q);
                stn(r, c, rn);
                acc += (double)rn * (double)rn;
            }
            stn(z, c, omega * rn * recip(dg));
        }
    });
    if (UPD) {
        double v[1] = {acc};
        block_partials<1>(v, partials);
    }
}

// p = z + beta p_old (first: p = z), q = A p, <p, q>
template <typename Coef, typename S>
__global__ __launch_bounds__(BLOCK) void k_fz_apply(Dims d, int kz, S ih2, Coef cf, int first,
                                                    const S* __restrict__ z,
                                                    const S* __restrict__ pold,
                                                    S* __restrict__ pnew, S* __restrict__ qv,
                                                    const SolverScalars* __restrict__ sc,
                                                    double* __restrict__ partials) {
    if (sc->done) return;
    Col q;
    q.init(d, kz);
    // p = z + beta p_old without a branch: on the first iteration p_old is
    // not read (z stands in for it, with beta = 0)
    const S beta = first ? S(0) : S(sc->beta);
    const S* po = first ? z : pold;
    auto fld = [&](unsigned idx, int, int, int) -> Pair<S> { return Pair<S>{ld(z, idx), ld(po, idx)}; };
    auto comb = [&](const Pair<S>& v) -> S { return v.a + beta * v.b; };
    auto pre = [](unsigned) { return NoPre{}; };
    double acc = 0.0;
    march_kz<Coef, S, true>(q, cf, kz, fld, comb, pre,
                         [&](int, unsigned c, const Nbr7<S>& R, const Nbr7<S>& X, NoPre) {
        S bl[3], bh[3], dg;
        faces7(R, bl, bh);
        const S aq = apply7(bl, bh, X, ih2, dg);
        if (q.valid) {
            stn(pnew, c, X.c);
            stn(qv, c, aq);
            acc += (double)X.c * (double)aq;
        }
    });
    double v[1] = {acc};
    block_partials<1>(v, partials);
}

// coarse rhs = mean over the 2x2x2 children of (r - A z); kz even.  z pairs
// summed in registers, x pairs by a lane shuffle, y pairs through LDS.
template <typename Coef, typename S>
__global__ __launch_bounds__(BLOCK) void k_fz_restrict(Dims d, Dims cd, int kz, S ih2, S rw, Coef cf,
                                                       const S* __restrict__ r,
                                                       const S* __restrict__ z,
                                                       S* __restrict__ rc,
                                                       const SolverScalars* __restrict__ sc) {
    if (sc->done) return;
    __shared__ S sh[BY][BX];
    Col q;
    q.init(d, kz);
    const int tx = threadIdx.x, ty = threadIdx.y;
    auto fld = [&](unsigned idx, int, int, int) -> S { return ld(z, idx); };
    auto pre = [&](unsigned c) -> S { return ld(r, c); };
    const unsigned cmax = (unsigned)(cd.nx * cd.ny * cd.nz - 1);
    S pair = S(0);
    march_kz<Coef, S, true>(q, cf, kz, fld, Ident<S>{}, pre,
                         [&](int k, unsigned, const Nbr7<S>& R, const Nbr7<S>& X, S rv) {
        S bl[3], bh[3], dg;
        faces7(R, bl, bh);
        const S az = apply7(bl, bh, X, ih2, dg);
        pair += q.valid ? rv - az : S(0);
        if (k & 1) {
            S v = pair + __shfl_xor(pair, 1, 64);
            sh[ty][tx] = v;
            __syncthreads();
            if (q.valid && (tx & 1) == 0 && (ty & 1) == 0) {
                const S s = sh[ty][tx] + sh[ty + 1][tx];
                const unsigned cc = ((unsigned)(k >> 1) * cd.ny + (q.j >> 1)) * cd.nx + (q.i >> 1);
                stn(rc, min(cc, cmax), s * rw);
            }
            __syncthreads();
            pair = S(0);
        }
    });
}

// r = -(b - mean) - A x (x FP64 read in precision S), stored as R;
// |f|^2 -> region 0, |r|^2 -> region 1, with FL | |A||x| |^2 -> region 2
template <typename Coef, typename S, typename R, bool FL = true>
__global__ __launch_bounds__(BLOCK) void k_fz_resid(Dims d, int kz, S ih2, Coef cf,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ x,
                                                    R* __restrict__ r,
                                                    const SolverScalars* __restrict__ sc,
                                                    double* __restrict__ partials, long stride) {
    Col q;
    q.init(d, kz);
    const double mean = sc->mean;
    auto fld = [&](unsigned idx, int, int, int) -> S { return S(ld(x, idx)); };
    auto pre = [&](unsigned c) -> double { return ld(b, c); };
    double v[3] = {0.0, 0.0, 0.0};
    march_kz<Coef, S, true>(q, cf, kz, fld, Ident<S>{}, pre,
                         [&](int, unsigned c, const Nbr7<S>& Rh, const Nbr7<S>& X, double bc) {
        S bl[3], bh[3], dg;
        faces7(Rh, bl, bh);
        const S ax = apply7(bl, bh, X, ih2, dg);
        if (q.valid) {
            const double f = -(bc - mean);
            const double rr = f - (double)ax;
            st(r, c, R(rr));
            v[0] += f * f;
            v[1] += rr * rr;
            if (FL) {
            const double aa = (fabs((double)bl[0] * (double)(X.c - X.xm)) + fabs((double)bh[0] * (double)(X.xp - X.c)) +
                               fabs((double)bl[1] * (double)(X.c - X.ym)) + fabs((double)bh[1] * (double)(X.yp - X.c)) +
                               fabs((double)bl[2] * (double)(X.c - X.zm)) + fabs((double)bh[2] * (double)(X.zp - X.c))) *
                              (double)ih2;
            v[2] += aa * aa;
            }
        }
    });
    block_partials_3r(v, partials, stride);
}

// ================================================================== host driver

static unsigned vgrid(long N) {
    const long nb = (N + BLOCK - 1) / BLOCK;
    return (unsigned)(nb < VBLOCKS ? nb : VBLOCKS);
}

// W: the context's box has walls (the level-0 coefficient policies, and so
// every level-0 kernel, are instantiated with wall bits)
template <typename T, typename S, bool W = false>
struct Solver {
    tpf_ctx* c;
    int dim;
    S w1, w2;       // damped-Jacobi weights of the two sweeps before (w1, w2) and after (w2, w1)

    CoefPhi<T, S, W> coef_phi(const void* phi) const {
        const Phys P = phys_of(c);
        const S inf = std::numeric_limits<S>::infinity();
        return CoefPhi<T, S, W>{static_cast<const T*>(phi), S(0.5 * P.rho2), S(0.5 * (P.rho1 - P.rho2)),
                             P.clamp ? S(0) : -inf, P.clamp ? S(1) : inf};
    }
    // fine-level coefficients: the half density computed by half_rho()
    CoefRho<S, W> coef_fine() const { return CoefRho<S, W>{tp<S>(c->rhoh)}; }
    void half_rho(const void* phi) {
        prof_begin(c, PC_VECTOR, (double)c->N * (sizeof(T) + sizeof(S)));
        k_half_rho<T, S, W><<<vgrid(c->N), BLOCK, 0, c->stream>>>(c->N, coef_phi(phi), tp<S>(c->rhoh));
        prof_end(c);
    }
    CoefStored<S> coef(int l) const {
        return CoefStored<S>{tp<S>(c->lv[l].beta[0]), tp<S>(c->lv[l].beta[1]),
                             tp<S>(c->lv[l].beta[2])};
    }
    S ih2(int l) const { return S(1.0 / (c->lv[l].h * c->lv[l].h)); }
    dim3 grid(int l) const { return grid_of(c->lv[l].n); }
    // level 0 carries the walls (its coefficients are formed from rho; the
    // stored coefficients of the coarse levels hold the zeros already)
    Dims dims(int l) const { return dims_of(c->lv[l].n, l == 0 ? c->walls : 0); }
    // restriction weight: mean over the 2^d children times the coarse-grid
    // correction weight (the coarse problem is linear, so scaling its
    // right-hand side scales the correction; R stays proportional to P^T)
    S rw() const { return S(c->mg_alpha / (dim == 3 ? 8.0 : 4.0)); }
    // damped Jacobi sweeps on the coarsest grid (largest dimension mx): 2 mx
    // by default; more do not lower the PCG iteration count
    int coarse_sweeps(int mx) const { return (c->coarse_sweeps_per_cell > 0 ? c->coarse_sweeps_per_cell : 2) * mx; }
    double fb(int l, double fields) const { return (double)c->lv[l].N * sizeof(S) * fields; }
    // fields moved by the coefficients: phi on the fine level, DIM arrays below
    double cfields(int l) const { return l == 0 ? (double)sizeof(T) / sizeof(S) : (double)dim; }
    long nbl(int l) const { return nblocks_of(c->lv[l].n); }
    // level 0 in 3D runs the z-marching kernels: kz planes per block
    bool march0() const { return dim == 3 && c->march && kz() > 0; }
    // planes per block of the z-marching kernels: 8 or 16 (the march is
    // unrolled for these); 0 when nz admits neither (plain kernels then).
    // 16 where the grid still gives at least 4096 blocks (at 256^3: 13.94 ->
    // 13.86 ms per step, one prologue per 16 planes), else 8.
    int kz() const {
        const int* n = c->lv[0].n;
        const int nz = n[2];
        if ((c->kz_override == 8 || c->kz_override == 16) && nz % c->kz_override == 0) return c->kz_override;
        const long blocks16 = (long)((n[0] + BX - 1) / BX) * ((n[1] + BY - 1) / BY) * (nz / 16);
        if (nz % 16 == 0 && blocks16 >= 4096) return 16;
        if (nz % 8 == 0) return 8;
        return 0;
    }
    dim3 mgrid() const {
        const Level& L = c->lv[0];
        return tile_grid((L.n[0] + BX - 1) / BX, (L.n[1] + BY - 1) / BY, L.n[2] / kz());
    }
    // blocks of the level-0 kernels that emit partial sums
    long nb0() const {
        if (!march0()) return nbl(0);
        const dim3 g = mgrid();
        return (long)g.x * g.y * g.z;
    }

    template <int DIM>
    void build_betas_t(const void* phi) {
        const dim3 b(BX, BY);
        half_rho(phi);
        if (c->nlev < 2) return;
        k_beta_from_phi<CoefRho<S, W>, S, DIM><<<grid(1), b, 0, c->stream>>>(
            dims(0), dims(1), coef_fine(), tp<S>(c->lv[1].beta[0]), tp<S>(c->lv[1].beta[1]),
            tp<S>(c->lv[1].beta[2]));
        for (int l = 2; l < c->nlev; ++l)
            k_beta_coarsen<S, DIM><<<grid(l), b, 0, c->stream>>>(
                dims(l - 1), dims(l), coef(l - 1), tp<S>(c->lv[l].beta[0]),
                tp<S>(c->lv[l].beta[1]), tp<S>(c->lv[l].beta[2]));
        for (int l = 1; l < c->nlev; ++l)
            if (separate_level<DIM>(l))
                k_dinv<S, DIM><<<grid(l), b, 0, c->stream>>>(dims(l), ih2(l), coef(l), tp<S>(c->lv[l].dinv));
    }
    // a coarse level that runs the separate down/up kernels (level_down,
    // level_up): not the tail, not the coarsest grid, not a fused level
    template <int DIM>
    bool separate_level(int l) const {
        if (l < 1 || l == c->nlev - 1) return false;
        const int tf = tail_first();
        if (tf >= 1 && l >= tf) return false;
        return !(DIM == 3 && c->coarse_fused && c->lv[l].N <= CFUSE_MAX_CELLS);
    }
    void build_betas(const void* phi) {
        if (dim == 2) build_betas_t<2>(phi); else build_betas_t<3>(phi);
    }

    dim3 restrict_block() const { return dim == 3 ? dim3(BX, 2, 2) : dim3(BX, 4, 1); }
    dim3 restrict_grid(int l) const {
        const Level& L = c->lv[l];
        return dim == 3 ? tile_grid((L.n[0] + BX - 1) / BX, (L.n[1] + 1) / 2, (L.n[2] + 1) / 2)
                        : tile_grid((L.n[0] + BX - 1) / BX, (L.n[1] + 3) / 4, 1);
    }

    // Pre-smoothing and restriction at level l.  The first sweep writes z (A),
    // the second zt (B), the restriction reads zt.
    template <int DIM, typename Coef>
    void level_down(int l, Coef cf, bool fine, bool first_done) {
        Level& L = c->lv[l];
        const dim3 b(BX, BY);
        S* z = tp<S>(L.z);
        S* zt = tp<S>(L.zt);
        S* r = tp<S>(L.r);
        const double cfl = cfields(l);
        if constexpr (std::is_same<Coef, CoefRho<S, W>>::value) {
            if (DIM == 3 && march0()) {
                Level& Lc = c->lv[l + 1];
                if (!first_done) {
                    prof_begin(c, PC_F_FIRST0, fb(l, 2 + cfl));
                    k_fz_first<Coef, S, S, 0><<<mgrid(), b, 0, c->stream>>>(dims(0), kz(), ih2(0), w1, cf, nullptr,
                                                                       r, nullptr, nullptr, z, c->scal, nullptr);
                    prof_end(c);
                }
                prof_begin(c, PC_F_SWEEP, fb(l, 3 + cfl));
                k_fz_jac<Coef, S, 0><<<mgrid(), b, 0, c->stream>>>(dims(0), kz(), ih2(0), w2, cf, r, z, zt,
                                                               nullptr, c->scal, nullptr, 0);
                prof_end(c);
                prof_begin(c, PC_F_RESTRICT, fb(l, 2 + cfl) + (double)Lc.N * sizeof(S));
                k_fz_restrict<Coef, S><<<mgrid(), b, 0, c->stream>>>(dims(0), dims(1), kz(), ih2(0), rw(), cf, r, zt,
                                                                 tp<S>(Lc.r), c->scal);
                prof_end(c);
                return;
            }
        }
        if constexpr (std::is_same<Coef, CoefStored<S>>::value) {
            if (!first_done) {     // a stored level: both sweeps in one pass (1 / d stored per solve)
                prof_begin(c, PC_COARSE_LEVELS, fb(l, 3 + cfl));
                k_jac2_first<S, DIM><<<grid(l), b, 0, c->stream>>>(dims(l), ih2(l), w1, w2, cf, r,
                                                                   tp<S>(L.dinv), zt, c->scal);
                prof_end(c);
                first_done = true;
                z = nullptr;
            }
        }
        if (!first_done) {
            prof_begin(c, fine ? PC_F_FIRST0 : PC_COARSE_LEVELS, fb(l, 2 + cfl));
            k_jac_first<Coef, S, DIM><<<grid(l), b, 0, c->stream>>>(dims(l), ih2(l), w1, cf, r, z, c->scal);
            prof_end(c);
        }
        if (z) {
            prof_begin(c, fine ? PC_F_SWEEP : PC_COARSE_LEVELS, fb(l, 3 + cfl));
            k_jac<Coef, S, DIM, 0><<<grid(l), b, 0, c->stream>>>(dims(l), ih2(l), w2, cf, r, z, zt, nullptr,
                                                                  c->scal, nullptr, 0);
            prof_end(c);
        }
        Level& Lc = c->lv[l + 1];
        prof_begin(c, fine ? PC_F_RESTRICT : PC_COARSE_LEVELS, fb(l, 2 + cfl) + (double)Lc.N * sizeof(S));
        k_restrict<Coef, S, DIM><<<restrict_grid(l), restrict_block(), 0, c->stream>>>(
            dims(l), dims(l + 1), ih2(l), rw(), cf, r, zt, tp<S>(Lc.r), c->scal);
        prof_end(c);
    }

    // Prolongation (B += P zc) and the two post-smoothing sweeps (B -> A,
    // A -> B) at level l; dot: the last sweep emits the flexible-CG dots.
    template <int DIM, typename Coef>
    void level_up(int l, Coef cf, bool fine, const S* zc, int dot) {
        Level& L = c->lv[l];
        const dim3 b(BX, BY);
        S* z = tp<S>(L.z);
        S* zt = tp<S>(L.zt);
        const S* r = tp<S>(L.r);
        const S* qv = tp<S>(c->qv);
        double* part = c->partials + c->max_blocks;
        const long stride = c->max_blocks;
        const double cb = (double)c->lv[l + 1].N * sizeof(S);
        const double cfl = cfields(l);
        prof_begin(c, fine ? PC_F_PROLONG : PC_COARSE_LEVELS, fb(l, 2) + cb);
        k_prolong<S, DIM><<<grid(l + 1), b, 0, c->stream>>>(dims(l), dims(l + 1), zc, zt, c->scal);
        prof_end(c);
        if constexpr (std::is_same<Coef, CoefRho<S, W>>::value) {
            if (DIM == 3 && march0()) {
                prof_begin(c, PC_F_SWEEP, fb(l, 3 + cfl));
                k_fz_jac<Coef, S, 0><<<mgrid(), b, 0, c->stream>>>(dims(0), kz(), ih2(0), w2, cf, r, zt, z,
                                                               nullptr, c->scal, nullptr, 0);
                prof_end(c);
                prof_begin(c, PC_F_SWEEPDOT, fb(l, 3 + (dot ? 1 : 0) + cfl));
                if (dot)
                    k_fz_jac<Coef, S, 2><<<mgrid(), b, 0, c->stream>>>(dims(0), kz(), ih2(0), w1, cf, r, z, zt,
                                                                   qv, c->scal, part, stride);
                else
                    k_fz_jac<Coef, S, 0><<<mgrid(), b, 0, c->stream>>>(dims(0), kz(), ih2(0), w1, cf, r, z, zt,
                                                                   nullptr, c->scal, nullptr, 0);
                prof_end(c);
                return;
            }
        }
        prof_begin(c, fine ? PC_F_SWEEP : PC_COARSE_LEVELS, fb(l, 3 + cfl));
        k_jac<Coef, S, DIM, 0><<<grid(l), b, 0, c->stream>>>(dims(l), ih2(l), w2, cf, r, zt, z, nullptr,
                                                              c->scal, nullptr, 0);
        prof_end(c);
        prof_begin(c, fine ? PC_F_SWEEPDOT : PC_COARSE_LEVELS, fb(l, 3 + (dot ? 1 : 0) + cfl));
        if (dot)
            k_jac<Coef, S, DIM, 1><<<grid(l), b, 0, c->stream>>>(dims(l), ih2(l), w1, cf, r, z, zt, qv,
                                                                  c->scal, part, stride);
        else
            k_jac<Coef, S, DIM, 0><<<grid(l), b, 0, c->stream>>>(dims(l), ih2(l), w1, cf, r, z, zt, nullptr,
                                                                  c->scal, nullptr, 0);
        prof_end(c);
    }

    // first level of the LDS tail (-1: none): the shallowest level >= 1 from
    // which all remaining levels fit in TAIL_LDS_BYTES
    int tail_first() const {
        if (c->no_tail || c->nlev < 2) return -1;
        size_t bytes = 0;
        int first = -1;
        for (int l = c->nlev - 1; l >= 1 && c->nlev - l <= TAIL_MAX_LEVELS; --l) {
            bytes += 3 * (size_t)c->lv[l].N * sizeof(S);
            if (bytes > TAIL_LDS_BYTES) break;
            first = l;
        }
        return first;
    }

    template <int DIM>
    const S* tail(int l0) {
        TailDesc D;
        D.nlev = c->nlev - l0;
        D.rw = (double)rw();
        int off = 0;
        for (int q = 0; q < D.nlev; ++q) {
            const Level& L = c->lv[l0 + q];
            for (int a = 0; a < 3; ++a) {
                D.n[q][a] = L.n[a];
                D.beta[q][a] = L.beta[a];
            }
            D.off[q] = off;
            off += 3 * (int)L.N;
            auto lg2 = [](int v) {
                int e = 0;
                while ((1 << e) < v) ++e;
                return (1 << e) == v ? e : -1;
            };
            const int lx = lg2(L.n[0]), ly = lg2(L.n[1]);
            D.lg[q][0] = lx >= 0 && ly >= 0 ? lx : -1;
            D.lg[q][1] = lx >= 0 && ly >= 0 ? lx + ly : -1;
            D.ih2[q] = 1.0 / (L.h * L.h);
        }
        const Level& Ll = c->lv[c->nlev - 1];
        const int mx = std::max(Ll.n[0], std::max(Ll.n[1], Ll.n[2]));
        prof_begin(c, PC_COARSE_LEVELS, (double)off * sizeof(S));
        k_tail<S, DIM><<<1, 1024, (size_t)off * sizeof(S), c->stream>>>(D, w1, w2, S(0.8), coarse_sweeps(mx),
                                                                        tp<S>(c->lv[l0].r),
                                                                        tp<S>(c->lv[l0].zt), c->scal);
        prof_end(c);
        return tp<S>(c->lv[l0].zt);
    }

    // V-cycle from level l >= 1 (stored coefficients); the correction ends in zt
    // k_cdown, the levels below, k_cup on stored-coefficient level l (3D)
    // with TE^3 tiles; the correction ends in z
    template <int TE>
    const S* fused_level(int l) {
        Level& L = c->lv[l];
        const Level& Lc = c->lv[l + 1];
        const CoefStored<S> cf = coef(l);
        const dim3 g = tile_grid((L.n[0] + TE - 1) / TE, (L.n[1] + TE - 1) / TE, (L.n[2] + TE - 1) / TE);
        const double cb = (double)Lc.N * sizeof(S);
        prof_begin(c, PC_COARSE_LEVELS, fb(l, 2 + 3) + cb);      // r, 3 coefficients -> zt, coarse r
        k_cdown<S, TE><<<g, BLOCK, 0, c->stream>>>(dims(l), dims(l + 1), ih2(l), w1, w2, rw(), cf, tp<S>(L.r),
                                                   tp<S>(L.zt), tp<S>(Lc.r), c->scal);
        prof_end(c);
        const S* zc = vcycle_coarse<3>(l + 1);
        prof_begin(c, PC_COARSE_LEVELS, fb(l, 3 + 3) + cb);      // zt, r, 3 coefficients, zc -> z
        k_cup<S, TE><<<g, BLOCK, 0, c->stream>>>(dims(l), dims(l + 1), ih2(l), w1, w2, cf, tp<S>(L.r), zc,
                                                 tp<S>(L.zt), tp<S>(L.z), c->scal);
        prof_end(c);
        return tp<S>(L.z);
    }

    template <int DIM>
    const S* vcycle_coarse(int l) {
        Level& L = c->lv[l];
        if (l == tail_first()) return tail<DIM>(l);
        if (l == c->nlev - 1) {
            const int mx = std::max(L.n[0], std::max(L.n[1], L.n[2]));
            prof_begin(c, PC_COARSE_LEVELS, fb(l, 3));
            k_coarse<S, DIM><<<1, 1024, 0, c->stream>>>(dims(l), ih2(l), S(0.8), coarse_sweeps(mx), coef(l),
                                                        tp<S>(L.r), tp<S>(L.zt), tp<S>(L.z), c->scal);
            prof_end(c);
            return tp<S>(L.zt);
        }
        if (DIM == 3 && c->coarse_fused && L.N <= CFUSE_MAX_CELLS) {
            // one launch down, one up (k_cdown, k_cup); the correction ends in
            // z, since k_cup reads zt on its halo while other blocks write.
            // 8^3 tiles, or 4^3 where 8^3 tiles would leave compute units idle
            const auto ntiles = [&](int e) {
                return (long)((L.n[0] + e - 1) / e) * ((L.n[1] + e - 1) / e) * ((L.n[2] + e - 1) / e);
            };
            if (ntiles(8) < 256) return fused_level<4>(l);
            return fused_level<8>(l);
        }
        level_down<DIM>(l, coef(l), false, false);
        const S* zc = vcycle_coarse<DIM>(l + 1);
        level_up<DIM>(l, coef(l), false, zc, 0);
        return tp<S>(L.zt);
    }

    // Full V-cycle from level 0 (phi coefficients), result in lv[0].zt.
    // first_done: the first pre-smoothing sweep was fused into the PCG update.
    // dot: the last sweep emits <r, z> partials to region 1.
    template <int DIM>
    void vcycle_t(const void* phi, bool first_done) {
        const auto cf = coef_fine();
        Level& L = c->lv[0];
        if (c->nlev == 1 && DIM == 3 && march0()) {
            // no coarsening possible: two Jacobi sweeps (still symmetric)
            const dim3 b(BX, BY);
            if (!first_done) {
                prof_begin(c, PC_F_FIRST0, fb(0, 2 + cfields(0)));
                k_fz_first<CoefRho<S, W>, S, S, 0><<<mgrid(), b, 0, c->stream>>>(dims(0), kz(), ih2(0), w1, cf, nullptr,
                                                                   tp<S>(L.r), nullptr, nullptr, tp<S>(L.z),
                                                                   c->scal, nullptr);
                prof_end(c);
            }
            prof_begin(c, PC_F_SWEEPDOT, fb(0, 3 + cfields(0)));
            k_fz_jac<CoefRho<S, W>, S, 2><<<mgrid(), b, 0, c->stream>>>(dims(0), kz(), ih2(0), w2, cf, tp<S>(L.r),
                                                           tp<S>(L.z), tp<S>(L.zt), tp<S>(c->qv), c->scal,
                                                           c->partials + c->max_blocks, c->max_blocks);
            prof_end(c);
            return;
        }
        if (c->nlev == 1) {
            // no coarsening possible: two Jacobi sweeps (still symmetric)
            if (!first_done) {
                prof_begin(c, PC_F_FIRST0, fb(0, 2 + cfields(0)));
                k_jac_first<CoefRho<S, W>, S, DIM><<<grid(0), dim3(BX, BY), 0, c->stream>>>(
                    dims(0), ih2(0), w1, cf, tp<S>(L.r), tp<S>(L.z), c->scal);
                prof_end(c);
            }
            prof_begin(c, PC_F_SWEEPDOT, fb(0, 3 + cfields(0)));
            k_jac<CoefRho<S, W>, S, DIM, 1><<<grid(0), dim3(BX, BY), 0, c->stream>>>(
                dims(0), ih2(0), w2, cf, tp<S>(L.r), tp<S>(L.z), tp<S>(L.zt), tp<S>(c->qv),
                c->scal, c->partials + c->max_blocks, c->max_blocks);
            prof_end(c);
            return;
        }
        level_down<DIM>(0, cf, true, first_done);
        const S* zc = vcycle_coarse<DIM>(1);
        level_up<DIM>(0, cf, true, zc, 1);
    }
    void vcycle(const void* phi, bool first_done) {
        if (dim == 2) vcycle_t<2>(phi, first_done); else vcycle_t<3>(phi, first_done);
    }

    // p = z + beta p, q = A p (-> alpha), then x, r update fused with the
    // first pre-smoothing sweep
    // xz: x is zero before this update (the first of a solve from zero)
    template <int DIM, typename X>
    void apply_update(const void* phi, int first, X* x, bool xz) {
        const auto cf = coef_fine();
        const dim3 b(BX, BY);
        S* pold = tp<S>(c->pv);
        S* pnew = tp<S>(c->pv2);
        if (DIM == 3 && march0()) {
            prof_begin(c, PC_F_APPLY, fb(0, (first ? 1 : 2) + 2 + cfields(0)));
            k_fz_apply<CoefRho<S, W>, S><<<mgrid(), b, 0, c->stream>>>(dims(0), kz(), ih2(0), cf, first, tp<S>(c->lv[0].zt),
                                                          pold, pnew, tp<S>(c->qv), c->scal, c->partials);
            prof_end(c);
            (void)finalize2(c, (int)nb0(), 0, FIN_ALPHA, 0.0);
            prof_begin(c, PC_F_FIRST, fb(0, 5 + cfields(0)) + (xz ? 1.0 : 2.0) * c->N * sizeof(X));
            if (xz)
                k_fz_first<CoefRho<S, W>, S, X, 2><<<mgrid(), b, 0, c->stream>>>(dims(0), kz(), ih2(0), w1, cf, x,
                                                                   tp<S>(c->lv[0].r), pnew, tp<S>(c->qv),
                                                                   tp<S>(c->lv[0].z), c->scal, c->partials);
            else
                k_fz_first<CoefRho<S, W>, S, X, 1><<<mgrid(), b, 0, c->stream>>>(dims(0), kz(), ih2(0), w1, cf, x,
                                                                   tp<S>(c->lv[0].r), pnew, tp<S>(c->qv),
                                                                   tp<S>(c->lv[0].z), c->scal, c->partials);
            prof_end(c);
            std::swap(c->pv, c->pv2);
            return;
        }
        prof_begin(c, PC_F_APPLY, fb(0, (first ? 1 : 2) + 2 + cfields(0)));
        k_apply<CoefRho<S, W>, S, DIM><<<grid(0), b, 0, c->stream>>>(
            dims(0), ih2(0), cf, first, tp<S>(c->lv[0].zt), pold, pnew, tp<S>(c->qv), c->scal, c->partials);
        prof_end(c);
        (void)finalize2(c, (int)nbl(0), 0, FIN_ALPHA, 0.0);
        prof_begin(c, PC_F_FIRST, fb(0, 5 + cfields(0)) + (xz ? 1.0 : 2.0) * c->N * sizeof(X));
        if (xz)
            k_jac_first_update<CoefRho<S, W>, S, X, DIM, true><<<grid(0), b, 0, c->stream>>>(
                dims(0), ih2(0), w1, cf, x, tp<S>(c->lv[0].r), pnew, tp<S>(c->qv), tp<S>(c->lv[0].z),
                c->scal, c->partials);
        else
            k_jac_first_update<CoefRho<S, W>, S, X, DIM, false><<<grid(0), b, 0, c->stream>>>(
                dims(0), ih2(0), w1, cf, x, tp<S>(c->lv[0].r), pnew, tp<S>(c->qv), tp<S>(c->lv[0].z),
                c->scal, c->partials);
        prof_end(c);
        std::swap(c->pv, c->pv2);
    }

    // PCG on level 0 for x (type X); residual already in lv[0].r and the
    // scalars initialised (ff, rr, tol2, done).  The iterations run ahead of
    // the host: it reads the done flag first after the iteration count of
    // the previous solve of the same kind (slot) in the same RK stage (the
    // counts repeat from step to step stage by stage, e.g. 3, 4, 4, 4), then
    // every 2 iterations.
    // Iterations launched after convergence exit at once; the profiler books
    // them as no-work launches.
    // one PCG iteration after the first: new direction and its operator
    // application, the x and r update with the first sweep, the rest of the
    // V-cycle, and the flexible-CG scalars
    template <typename X>
    void iteration(const void* phi, int first, X* x, bool xz = false) {
        if (dim == 2) apply_update<2, X>(phi, first, x, xz);
        else apply_update<3, X>(phi, first, x, xz);
        vcycle(phi, true);
        (void)finalize3(c, (int)nb0(), (int)nb0(), (int)nb0(), FIN_BETA, 0.0);
    }

    // Two iterations (not the first of a solve) captured as one HIP graph on
    // a private stream and kept per (x, direction buffer): the pair swaps the
    // direction buffers twice, so it leaves them as it found them and its
    // launches are the same every time.  *out = nullptr: no graph (the cache
    // is full), the caller launches directly.
    template <typename X>
    hipError_t pair_graph(const void* phi, X* x, hipGraphExec_t* out) {
        *out = nullptr;
        const void* key[2] = {static_cast<const void*>(x), c->pv};
        for (int g = 0; g < c->n_pcg_graphs; ++g)
            if (c->pcg_graphs[g].key[0] == key[0] && c->pcg_graphs[g].key[1] == key[1]) {
                *out = c->pcg_graphs[g].exec;
                return hipSuccess;
            }
        if (c->n_pcg_graphs == (int)(sizeof(c->pcg_graphs) / sizeof(c->pcg_graphs[0]))) return hipSuccess;
        if (!c->cap_stream) {
            hipError_t ec = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
            if (ec != hipSuccess) {
                c->cap_stream = nullptr;
                return ec;
            }
        }
        hipStream_t user = c->stream;
        c->stream = c->cap_stream;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            iteration(phi, 0, x);
            iteration(phi, 0, x);
            e = hipStreamEndCapture(c->stream, &g);
        }
        c->stream = user;
        hipGraphExec_t ex = nullptr;
        if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) return e;
        c->pcg_graphs[c->n_pcg_graphs].key[0] = key[0];
        c->pcg_graphs[c->n_pcg_graphs].key[1] = key[1];
        c->pcg_graphs[c->n_pcg_graphs].exec = ex;
        ++c->n_pcg_graphs;
        *out = ex;
        return hipSuccess;
    }

    // x_zero: x starts at zero and is not read before the first update writes
    // it (nothing is written when the solve stops before that update)
    template <typename X>
    hipError_t pcg(const void* phi, X* x, int maxit, int slot, SolverScalars* last, bool* have_last,
                   bool x_zero = false) {
        vcycle(phi, false);                                       // z = M r, <r,z>
        (void)finalize2(c, 0, (int)nb0(), FIN_RZ0, 0.0);
        int it = 0;
        bool first = true;
        int& pred = c->pred_iters[slot][c->rk_stage & 3];
        int window = pred > 0 ? pred : 4;
        snap_.resize((size_t)maxit + 1);
        SolverScalars s{};
        while (it < maxit) {
            for (int k = 0; k < window && it < maxit;) {
                if (!first && c->pcg_graph && !c->prof_mask && k + 1 < window && it + 1 < maxit) {
                    hipGraphExec_t ex = nullptr;
                    hipError_t e = pair_graph(phi, x, &ex);
                    if (e != hipSuccess) return e;
                    if (ex) {
                        snapshot(snap_[it]);
                        snapshot(snap_[it + 1]);
                        e = hipGraphLaunch(ex, c->stream);
                        if (e != hipSuccess) return e;
                        k += 2;
                        it += 2;
                        continue;
                    }
                }
                snapshot(snap_[it]);
                iteration(phi, first ? 1 : 0, x, first && x_zero);
                first = false;
                ++k;
                ++it;
            }
            window = 2;
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            e = fetch_scalars(c, &s);
            if (e != hipSuccess) return e;
            *have_last = true;
            if (s.done) break;
        }
        // iters = -1: done before the first iteration (k_inner_setup_first)
        const int useful = s.iters < 0 ? 0 : s.iters;
        if (s.done && useful < it) {
            ProfSnap now;
            snapshot(now);
            for (int q = 0; q < NPROF; ++q) {
                c->prof_noop[q] += now.n[q] - snap_[useful].n[q];
                c->prof_noop_bytes[q] += now.b[q] - snap_[useful].b[q];
            }
        }
        if (s.done && s.iters >= 0) pred = s.iters;
        // nothing is launched after the last read: it holds the final scalars
        *last = s;
        return hipGetLastError();
    }
    struct ProfSnap {
        long n[NPROF];
        double b[NPROF];
    };
    std::vector<ProfSnap> snap_;
    void snapshot(ProfSnap& o) const {
        for (int q = 0; q < NPROF; ++q) {
            o.n[q] = c->prof_issued[q];
            o.b[q] = c->prof_issued_bytes[q];
        }
    }

    // r = f - A x with the coefficient policy cf (FP64 path: the fine-level
    // half densities; mixed path: FP64 coefficients straight from phi)
    // FL: also the rounding floor |A||x| (without it the floor is 0, so the
    // convergence test is the tolerance alone)
    template <typename R, bool FL = true, typename Coef>
    void residual(Coef cf, R* r) {
        prof_begin(c, PC_RESID, (double)c->N * (8 + 8 + sizeof(T) + sizeof(R)));
        if (march0())
            k_fz_resid<Coef, S, R, FL><<<mgrid(), dim3(BX, BY), 0, c->stream>>>(
                dims(0), kz(), ih2(0), cf, c->b, c->p, r, c->scal, c->partials, c->max_blocks);
        else if (dim == 3)
            k_resid<Coef, S, R, 3, FL><<<grid(0), dim3(BX, BY), 0, c->stream>>>(
                dims(0), ih2(0), cf, c->b, c->p, r, c->scal, c->partials, c->max_blocks);
        else
            k_resid<Coef, S, R, 2, FL><<<grid(0), dim3(BX, BY), 0, c->stream>>>(
                dims(0), ih2(0), cf, c->b, c->p, r, c->scal, c->partials, c->max_blocks);
        prof_end(c);
    }
};

hipError_t launch_rhs_mean(tpf_ctx* c) {
    const unsigned nb = vgrid(c->N);
    k_sum<<<nb, BLOCK, 0, c->stream>>>(c->N, c->b, c->partials);
    return finalize2(c, (int)nb, 0, FIN_MEAN, 0.0);
}

static hipError_t remove_mean(tpf_ctx* c, double* x) {
    const unsigned nb = vgrid(c->N);
    prof_begin(c, PC_VECTOR, (double)c->N * 8 * 3);
    k_sum<<<nb, BLOCK, 0, c->stream>>>(c->N, x, c->partials);
    prof_end(c);
    hipError_t e = finalize2(c, (int)nb, 0, FIN_SUM, 0.0);
    if (e != hipSuccess) return e;
    k_sub_mean<<<nb, BLOCK, 0, c->stream>>>(c->N, x, c->scal);
    return hipGetLastError();
}

static tpf_status read_scalars(tpf_ctx* c, SolverScalars* s) {
    const hipError_t e = fetch_scalars(c, s);
    if (e != hipSuccess) return hip_fail(e, "reading solver scalars");
    return TPF_OK;
}

// Damped-Jacobi weights of the two smoothing sweeps.  3D: the roots of the
// degree-2 Chebyshev polynomial on [1/2, 2] (the spectrum of D^-1 A lies in
// (0, 2]; the sweeps damp its upper three quarters): 1 / (5/4 -+ (3/4) cos(pi/4)).
// 2D: 0.8 twice (the Chebyshev pair measured no better there).
static void weights_of(int dim, double& w1, double& w2) {
    if (dim == 2) {
        w1 = w2 = 0.8;
        return;
    }
    const double c = 0.75 * std::cos(M_PI / 4.0);
    w1 = 1.0 / (1.25 + c);
    w2 = 1.0 / (1.25 - c);
}

// Zero-mean gauge of the pressure (Z13 of the readings): applied where the
// pressure leaves the library.  Inside a step only G p is used, which the
// gauge does not change, so the solves skip it.
tpf_status gauge_pressure(tpf_ctx* c) {
    hipError_t e = remove_mean(c, c->p);
    return e == hipSuccess ? TPF_OK : hip_fail(e, "mean removal");
}

// Solve with beta from phi (state precision); right-hand side in c->b with
// its mean in scal->mean; x = c->p (warm start in, solution out; its mean is
// whatever the warm start carried, see gauge_pressure).
template <bool W>
static tpf_status poisson_solve_t(tpf_ctx* c, const void* phi, int* iters, double* relres, int* outer) {
    const double rtol = c->P.poisson_rtol;
    const int maxit = c->P.poisson_maxit;
    SolverScalars s;
    hipError_t e;
    if (!c->mixed) {
        double w1, w2;
        weights_of(c->dim, w1, w2);
        Solver<double, double, W> sv{c, c->dim, w1, w2};
        const bool fixed = c->fixed_inner > 0;
        sv.build_betas(phi);
        sv.template residual<double>(sv.coef_fine(), tp<double>(c->lv[0].r));
        (void)finalize3(c, (int)sv.nb0(), (int)sv.nb0(), (int)sv.nb0(), FIN_INIT, fixed ? 0.0 : rtol * rtol);
        bool have = false;
        e = sv.template pcg<double>(phi, c->p, fixed ? c->fixed_inner : maxit, 0, &s, &have);
        if (e != hipSuccess) return hip_fail(e, "FP64 PCG");
        if (!have) {
            tpf_status st = read_scalars(c, &s);
            if (st != TPF_OK) return st;
        }
        if (!std::isfinite(s.ff) || !std::isfinite(s.rr)) {
            set_error("non-finite pressure right-hand side or residual");
            return TPF_ENONFINITE;
        }
        *iters = s.iters;
        *outer = 1;
        *relres = s.ff > 0 ? std::sqrt(s.rr / s.ff) : 0.0;
        if (!s.done && !fixed) {
            set_error("pressure solve did not converge within poisson_maxit iterations");
            return TPF_ENOCONV;
        }
        return TPF_OK;
    }
    // ---- mixed: FP64 defect correction around the FP32 multigrid-PCG
    double w1, w2;
    weights_of(c->dim, w1, w2);
    Solver<float, float, W> sv{c, c->dim, float(w1), float(w2)};
    Solver<float, double, W> s64{c, c->dim, 0.0};
    sv.build_betas(phi);
    const double rin = c->P.poisson_rtol_inner;
    int total = 0;
    // fixed-iteration mode: exactly fixed_outer passes of fixed_inner PCG
    // iterations, then one more residual for the reported relres
    const bool fixed = c->fixed_inner > 0;
    const int max_outer = fixed ? c->fixed_outer + 1 : 12;
    std::string trail;      // relative outer residual after each pass, for the failure message
    for (int o = 0; o < max_outer; ++o) {
        // FP64 residual, FP64 beta.  The first pass leaves out the rounding
        // floor: a start already at the floor costs one inner solve, after
        // which the next pass (with the floor) stops.
        if (o == 0)
            s64.template residual<float, false>(s64.coef_phi(phi), tp<float>(c->lv[0].r));
        else
            s64.template residual<float, true>(s64.coef_phi(phi), tp<float>(c->lv[0].r));
        (void)finalize3(c, (int)s64.nb0(), (int)s64.nb0(), (int)s64.nb0(), FIN_INIT, fixed ? 0.0 : rtol * rtol);
        // the inner solve aims straight at the outer tolerance (INNER_MARGIN of the
        // reduction it needs), but never below rin, the depth an FP32 PCG
        // reaches reliably; a further outer pass picks up the rest.  The
        // first pass (a converged start is rare) sets this up on the device
        // and reads the outer residual with the inner solve's scalars; later
        // passes read it first, to stop without another inner solve.
        if (o == 0) {
            k_inner_setup_first<<<1, 64, 0, c->stream>>>(c->scal, rtol, rin, fixed ? 1 : 0);
        } else {
            tpf_status st = read_scalars(c, &s);
            if (st != TPF_OK) return st;
            if (!std::isfinite(s.ff) || !std::isfinite(s.rr)) {
                set_error("non-finite pressure right-hand side or residual");
                return TPF_ENONFINITE;
            }
            if (s.done || (fixed && o == c->fixed_outer)) {
                *outer = o;
                *iters = total;
                *relres = s.ff > 0 ? std::sqrt(s.rr / s.ff) : 0.0;
                return TPF_OK;
            }
            char buf[48];
            std::snprintf(buf, sizeof(buf), " %.2e (floor %.1e)", s.ff > 0 ? std::sqrt(s.rr / s.ff) : 0.0,
                          s.ff > 0 ? std::sqrt(s.floor2 / s.ff) : 0.0);
            trail += buf;
            const double need = INNER_MARGIN * rtol * std::sqrt(s.ff / s.rr);
            const double tin = fixed ? 0.0 : std::min(0.1, std::max(rin, need));
            k_inner_setup<<<1, 64, 0, c->stream>>>(c->scal, tin * tin);
        }
        // the correction starts at zero through its first update (x_zero)
        bool have = false;
        e = sv.template pcg<float>(phi, tp<float>(c->ev), fixed ? c->fixed_inner : maxit, 1 + std::min(o, 2), &s, &have,
                                   true);
        if (e != hipSuccess) return hip_fail(e, "FP32 inner PCG");
        if (!have) {
            tpf_status st = read_scalars(c, &s);
            if (st != TPF_OK) return st;
        }
        if (s.iters < 0) {                 // decided by the outer residual of pass 0
            if (!std::isfinite(s.ff) || !std::isfinite(s.rr)) {
                set_error("non-finite pressure right-hand side or residual");
                return TPF_ENONFINITE;
            }
            *outer = 0;
            *iters = 0;
            *relres = s.ff > 0 ? std::sqrt(s.rr / s.ff) : 0.0;
            return TPF_OK;
        }
        total += s.iters;
        // an inner solve stopped by maxit (FP32 stagnation) still lowers the
        // A-norm error: its correction is applied and the outer loop goes on
        if (!std::isfinite(s.rr)) {
            set_error("non-finite inner pressure residual");
            return TPF_ENONFINITE;
        }
        // no update, no correction: the solve stopped before its first
        // update wrote the correction
        if (s.iters > 0) {
            prof_begin(c, PC_VECTOR, (double)c->N * (8 + 4 + 8));
            k_correct<<<vgrid(c->N), BLOCK, 0, c->stream>>>(c->N, c->p, tp<float>(c->ev));
            prof_end(c);
        }
    }
    set_error("pressure defect correction did not converge (relative residual after each pass:" + trail + ")");
    return TPF_ENOCONV;
}

tpf_status poisson_solve(tpf_ctx* c, const void* phi, int* iters, double* relres, int* outer) {
    return c->walls ? poisson_solve_t<true>(c, phi, iters, relres, outer)
                    : poisson_solve_t<false>(c, phi, iters, relres, outer);
}

}  // namespace tpf
