// Variable-density pressure Poisson solve, matrix free:
//     D(beta G p) = D f* - mean(D f*),   mean(p) = 0,   beta_a = 1 / A_a rho
// Conjugate gradients on the SPD form  A = -D(beta G .)  (zero-mean subspace),
// preconditioned by one geometric multigrid V-cycle (cell-centred coarsening
// by 2, rediscretised coarse operators with face-averaged beta, damped Jacobi
// smoothing, averaging restriction, piecewise-constant prolongation, fixed
// Jacobi sweeps on the coarsest grid in one workgroup).  Every piece of the
// V-cycle is a fixed linear symmetric operator, so it is a valid CG
// preconditioner.
//
// Mixed precision: the outer loop forms the residual in FP64 (FP64 beta from
// phi, FP64 right-hand side and iterate) and solves for the correction with
// the FP32 multigrid-PCG (defect correction).
//
// Scalars (alpha, beta, norms, the done flag) stay on the device; every
// solver kernel returns immediately once done is set, so the host queues
// several iterations between convergence checks.
#include <cmath>

#include "tpf_internal.hpp"

namespace tpf {

template <typename T>
static inline T* tp(void* p) { return static_cast<T*>(p); }

// ---------------------------------------------------------------- operator
// (A x)[c] = sum_a [beta_a[c](x[c]-x[c-e_a]) - beta_a[c+e_a](x[c+e_a]-x[c])] / h^2
template <typename S, int DIM>
__device__ __forceinline__ S apply_at(const Cell& C, const S* const* beta, const S* x, S ih2,
                                      S& diag) {
    const long c = C.id();
    const S xc = x[c];
    S acc = S(0), dg = S(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const long cp = C.off(a, 1), cm = C.off(a, -1);
        const S bl = beta[a][c], bh = beta[a][cp];
        acc += bl * (xc - x[cm]) - bh * (x[cp] - xc);
        dg += bl + bh;
    }
    diag = dg * ih2;
    return acc * ih2;
}

struct Betas {
    const void* b[3];
};

template <typename S>
struct BP {
    const S* b[3];
};
template <typename S>
__host__ __device__ inline BP<S> bp(const Betas& B) {
    return BP<S>{{static_cast<const S*>(B.b[0]), static_cast<const S*>(B.b[1]),
                  static_cast<const S*>(B.b[2])}};
}

// ---------------------------------------------------------------- coefficients
template <typename T, typename S, int DIM>
__global__ __launch_bounds__(BLOCK) void k_beta_fine(Dims d, Phys P, const T* __restrict__ phi,
                                                     S* b0, S* b1, S* b2) {
    Cell C;
    if (!cell_of_thread(d, C)) return;
    S* b[3] = {b0, b1, b2};
    const long c = C.id();
    const double f = (double)phi[c];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double fm = (double)phi[C.off(a, -1)];
        b[a][c] = S(1.0 / (0.5 * (rho_of(P, fm) + rho_of(P, f))));
    }
}

// coarse face coefficient = mean of the fine face coefficients it covers
template <typename S, int DIM>
__global__ __launch_bounds__(BLOCK) void k_beta_coarsen(Dims fd, Dims cd, Betas fine, S* b0, S* b1,
                                                        S* b2) {
    Cell C;
    if (!cell_of_thread(cd, C)) return;
    const BP<S> f = bp<S>(fine);
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
            s += f.b[a][fc];
        }
        b[a][C.id()] = s * S(1.0 / (1 << (DIM - 1)));
    }
}

// ---------------------------------------------------------------- residuals
// FP64 path: r = -(b - mean) - A x,  partials (|f|^2, |r|^2)
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_resid_init(Dims d, double ih2, Betas B,
                                                      const double* __restrict__ b,
                                                      const double* __restrict__ x,
                                                      double* __restrict__ r,
                                                      const SolverScalars* __restrict__ sc,
                                                      double* __restrict__ partials) {
    Cell C;
    double v[2] = {0.0, 0.0};
    if (cell_of_thread(d, C)) {
        const BP<double> bb = bp<double>(B);
        double dg;
        const long c = C.id();
        const double f = -(b[c] - sc->mean);
        const double rc = f - apply_at<double, DIM>(C, bb.b, x, ih2, dg);
        r[c] = rc;
        v[0] = f * f;
        v[1] = rc * rc;
    }
    block_partials<2>(v, partials);
}

// Mixed path outer residual in FP64 with beta recomputed from phi in FP64;
// the solver-precision copy goes to rs.
template <typename T, typename S, int DIM>
__global__ __launch_bounds__(BLOCK) void k_resid64(Dims d, Phys P, const T* __restrict__ phi,
                                                   const double* __restrict__ b,
                                                   const double* __restrict__ x,
                                                   S* __restrict__ rs,
                                                   const SolverScalars* __restrict__ sc,
                                                   double* __restrict__ partials) {
    Cell C;
    double v[2] = {0.0, 0.0};
    if (cell_of_thread(d, C)) {
        const long c = C.id();
        const double fc = (double)phi[c];
        const double xc = x[c];
        const double rho_c = rho_of(P, fc);
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const long cp = C.off(a, 1), cm = C.off(a, -1);
            const double bl = 1.0 / (0.5 * (rho_of(P, (double)phi[cm]) + rho_c));
            const double bh = 1.0 / (0.5 * (rho_c + rho_of(P, (double)phi[cp])));
            acc += bl * (xc - x[cm]) - bh * (x[cp] - xc);
        }
        const double f = -(b[c] - sc->mean);
        const double rc = f - acc * (P.inv_h * P.inv_h);
        rs[c] = S(rc);
        v[0] = f * f;
        v[1] = rc * rc;
    }
    block_partials<2>(v, partials);
}

// ---------------------------------------------------------------- smoothing
template <typename S, int DIM>
__global__ __launch_bounds__(BLOCK) void k_jacobi0(Dims d, S ih2, S omega, Betas B,
                                                   const S* __restrict__ r, S* __restrict__ z,
                                                   const SolverScalars* __restrict__ sc) {
    if (sc->done) return;
    Cell C;
    if (!cell_of_thread(d, C)) return;
    const BP<S> bb = bp<S>(B);
    const long c = C.id();
    S dg = S(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) dg += bb.b[a][c] + bb.b[a][C.off(a, 1)];
    z[c] = omega * r[c] / (dg * ih2);
}

template <typename S, int DIM>
__global__ __launch_bounds__(BLOCK) void k_jacobi(Dims d, S ih2, S omega, Betas B,
                                                  const S* __restrict__ r, const S* __restrict__ z,
                                                  S* __restrict__ zt,
                                                  const SolverScalars* __restrict__ sc) {
    if (sc->done) return;
    Cell C;
    if (!cell_of_thread(d, C)) return;
    const BP<S> bb = bp<S>(B);
    S dg;
    const S az = apply_at<S, DIM>(C, bb.b, z, ih2, dg);
    const long c = C.id();
    zt[c] = z[c] + omega * (r[c] - az) / dg;
}

// coarse rhs = mean over the children of (r - A z); one thread per coarse cell
template <typename S, int DIM>
__global__ __launch_bounds__(BLOCK) void k_restrict(Dims fd, Dims cd, S ih2, Betas B,
                                                    const S* __restrict__ r,
                                                    const S* __restrict__ z, S* __restrict__ rc,
                                                    const SolverScalars* __restrict__ sc) {
    if (sc->done) return;
    Cell Cc;
    if (!cell_of_thread(cd, Cc)) return;
    const BP<S> bb = bp<S>(B);
    S s = S(0);
    const int nk = DIM == 3 ? 2 : 1;
    for (int dk = 0; dk < nk; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
                Cell F{2 * Cc.i + di, 2 * Cc.j + dj, DIM == 3 ? 2 * Cc.k + dk : 0, fd.nx, fd.ny, fd.nz};
                S dg;
                s += r[F.id()] - apply_at<S, DIM>(F, bb.b, z, ih2, dg);
            }
    rc[Cc.id()] = s * S(1.0 / (DIM == 3 ? 8 : 4));
}

template <typename S, int DIM>
__global__ __launch_bounds__(BLOCK) void k_prolong(Dims fd, Dims cd, const S* __restrict__ zc,
                                                   S* __restrict__ z,
                                                   const SolverScalars* __restrict__ sc) {
    if (sc->done) return;
    Cell C;
    if (!cell_of_thread(fd, C)) return;
    const long pc = ((long)(DIM == 3 ? C.k >> 1 : 0) * cd.ny + (C.j >> 1)) * cd.nx + (C.i >> 1);
    z[C.id()] += zc[pc];
}

// coarsest grid: `sweeps` damped Jacobi sweeps from zero, one workgroup
template <typename S, int DIM>
__global__ __launch_bounds__(1024) void k_coarse(Dims d, S ih2, S omega, int sweeps, Betas B,
                                                 const S* __restrict__ r, S* z, S* zt,
                                                 const SolverScalars* __restrict__ sc) {
    if (sc->done) return;
    const BP<S> bb = bp<S>(B);
    const long N = (long)d.nx * d.ny * d.nz;
    for (long q = threadIdx.x; q < N; q += blockDim.x) z[q] = S(0);
    __syncthreads();
    S* src = z;
    S* dst = zt;
    for (int s = 0; s < sweeps; ++s) {
        for (long q = threadIdx.x; q < N; q += blockDim.x) {
            Cell C;
            C.i = (int)(q % d.nx);
            C.j = (int)((q / d.nx) % d.ny);
            C.k = (int)(q / ((long)d.nx * d.ny));
            C.nx = d.nx;
            C.ny = d.ny;
            C.nz = d.nz;
            S dg;
            const S az = apply_at<S, DIM>(C, bb.b, src, ih2, dg);
            dst[q] = src[q] + omega * (r[q] - az) / dg;
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

// ---------------------------------------------------------------- CG vector ops
template <typename S, int DIM>
__global__ __launch_bounds__(BLOCK) void k_apply_dot(Dims d, S ih2, Betas B,
                                                     const S* __restrict__ p, S* __restrict__ q,
                                                     const SolverScalars* __restrict__ sc,
                                                     double* __restrict__ partials) {
    if (sc->done) return;
    Cell C;
    double v[1] = {0.0};
    if (cell_of_thread(d, C)) {
        const BP<S> bb = bp<S>(B);
        S dg;
        const S aq = apply_at<S, DIM>(C, bb.b, p, ih2, dg);
        const long c = C.id();
        q[c] = aq;
        v[0] = (double)p[c] * (double)aq;
    }
    block_partials<1>(v, partials);
}

template <typename S, typename X>
__global__ __launch_bounds__(BLOCK) void k_update_xr(long N, X* __restrict__ x, S* __restrict__ r,
                                                     const S* __restrict__ p,
                                                     const S* __restrict__ q,
                                                     const SolverScalars* __restrict__ sc,
                                                     double* __restrict__ partials) {
    if (sc->done) return;
    const long c = (long)blockIdx.x * BLOCK + threadIdx.x;
    double v[1] = {0.0};
    if (c < N) {
        const double alpha = sc->alpha;
        x[c] = X((double)x[c] + alpha * (double)p[c]);
        const S rn = S((double)r[c] - alpha * (double)q[c]);
        r[c] = rn;
        v[0] = (double)rn * (double)rn;
    }
    block_partials<1>(v, partials);
}

template <typename S>
__global__ __launch_bounds__(BLOCK) void k_dot(long N, const S* __restrict__ a,
                                               const S* __restrict__ b,
                                               const SolverScalars* __restrict__ sc,
                                               double* __restrict__ partials) {
    if (sc->done) return;
    const long c = (long)blockIdx.x * BLOCK + threadIdx.x;
    double v[1] = {0.0};
    if (c < N) v[0] = (double)a[c] * (double)b[c];
    block_partials<1>(v, partials);
}

template <typename S>
__global__ __launch_bounds__(BLOCK) void k_update_p(long N, int first, const S* __restrict__ z,
                                                    S* __restrict__ p,
                                                    const SolverScalars* __restrict__ sc) {
    if (sc->done) return;
    const long c = (long)blockIdx.x * BLOCK + threadIdx.x;
    if (c >= N) return;
    p[c] = first ? z[c] : S((double)z[c] + sc->beta * (double)p[c]);
}

template <typename S>
__global__ void k_fill_s(long N, S* __restrict__ x, S v) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < N) x[c] = v;
}

__global__ __launch_bounds__(BLOCK) void k_correct(long N, double* __restrict__ x,
                                                   const float* __restrict__ e) {
    const long c = (long)blockIdx.x * BLOCK + threadIdx.x;
    if (c < N) x[c] += (double)e[c];
}

__global__ __launch_bounds__(BLOCK) void k_sum(long N, const double* __restrict__ x,
                                               double* __restrict__ partials) {
    const long c = (long)blockIdx.x * BLOCK + threadIdx.x;
    double v[1] = {c < N ? x[c] : 0.0};
    block_partials<1>(v, partials);
}

__global__ __launch_bounds__(BLOCK) void k_sub_mean(long N, double* __restrict__ x,
                                                    const SolverScalars* __restrict__ sc) {
    const long c = (long)blockIdx.x * BLOCK + threadIdx.x;
    if (c < N) x[c] -= sc->sum / (double)N;
}

// ---------------------------------------------------------------- finalize
__global__ __launch_bounds__(BLOCK) void k_finalize(int nb, int nv, int op, double arg, long N,
                                                    const double* __restrict__ partials,
                                                    SolverScalars* sc) {
    const bool skip = (op == FIN_ALPHA || op == FIN_BETA || op == FIN_RZ0) && sc->done;
    if (skip) return;
    double v[2] = {0.0, 0.0};
    for (int b = thread_linear(); b < nb; b += BLOCK) {
        v[0] += partials[b];
        if (nv > 1) v[1] += partials[(long)nb + b];
    }
    block_sum<2>(v);
    if (thread_linear() != 0) return;
    switch (op) {
    case FIN_MEAN:
        sc->mean = v[0] / (double)N;
        break;
    case FIN_INIT:
        sc->ff = v[0];
        sc->rr = v[1];
        sc->tol2 = arg;
        sc->iters = 0;
        sc->done = (v[0] == 0.0 || v[1] <= arg * v[0]) ? 1 : 0;
        break;
    case FIN_RZ0:
        sc->rz = v[0];
        if (!(v[0] > 0.0)) sc->done = 1;
        break;
    case FIN_ALPHA:
        sc->pq = v[0];
        sc->alpha = (v[0] > 0.0) ? sc->rz / v[0] : 0.0;
        if (!(v[0] > 0.0)) sc->done = 1;
        break;
    case FIN_BETA:
        sc->rr = v[0];
        sc->beta = v[1] / sc->rz;
        sc->rz = v[1];
        sc->iters += 1;
        if (v[0] <= sc->tol2 * sc->ff || !(v[1] > 0.0)) sc->done = 1;
        break;
    case FIN_SUM:
        sc->sum = v[0];
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

hipError_t launch_finalize(tpf_ctx* c, int nblocks, int nv, int op) {
    prof_begin(c, PC_FINALIZE, (double)nblocks * nv * 8);
    k_finalize<<<1, BLOCK, 0, c->stream>>>(nblocks, nv, op, 0.0, c->N, c->partials, c->scal);
    prof_end(c);
    return hipGetLastError();
}

// ================================================================== host driver

template <typename S>
struct Solver {
    tpf_ctx* c;
    int dim;
    S omega;
    int nu;  // pre = post smoothing sweeps

    Betas betas(int l) const {
        return Betas{{c->lv[l].beta[0], c->lv[l].beta[1], c->lv[l].beta[2]}};
    }
    S ih2(int l) const { return S(1.0 / (c->lv[l].h * c->lv[l].h)); }
    dim3 grid(int l) const { return grid_of(c->lv[l].n); }
    Dims dims(int l) const { return dims_of(c->lv[l].n); }
    double lbytes(int l, int fields) const { return (double)c->lv[l].N * sizeof(S) * fields; }

    template <int DIM>
    void build_betas_t(const void* phi) {
        const Phys P = phys_of(c);
        const dim3 b(BX, BY);
        if (c->mixed)
            k_beta_fine<float, S, DIM><<<grid(0), b, 0, c->stream>>>(
                dims(0), P, static_cast<const float*>(phi), tp<S>(c->lv[0].beta[0]),
                tp<S>(c->lv[0].beta[1]), tp<S>(c->lv[0].beta[2]));
        else
            k_beta_fine<double, S, DIM><<<grid(0), b, 0, c->stream>>>(
                dims(0), P, static_cast<const double*>(phi), tp<S>(c->lv[0].beta[0]),
                tp<S>(c->lv[0].beta[1]), tp<S>(c->lv[0].beta[2]));
        for (int l = 1; l < c->nlev; ++l)
            k_beta_coarsen<S, DIM><<<grid(l), b, 0, c->stream>>>(
                dims(l - 1), dims(l), betas(l - 1), tp<S>(c->lv[l].beta[0]),
                tp<S>(c->lv[l].beta[1]), tp<S>(c->lv[l].beta[2]));
    }
    void build_betas(const void* phi) {
        if (dim == 2) build_betas_t<2>(phi); else build_betas_t<3>(phi);
    }

    // z_l ~= A_l^{-1} r_l ; returns the buffer holding the result
    template <int DIM>
    S* vcycle_t(int l) {
        Level& L = c->lv[l];
        const dim3 b(BX, BY);
        const int fine = (l == 0);
        S* z = tp<S>(L.z);
        S* zt = tp<S>(L.zt);
        const S* r = tp<S>(L.r);
        if (l == c->nlev - 1) {
            const int mx = L.n[0] > L.n[1] ? L.n[0] : L.n[1];
            const int sweeps = 8 * (mx > L.n[2] ? mx : L.n[2]);
            prof_begin(c, PC_COARSE_LEVELS, lbytes(l, 3));
            k_coarse<S, DIM><<<1, 1024, 0, c->stream>>>(dims(l), ih2(l), S(0.8), sweeps, betas(l), r,
                                                        z, zt, c->scal);
            prof_end(c);
            return z;
        }
        const int cls_j = fine ? PC_JACOBI_FINE : PC_COARSE_LEVELS;
        prof_begin(c, cls_j, lbytes(l, 2 + DIM));
        k_jacobi0<S, DIM><<<grid(l), b, 0, c->stream>>>(dims(l), ih2(l), omega, betas(l), r, z, c->scal);
        prof_end(c);
        for (int s = 1; s < nu; ++s) {
            prof_begin(c, cls_j, lbytes(l, 3 + DIM));
            k_jacobi<S, DIM><<<grid(l), b, 0, c->stream>>>(dims(l), ih2(l), omega, betas(l), r, z, zt, c->scal);
            prof_end(c);
            S* t = z; z = zt; zt = t;
        }
        Level& Lc = c->lv[l + 1];
        prof_begin(c, fine ? PC_RESTRICT_FINE : PC_COARSE_LEVELS,
                   lbytes(l, 2 + DIM) + (double)Lc.N * sizeof(S));
        k_restrict<S, DIM><<<grid(l + 1), b, 0, c->stream>>>(dims(l), dims(l + 1), ih2(l), betas(l), r,
                                                             z, tp<S>(Lc.r), c->scal);
        prof_end(c);
        S* zc = vcycle_t<DIM>(l + 1);
        prof_begin(c, fine ? PC_PROLONG_FINE : PC_COARSE_LEVELS, lbytes(l, 2) + (double)Lc.N * sizeof(S));
        k_prolong<S, DIM><<<grid(l), b, 0, c->stream>>>(dims(l), dims(l + 1), zc, z, c->scal);
        prof_end(c);
        for (int s = 0; s < nu; ++s) {
            prof_begin(c, cls_j, lbytes(l, 3 + DIM));
            k_jacobi<S, DIM><<<grid(l), b, 0, c->stream>>>(dims(l), ih2(l), omega, betas(l), r, z, zt, c->scal);
            prof_end(c);
            S* t = z; z = zt; zt = t;
        }
        return z;
    }
    S* vcycle() { return dim == 2 ? vcycle_t<2>(0) : vcycle_t<3>(0); }

    unsigned vblocks() const { return (unsigned)((c->N + BLOCK - 1) / BLOCK); }

    // PCG on level 0 for x (type X), residual already in lv[0].r and the
    // scalars initialised (ff, rr, tol2, done).  Returns hip error.
    template <typename X>
    hipError_t pcg(X* x, int maxit, int check_every) {
        const long N = c->N;
        const unsigned nbv = vblocks();
        S* r = tp<S>(c->lv[0].r);
        S* p = tp<S>(c->pv);
        S* q = tp<S>(c->qv);
        const double vb = (double)N * sizeof(S);
        S* z = vcycle();
        prof_begin(c, PC_VEC_FINE, 2 * vb);
        k_dot<S><<<nbv, BLOCK, 0, c->stream>>>(N, r, z, c->scal, c->partials);
        prof_end(c);
        (void)launch_finalize(c, (int)nbv, 1, FIN_RZ0);
        prof_begin(c, PC_VEC_FINE, 2 * vb);
        k_update_p<S><<<nbv, BLOCK, 0, c->stream>>>(N, 1, z, p, c->scal);
        prof_end(c);
        const int nb_apply = (int)nblocks_of(c->n);
        int it = 0;
        while (it < maxit) {
            for (int k = 0; k < check_every && it < maxit; ++k, ++it) {
                prof_begin(c, PC_APPLY_FINE, vb * (2 + dim));
                if (dim == 2)
                    k_apply_dot<S, 2><<<grid(0), dim3(BX, BY), 0, c->stream>>>(dims(0), ih2(0), betas(0), p, q, c->scal, c->partials);
                else
                    k_apply_dot<S, 3><<<grid(0), dim3(BX, BY), 0, c->stream>>>(dims(0), ih2(0), betas(0), p, q, c->scal, c->partials);
                prof_end(c);
                (void)launch_finalize(c, nb_apply, 1, FIN_ALPHA);
                prof_begin(c, PC_VEC_FINE, 4 * vb + 2.0 * N * sizeof(X));
                k_update_xr<S, X><<<nbv, BLOCK, 0, c->stream>>>(N, x, r, p, q, c->scal, c->partials);
                prof_end(c);
                z = vcycle();
                prof_begin(c, PC_VEC_FINE, 2 * vb);
                k_dot<S><<<nbv, BLOCK, 0, c->stream>>>(N, r, z, c->scal, c->partials + nbv);
                prof_end(c);
                (void)launch_finalize(c, (int)nbv, 2, FIN_BETA);
                prof_begin(c, PC_VEC_FINE, 3 * vb);
                k_update_p<S><<<nbv, BLOCK, 0, c->stream>>>(N, 0, z, p, c->scal);
                prof_end(c);
            }
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            int done = 0;
            e = hipMemcpyAsync(&done, &c->scal->done, sizeof(int), hipMemcpyDeviceToHost, c->stream);
            if (e != hipSuccess) return e;
            e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) return e;
            if (done) break;
        }
        return hipGetLastError();
    }
};

hipError_t launch_rhs_mean(tpf_ctx* c) {
    const unsigned nb = (unsigned)((c->N + BLOCK - 1) / BLOCK);
    k_sum<<<nb, BLOCK, 0, c->stream>>>(c->N, c->b, c->partials);
    return launch_finalize(c, (int)nb, 1, FIN_MEAN);
}

static hipError_t remove_mean(tpf_ctx* c, double* x) {
    const unsigned nb = (unsigned)((c->N + BLOCK - 1) / BLOCK);
    k_sum<<<nb, BLOCK, 0, c->stream>>>(c->N, x, c->partials);
    hipError_t e = launch_finalize(c, (int)nb, 1, FIN_SUM);
    if (e != hipSuccess) return e;
    k_sub_mean<<<nb, BLOCK, 0, c->stream>>>(c->N, x, c->scal);
    return hipGetLastError();
}

static tpf_status read_scalars(tpf_ctx* c, SolverScalars* s) {
    hipError_t e = hipMemcpyAsync(s, c->scal, sizeof(SolverScalars), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "reading solver scalars");
    return TPF_OK;
}

// Solve with beta from phi (state precision); right-hand side in c->b with
// its mean in scal->mean; x = c->p (warm start in, solution out, zero mean).
tpf_status poisson_solve(tpf_ctx* c, const void* phi, int* iters, double* relres, int* outer) {
    const double rtol = c->P.poisson_rtol;
    const int maxit = c->P.poisson_maxit;
    const int check = 4;
    SolverScalars s;
    hipError_t e;
    if (!c->mixed) {
        Solver<double> sv{c, c->dim, c->dim == 2 ? 0.8 : 6.0 / 7.0, 2};
        sv.build_betas(phi);
        prof_begin(c, PC_VEC_FINE, (double)c->N * 8 * (3 + c->dim));
        if (c->dim == 2)
            k_resid_init<2><<<grid_of(c->n), dim3(BX, BY), 0, c->stream>>>(
                dims_of(c->n), 1.0 / (c->h * c->h), sv.betas(0), c->b, c->p,
                tp<double>(c->lv[0].r), c->scal, c->partials);
        else
            k_resid_init<3><<<grid_of(c->n), dim3(BX, BY), 0, c->stream>>>(
                dims_of(c->n), 1.0 / (c->h * c->h), sv.betas(0), c->b, c->p,
                tp<double>(c->lv[0].r), c->scal, c->partials);
        prof_end(c);
        k_finalize<<<1, BLOCK, 0, c->stream>>>((int)nblocks_of(c->n), 2, FIN_INIT, rtol * rtol, c->N,
                                               c->partials, c->scal);
        e = sv.pcg<double>(c->p, maxit, check);
        if (e != hipSuccess) return hip_fail(e, "FP64 PCG");
        e = remove_mean(c, c->p);
        if (e != hipSuccess) return hip_fail(e, "mean removal");
        tpf_status st = read_scalars(c, &s);
        if (st != TPF_OK) return st;
        if (!std::isfinite(s.ff) || !std::isfinite(s.rr)) {
            set_error("non-finite pressure right-hand side or residual");
            return TPF_ENONFINITE;
        }
        *iters = s.iters;
        *outer = 1;
        *relres = s.ff > 0 ? std::sqrt(s.rr / s.ff) : 0.0;
        if (!s.done) {
            set_error("pressure solve did not converge within poisson_maxit iterations");
            return TPF_ENOCONV;
        }
        return TPF_OK;
    }
    // ---- mixed: FP64 defect correction around the FP32 multigrid-PCG
    Solver<float> sv{c, c->dim, float(c->dim == 2 ? 0.8 : 6.0 / 7.0), 2};
    sv.build_betas(phi);
    const double rin = c->P.poisson_rtol_inner;
    int total = 0;
    const int max_outer = 12;
    for (int o = 0; o < max_outer; ++o) {
        prof_begin(c, PC_RESID64, (double)c->N * (4 + 8 + 8 + 4));
        if (c->dim == 2)
            k_resid64<float, float, 2><<<grid_of(c->n), dim3(BX, BY), 0, c->stream>>>(
                dims_of(c->n), phys_of(c), static_cast<const float*>(phi), c->b, c->p,
                tp<float>(c->lv[0].r), c->scal, c->partials);
        else
            k_resid64<float, float, 3><<<grid_of(c->n), dim3(BX, BY), 0, c->stream>>>(
                dims_of(c->n), phys_of(c), static_cast<const float*>(phi), c->b, c->p,
                tp<float>(c->lv[0].r), c->scal, c->partials);
        prof_end(c);
        k_finalize<<<1, BLOCK, 0, c->stream>>>((int)nblocks_of(c->n), 2, FIN_INIT, rtol * rtol, c->N,
                                               c->partials, c->scal);
        tpf_status st = read_scalars(c, &s);
        if (st != TPF_OK) return st;
        if (!std::isfinite(s.ff) || !std::isfinite(s.rr)) {
            set_error("non-finite pressure right-hand side or residual");
            return TPF_ENONFINITE;
        }
        if (s.done) {
            *outer = o;
            *iters = total;
            *relres = s.ff > 0 ? std::sqrt(s.rr / s.ff) : 0.0;
            e = remove_mean(c, c->p);
            if (e != hipSuccess) return hip_fail(e, "mean removal");
            return TPF_OK;
        }
        k_inner_setup<<<1, 64, 0, c->stream>>>(c->scal, rin * rin);
        k_fill_s<float><<<(unsigned)((c->N + 255) / 256), 256, 0, c->stream>>>(c->N, tp<float>(c->ev), 0.0f);
        e = sv.pcg<float>(tp<float>(c->ev), maxit, check);
        if (e != hipSuccess) return hip_fail(e, "FP32 inner PCG");
        st = read_scalars(c, &s);
        if (st != TPF_OK) return st;
        total += s.iters;
        if (!s.done) {
            set_error("inner pressure solve did not converge within poisson_maxit iterations");
            return TPF_ENOCONV;
        }
        prof_begin(c, PC_VEC_FINE, (double)c->N * (8 + 4 + 8));
        k_correct<<<(unsigned)((c->N + BLOCK - 1) / BLOCK), BLOCK, 0, c->stream>>>(c->N, c->p, tp<float>(c->ev));
        prof_end(c);
    }
    set_error("pressure defect correction did not converge");
    return TPF_ENOCONV;
}

}  // namespace tpf
