// Batched persistent form of the step: many independent 2D cases, one
// workgroup per case for the whole RK4 step, one launch per step.
//
// Every stage operator of a case runs as a block-stride loop over the case's
// cells (64 consecutive x cells per wave, coalesced), separated by workgroup
// barriers; the pressure solve is the same multigrid-preconditioned CG as the
// single-case path (damped Jacobi, two sweeps before and after, averaging
// restriction, piecewise-constant prolongation, fixed Jacobi sweeps on the
// coarsest grid) with every reduction a workgroup reduction.  Nothing is
// shared between cases, so a case converges, fails or finishes on its own:
// there is no host synchronisation inside a step.  The coarsest multigrid
// levels of each case live in LDS.
//
// A case may close either axis with free-slip walls.  The stage operators
// read across them by the mirror rules of the operator bodies (the level-0
// cells carry wall bits); the pressure operator is closed by zero face
// coefficients on the wall faces of every level (a coarse wall face is the
// mean of two zero fine faces), so the periodic neighbour a solver kernel
// reads across a wall is multiplied by zero and the multigrid, the CG and
// the gauge run unchanged.
#pragma once
#include <limits>

#include "tpf_internal.hpp"

namespace tpf {

constexpr int BMAXLEV = 10;

// One case of a batch: grid, physics and the addresses of its fields.
struct BCase {
    Phys P;
    int nx, ny, nlev, maxit;
    int walls;          // bit a: free-slip walls at both ends of axis a
    int need_mu, need_kappa, lds_first, lds_bytes;
    double rtol, rtol_inner;
    void* y[4][3];      // state slots: phi, u_x, u_y
    void* nrm[2];
    void* rflux[2];
    void* mflux[2];
    void* fs[2];
    void* mu;
    void* kappa;
    double* b;
    double* p;          // pressure (solution and warm start), FP64
    double* ph[3];      // pressure history for the warm starts (as the single-case step)
    void* pv;           // CG directions (solver precision), two buffers used in turn
    void* pv2;
    void* qv;           // A p
    void* ev;           // mixed: inner solution (correction)
    void* lb[BMAXLEV][2];   // face coefficients per level (global)
    void* lz[BMAXLEV];
    void* lzt[BMAXLEV];
    void* lr[BMAXLEV];
    int ln[BMAXLEV][2];
    int lds_off[BMAXLEV];   // element offsets of LDS-resident levels (r, z, zt, b0, b1)
    double lh[BMAXLEV];     // grid spacing per level
};

// Per-case status and bookkeeping, device resident.
struct BState {
    int yn, acc;        // slots holding y_n and the RK accumulator
    int status;         // TPF_OK, or the failure that froze the case
    int nonfinite;      // set by the stage ops when a non-finite value appears
    int iters, outer;   // last pressure solve
    int fails, hist_valid;   // hist_valid: the pressure history is from a completed step
    double t;
    double relres;      // last pressure solve
    long long step;
    double mass0;
    long long solves, outer_total, inner_total;   // pressure solves and their iterations since the last reset
};

// ------------------------------------------------------------------ reductions
template <int NT>
__device__ __forceinline__ double bsum(double x, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    const int t = threadIdx.x;
    if ((t & 63) == 0) red[t >> 6] = x;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}

template <int NT>
__device__ __forceinline__ void bsum2(double& x, double& y, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        x += __shfl_down(x, o, 64);
        y += __shfl_down(y, o, 64);
    }
    const int t = threadIdx.x;
    if ((t & 63) == 0) {
        red[t >> 6] = x;
        red[NT / 64 + (t >> 6)] = y;
    }
    __syncthreads();
    double s = 0.0, u = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        s += red[w];
        u += red[NT / 64 + w];
    }
    __syncthreads();
    x = s;
    y = u;
}

// ------------------------------------------------------------------ levels
// two-element vector of S (an aligned pair of x neighbours)
template <typename S>
struct BVec2;
template <>
struct BVec2<float> { using type = float2; };
template <>
struct BVec2<double> { using type = double2; };

template <typename S>
struct BLev {
    Dims d;
    S ih2;
    const S* b0;
    const S* b1;
    S* z;
    S* zt;
    S* r;
};

// (A x)[c] with face coefficients b0, b1 (A = -D beta G, positive
// semidefinite) and the diagonal.
template <typename S>
__device__ __forceinline__ S bapply(const BLev<S>& L, const Cell& C, const S* x, S& dg) {
    const unsigned c = C.id;
    const S bl0 = L.b0[c], bh0 = L.b0[C.nb(0, 1)];
    const S bl1 = L.b1[c], bh1 = L.b1[C.nb(1, 1)];
    const S xc = x[c];
    const S acc = bl0 * (xc - x[C.nb(0, -1)]) - bh0 * (x[C.nb(0, 1)] - xc) +
                  bl1 * (xc - x[C.nb(1, -1)]) - bh1 * (x[C.nb(1, 1)] - xc);
    dg = (bl0 + bh0 + bl1 + bh1) * L.ih2;
    return acc * L.ih2;
}

// The operands of (A x)[c]: x at c and its four neighbours, the face
// coefficients of c's four faces.  Loaded apart from the arithmetic so that
// a thread can have the loads of several cells in flight (BatchBlock::cells_g).
template <typename S>
struct Stencil {
    S xc, xw, xe, xs, xn, bl0, bh0, bl1, bh1;
    __device__ __forceinline__ void load(const BLev<S>& L, const Cell& C, const S* x) {
        const unsigned c = C.id;
        bl0 = L.b0[c];
        bh0 = L.b0[C.nb(0, 1)];
        bl1 = L.b1[c];
        bh1 = L.b1[C.nb(1, 1)];
        xc = x[c];
        xw = x[C.nb(0, -1)];
        xe = x[C.nb(0, 1)];
        xs = x[C.nb(1, -1)];
        xn = x[C.nb(1, 1)];
    }
    // the arithmetic of bapply, term for term
    __device__ __forceinline__ S apply(S ih2, S& dg) const {
        const S acc = bl0 * (xc - xw) - bh0 * (xe - xc) + bl1 * (xc - xs) - bh1 * (xn - xc);
        dg = (bl0 + bh0 + bl1 + bh1) * ih2;
        return acc * ih2;
    }
};

// W: some case of the batch has walls (the kernel variant that reads wall
// bits; without it every wall test folds away at compile time)
template <typename T, typename S, int NT, bool W>
struct BatchBlock {
    const BCase& K;
    BState* st;
    double* red;
    S* lds;

    // the cells of a (nx, ny) grid, 64 consecutive x per wave (with the
    // wall bits of d)
    template <typename F>
    __device__ __forceinline__ void cells(const Dims& d, F f) const {
        for (int j = threadIdx.x / 64; j < d.ny; j += NT / 64)
            for (int i = threadIdx.x % 64; i < d.nx; i += 64) f(make_cell_w(d, i, j, 0));
    }

    // The same cells, visited in groups of UG: f(C, on) gets the group's UG
    // cells (on[u] false past the grid) and reads the operands of all of them
    // before it computes and stores any, so one thread has UG cells' loads in
    // flight at once instead of one.  A workgroup owns a whole case, and at
    // 36 cells per thread on a 192^2 grid the one-cell-at-a-time loop waits
    // out one memory latency per cell.  The visiting order (and so the order
    // of every per-thread sum) is that of cells().
    static constexpr int UG = 4;
    template <int U = UG, typename F>
    __device__ __forceinline__ void cells_g(const Dims& d, F f) const {
        const int gx = (d.nx + 63) / 64;
        const int j0 = threadIdx.x / 64, i0 = threadIdx.x % 64;
        const int rows = j0 < d.ny ? (d.ny - j0 + NT / 64 - 1) / (NT / 64) : 0;
        const int nt = gx * rows;
        for (int t0 = 0; t0 < nt; t0 += U) {
            Cell C[U];
            bool on[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + u;
                const int jj = t / gx;
                const int i = (t - jj * gx) * 64 + i0, j = j0 + jj * (NT / 64);
                on[u] = t < nt && i < d.nx;
                C[u] = make_cell_w(d, on[u] ? i : 0, on[u] ? j : 0, 0);
            }
            f(C, on);
        }
    }

    // level l; level 0 carries the case's walls (the coarse levels need none:
    // their solver kernels read periodic neighbours only)
    __device__ __forceinline__ Dims dims(int l) const {
        return Dims{K.ln[l][0], K.ln[l][1], 1, 0, (W && l == 0) ? K.walls : 0};
    }
    __device__ __forceinline__ int ncell(int l) const { return K.ln[l][0] * K.ln[l][1]; }

    __device__ __forceinline__ BLev<S> lev(int l) const {
        BLev<S> L;
        L.d = dims(l);
        L.ih2 = S(1.0 / (K.lh[l] * K.lh[l]));
        if (l >= K.lds_first) {
            const int N = ncell(l);
            S* base = lds + K.lds_off[l];
            L.r = base;
            L.z = base + N;
            L.zt = base + 2 * N;
            L.b0 = base + 3 * N;
            L.b1 = base + 4 * N;
        } else {
            L.r = static_cast<S*>(K.lr[l]);
            L.z = static_cast<S*>(K.lz[l]);
            L.zt = static_cast<S*>(K.lzt[l]);
            L.b0 = static_cast<const S*>(K.lb[l][0]);
            L.b1 = static_cast<const S*>(K.lb[l][1]);
        }
        return L;
    }

    // ---------------------------------------------------------- coefficients
    // fine level: beta_a = 1 / (h(c - e_a) + h(c)), h = rho(phi) / 2 with the
    // clamped linear law, and 0 on wall faces; coarser levels: mean of the
    // two fine faces covering each coarse face.  Then the LDS-resident levels
    // receive their copies.
    __device__ void build_betas(const T* phi) {
        const Phys& P = K.P;
        const S h2 = S(0.5 * P.rho2), dh = S(0.5 * (P.rho1 - P.rho2));
        const S lo = P.clamp ? S(0) : -std::numeric_limits<S>::infinity();
        const S hi = P.clamp ? S(1) : std::numeric_limits<S>::infinity();
        S* b0 = static_cast<S*>(K.lb[0][0]);
        S* b1 = static_cast<S*>(K.lb[0][1]);
        cells(dims(0), [&](const Cell& C) {
            auto hr = [&](unsigned q) { return h2 + dh * med3(S(phi[q]), lo, hi); };
            const S hc = hr(C.id);
            b0[C.id] = C.wall(0, -1) ? S(0) : S(1) / (hr(C.nb(0, -1)) + hc);
            b1[C.id] = C.wall(1, -1) ? S(0) : S(1) / (hr(C.nb(1, -1)) + hc);
        });
        __syncthreads();
        for (int l = 1; l < K.nlev; ++l) {
            const Dims fd = dims(l - 1);
            const S* f0 = static_cast<const S*>(K.lb[l - 1][0]);
            const S* f1 = static_cast<const S*>(K.lb[l - 1][1]);
            S* c0 = static_cast<S*>(K.lb[l][0]);
            S* c1 = static_cast<S*>(K.lb[l][1]);
            cells(dims(l), [&](const Cell& C) {
                const int i0 = 2 * C.i, j0 = 2 * C.j;
                // x faces: fine faces (i0, j0), (i0, j0+1); y faces: (i0, j0), (i0+1, j0)
                c0[C.id] = S(0.5) * (f0[j0 * fd.nx + i0] + f0[(j0 + 1) * fd.nx + i0]);
                c1[C.id] = S(0.5) * (f1[j0 * fd.nx + i0] + f1[j0 * fd.nx + i0 + 1]);
            });
            __syncthreads();
        }
        for (int l = K.lds_first; l < K.nlev; ++l) {
            const BLev<S> L = lev(l);
            const int N = ncell(l);
            const S* g0 = static_cast<const S*>(K.lb[l][0]);
            const S* g1 = static_cast<const S*>(K.lb[l][1]);
            for (int q = threadIdx.x; q < N; q += NT) {
                const_cast<S*>(L.b0)[q] = g0[q];
                const_cast<S*>(L.b1)[q] = g1[q];
            }
        }
        __syncthreads();
    }

    // dst = src + omega (r - A src) / d on level L (one damped Jacobi sweep)
    // (dot: also sum <r, dst> over the thread's cells into *dot; up: also add
    // each new value to the four children in up->zt, the piecewise-constant
    // prolongation into the finer level, whose sizes are twice L's)
    __device__ __forceinline__ void jacobi(const BLev<S>& L, const S* src, S* dst, S omega,
                                           double* dot = nullptr, const BLev<S>* up = nullptr) const {
        cells_g(L.d, [&](const Cell* C, const bool* on) {
            Stencil<S> v[UG];
            S r[UG], zn[UG];
#pragma unroll
            for (int u = 0; u < UG; ++u)
                if (on[u]) {
                    v[u].load(L, C[u], src);
                    r[u] = L.r[C[u].id];
                }
#pragma unroll
            for (int u = 0; u < UG; ++u)
                if (on[u]) {
                    S dg;
                    const S az = v[u].apply(L.ih2, dg);
                    zn[u] = v[u].xc + omega * (r[u] - az) / dg;
                    dst[C[u].id] = zn[u];
                    if (dot) *dot += (double)r[u] * (double)zn[u];
                }
            if (up) prolong_children(*up, C, on, zn);
        });
    }

    // up->zt += the coarse value zn of each of the group's cells, at its
    // four children (disjoint between coarse cells; coarsening keeps every
    // level's sizes even, so all four exist and each pair of x children is
    // one aligned two-element vector)
    __device__ __forceinline__ void prolong_children(const BLev<S>& F, const Cell* C, const bool* on,
                                                     const S* zn) const {
        using V2 = typename BVec2<S>::type;
        const int fx = F.d.nx;
#pragma unroll
        for (int u = 0; u < UG; ++u)
            if (on[u]) {
                V2* lo = reinterpret_cast<V2*>(F.zt + (2 * C[u].j) * fx + 2 * C[u].i);
                V2* hi = reinterpret_cast<V2*>(F.zt + (2 * C[u].j + 1) * fx + 2 * C[u].i);
                V2 a = *lo, b = *hi;
                a.x = a.x + zn[u];
                a.y = a.y + zn[u];
                b.x = b.x + zn[u];
                b.y = b.y + zn[u];
                *lo = a;
                *hi = b;
            }
    }

    // ---------------------------------------------------------- coarsest grid
    // The same damped Jacobi sweeps from zero as the workgroup loop, for a
    // coarsest grid of at most 64 cells: the first wave holds it, one cell
    // per lane, and each sweep reads the four neighbours' values from their
    // lanes (cross-lane permutes), so the sweeps need no workgroup barrier.
    // Lanes past the grid mirror cell 0 and write nothing.  Result in zt.
    // up: also add the result to its four children in up->zt (as jacobi does)
    __device__ __forceinline__ void coarsest_in_wave(const BLev<S>& L, int N, int sweeps, S wc,
                                                     const BLev<S>* up = nullptr) const {
        if (threadIdx.x >= 64) return;
        const int lane = threadIdx.x;
        const int q = lane < N ? lane : 0;
        const Cell C = make_cell(L.d, q % L.d.nx, q / L.d.nx, 0);
        const S bl0 = L.b0[q], bh0 = L.b0[C.nb(0, 1)];
        const S bl1 = L.b1[q], bh1 = L.b1[C.nb(1, 1)];
        const S r = L.r[q];
        const S dg = (bl0 + bh0 + bl1 + bh1) * L.ih2;
        const int lw = (int)C.nb(0, -1), le = (int)C.nb(0, 1), ls = (int)C.nb(1, -1), ln = (int)C.nb(1, 1);
        S z = S(0);
        for (int s = 0; s < sweeps; ++s) {
            const S zw = __shfl(z, lw, 64), ze = __shfl(z, le, 64);
            const S zs = __shfl(z, ls, 64), zn = __shfl(z, ln, 64);
            const S az = (bl0 * (z - zw) - bh0 * (ze - z) + bl1 * (z - zs) - bh1 * (zn - z)) * L.ih2;
            z = z + wc * (r - az) / dg;
        }
        if (lane < N) {
            L.zt[q] = z;
            if (up) {
                const int fx = up->d.nx;
                const unsigned f = (unsigned)((2 * C.j) * fx + 2 * C.i);
                up->zt[f] = up->zt[f] + z;
                up->zt[f + 1] = up->zt[f + 1] + z;
                up->zt[f + fx] = up->zt[f + fx] + z;
                up->zt[f + fx + 1] = up->zt[f + fx + 1] + z;
            }
        }
    }

    // ---------------------------------------------------------- V-cycle
    // z = M r on level 0 (r in lev(0).r); the result ends in lev(0).zt.
    // Returns <r, zt> of level 0 (summed by the last sweep, per thread in cell
    // order, then over the workgroup).
    // z_ready: z = omega r / d of level 0 was formed by the PCG update pass
    __device__ __forceinline__ double vcycle(S omega, bool z_ready = false) {
        const int nl = K.nlev;
        if (nl == 1) {
            const BLev<S> L = lev(0);
            cells(L.d, [&](const Cell& C) {
                S dg;
                (void)bapply(L, C, L.r, dg);   // diagonal only
                L.z[C.id] = omega * L.r[C.id] / dg;
            });
            __syncthreads();
            cells(L.d, [&](const Cell& C) {
                S dg;
                const S az = bapply(L, C, L.z, dg);
                L.zt[C.id] = L.z[C.id] + omega * (L.r[C.id] - az) / dg;
            });
            __syncthreads();
            double rz = 0.0;
            cells(L.d, [&](const Cell& C) { rz += (double)L.r[C.id] * (double)L.zt[C.id]; });
            return bsum<NT>(rz, red);
        }
        for (int l = 0; l + 1 < nl; ++l) {
            const BLev<S> L = lev(l);
            // the first sweep from zero: on level 0 here (unless the PCG update
            // pass formed it), on the coarser levels in the restriction above
            if (l == 0 && !z_ready) {
            cells_g(L.d, [&](const Cell* C, const bool* on) {      // z = omega r / d
                S b0l[UG], b0h[UG], b1l[UG], b1h[UG], r[UG];
#pragma unroll
                for (int u = 0; u < UG; ++u)
                    if (on[u]) {
                        const unsigned c = C[u].id;
                        b0l[u] = L.b0[c];
                        b0h[u] = L.b0[C[u].nb(0, 1)];
                        b1l[u] = L.b1[c];
                        b1h[u] = L.b1[C[u].nb(1, 1)];
                        r[u] = L.r[c];
                    }
#pragma unroll
                for (int u = 0; u < UG; ++u)
                    if (on[u]) {
                        const S dg = (b0l[u] + b0h[u] + b1l[u] + b1h[u]) * L.ih2;
                        L.z[C[u].id] = omega * r[u] / dg;
                    }
            });
            __syncthreads();
            }
            jacobi(L, L.z, L.zt, omega);                            // zt = z + omega (r - A z) / d
            __syncthreads();
            const BLev<S> Lc = lev(l + 1);
            const bool zc_first = l + 2 < nl;     // the coarse level is not the coarsest
            cells(Lc.d, [&](const Cell& Cc) {          // rc = mean of children of (r - A zt)
                S s = S(0);
                for (int dj = 0; dj < 2; ++dj)
                    for (int di = 0; di < 2; ++di) {
                        const Cell C = make_cell(L.d, 2 * Cc.i + di, 2 * Cc.j + dj, 0);
                        S dg;
                        s += L.r[C.id] - bapply(L, C, L.zt, dg);
                    }
                const S rc = s * S(0.25);
                Lc.r[Cc.id] = rc;
                if (zc_first) {                        // and the coarse z = omega rc / d (pointwise)
                    const unsigned c = Cc.id;
                    const S dg = (Lc.b0[c] + Lc.b0[Cc.nb(0, 1)] + Lc.b1[c] + Lc.b1[Cc.nb(1, 1)]) * Lc.ih2;
                    Lc.z[c] = omega * rc / dg;
                }
            });
            __syncthreads();
        }
        bool pro_done = false;  // the prolongation into the next finer level is done
        {   // coarsest: fixed damped Jacobi sweeps from zero, result in zt
            const BLev<S> L = lev(nl - 1);
            const int N = ncell(nl - 1);
            const int sweeps = 8 * max(L.d.nx, L.d.ny);
            const S wc = S(0.8);
            if (N <= 64) {
                const BLev<S> Lf = lev(nl - 2);
                coarsest_in_wave(L, N, sweeps, wc, &Lf);    // with the prolongation into nl - 2
                pro_done = true;
                __syncthreads();
            } else {
            for (int q = threadIdx.x; q < N; q += NT) L.zt[q] = S(0);
            __syncthreads();
            S* src = L.zt;
            S* dst = L.z;
            for (int s = 0; s < sweeps; ++s) {
                cells(L.d, [&](const Cell& C) {
                    S dg;
                    const S az = bapply(L, C, src, dg);
                    dst[C.id] = src[C.id] + wc * (L.r[C.id] - az) / dg;
                });
                __syncthreads();
                S* tmp = src;
                src = dst;
                dst = tmp;
            }
            if (src != L.zt) {
                for (int q = threadIdx.x; q < N; q += NT) L.zt[q] = src[q];
                __syncthreads();
            }
            }
        }
        for (int l = nl - 2; l >= 0; --l) {
            const BLev<S> L = lev(l);
            const BLev<S> Lc = lev(l + 1);
            // zt += P zc (piecewise constant), then z = zt + omega (r - A zt) / d and
            // zt = z + omega (r - A z) / d.  The prolongation is pointwise from the
            // coarse side, so the coarse level's last pass adds its values to the
            // children as it writes them (pro_done); a pass of its own only after
            // a coarsest grid solved by the block-wide loop.  Not fused into the
            // first sweep (zt + P zc at all five stencil points): a workgroup owns
            // the case, and that pass held 15 loads per cell in registers, which
            // cost more latency than the extra barrier.
            if (!pro_done) {
            cells_g(L.d, [&](const Cell* C, const bool* on) {
                S zf[UG], zc[UG];
#pragma unroll
                for (int u = 0; u < UG; ++u)
                    if (on[u]) {
                        zf[u] = L.zt[C[u].id];
                        zc[u] = Lc.zt[(C[u].j >> 1) * Lc.d.nx + (C[u].i >> 1)];
                    }
#pragma unroll
                for (int u = 0; u < UG; ++u)
                    if (on[u]) L.zt[C[u].id] = zf[u] + zc[u];
            });
            __syncthreads();
            }
            jacobi(L, L.zt, L.z, omega);
            __syncthreads();
            if (l > 0) {
                const BLev<S> Lf = lev(l - 1);
                jacobi(L, L.z, L.zt, omega, nullptr, &Lf);  // with the prolongation into l - 1
                pro_done = true;
                __syncthreads();
            }
        }
        double rz = 0.0;
        jacobi(lev(0), lev(0).z, lev(0).zt, omega, &rz);
        return bsum<NT>(rz, red);
    }

    // ---------------------------------------------------------- PCG
    // Solve A x = r0 (initial residual already in lev(0).r, |f|^2 = ff) to
    // |r|^2 <= tol2 ff.  x in precision X.  Returns iterations (>= 0), or -1
    // when maxit was reached, -2 on breakdown with a non-finite value.
    // x_zero: x starts at 0 and is not read (the first update writes it);
    // the x of a solve that returns 0 is then not written at all.
    template <typename X>
    __device__ int pcg(X* x, double ff, double rr, double tol2, S omega, bool x_zero = false) {
        if (ff == 0.0 || rr <= tol2 * ff) return 0;
        const BLev<S> L = lev(0);
        S* p = static_cast<S*>(K.pv);      // direction of the last iteration
        S* pn = static_cast<S*>(K.pv2);    // direction of this iteration
        S* q = static_cast<S*>(K.qv);
        double rz = 0.0, beta = 0.0;
        const S* pold = L.zt;              // first direction: zt + 0 zt = zt
        for (int it = 0; it < K.maxit; ++it) {
            // preconditioned residual (one call site: the V-cycle is inlined once)
            const double rzn = vcycle(omega, it > 0);
            if (it > 0) {
                beta = rzn / rz;
                S* cur = pn;               // the last iteration's direction is this one's p
                pn = p;
                p = cur;
                pold = p;
            }
            rz = rzn;
            if (!(rz > 0.0)) return isfinite(rz) ? it : -2;
            // new direction pn = zt + beta p, then q = A pn and <pn, q> (two
            // passes: the same values as forming pn at the five stencil points)
            const S sb = S(beta);
            cells_g(L.d, [&](const Cell* C, const bool* on) {
                S zv[UG], pv[UG];
#pragma unroll
                for (int u = 0; u < UG; ++u)
                    if (on[u]) {
                        zv[u] = L.zt[C[u].id];
                        pv[u] = pold[C[u].id];
                    }
#pragma unroll
                for (int u = 0; u < UG; ++u)
                    if (on[u]) pn[C[u].id] = zv[u] + sb * pv[u];
            });
            __syncthreads();
            double pq = 0.0;
            cells_g(L.d, [&](const Cell* C, const bool* on) {
                Stencil<S> v[UG];
#pragma unroll
                for (int u = 0; u < UG; ++u)
                    if (on[u]) v[u].load(L, C[u], pn);
#pragma unroll
                for (int u = 0; u < UG; ++u)
                    if (on[u]) {
                        S dg;
                        const S a = v[u].apply(L.ih2, dg);
                        q[C[u].id] = a;
                        pq += (double)v[u].xc * (double)a;
                    }
            });
            pq = bsum<NT>(pq, red);
            if (!(pq > 0.0)) return isfinite(pq) ? it : -2;
            const double alpha = rz / pq;
            double r2 = 0.0;
            // x, r update, and the first pre-smoothing sweep of the next
            // V-cycle (z = omega r / d, pointwise) from the new r
            const bool xz = x_zero && it == 0;
            cells_g(L.d, [&](const Cell* C, const bool* on) {
                X xv[UG];
                S pv[UG], rv[UG], qv[UG], b0l[UG], b0h[UG], b1l[UG], b1h[UG];
#pragma unroll
                for (int u = 0; u < UG; ++u)
                    if (on[u]) {
                        const unsigned c = C[u].id;
                        xv[u] = xz ? X(0) : x[c];
                        pv[u] = pn[c];
                        rv[u] = L.r[c];
                        qv[u] = q[c];
                        b0l[u] = L.b0[c];
                        b0h[u] = L.b0[C[u].nb(0, 1)];
                        b1l[u] = L.b1[c];
                        b1h[u] = L.b1[C[u].nb(1, 1)];
                    }
#pragma unroll
                for (int u = 0; u < UG; ++u)
                    if (on[u]) {
                        const unsigned c = C[u].id;
                        x[c] = xv[u] + X(alpha) * X(pv[u]);
                        const S rn = rv[u] - S(alpha) * qv[u];
                        L.r[c] = rn;
                        r2 += (double)rn * (double)rn;
                        const S dg = (b0l[u] + b0h[u] + b1l[u] + b1h[u]) * L.ih2;
                        L.z[c] = omega * rn / dg;
                    }
            });
            r2 = bsum<NT>(r2, red);
            if (!isfinite(r2)) return -2;
            if (r2 <= tol2 * ff) return it + 1;
        }
        return -1;
    }

    // r = f - A x with f = -(b - mean) on level 0; FP64 coefficients straight
    // from phi when R64 (the outer residual of the mixed path), else the
    // stored level-0 coefficients.  r stored in precision S.  ff, rr out.
    // aa: | |A||x| |^2, the squared sum of the face-flux magnitudes per cell
    // (the rounding level of the explicit FP64 residual, as in the
    // single-case solver)
    template <bool FROM_PHI>
    __device__ void residual(const T* phi, double mean, double& ff, double& rr, double& aa) {
        const BLev<S> L = lev(0);
        const Phys& P = K.P;
        const double h2 = 0.5 * P.rho2, dh = 0.5 * (P.rho1 - P.rho2);
        const double ih2 = 1.0 / (K.lh[0] * K.lh[0]);
        const double* b = K.b;
        const double* x = K.p;
        ff = 0.0;
        rr = 0.0;
        aa = 0.0;
        cells_g<2>(L.d, [&](const Cell* C, const bool* on) {
            // operands of two cells first: b, x at the cell and its four
            // neighbours, and phi there (FROM_PHI) or the stored coefficients
            double bv[2], x5[2][5], c5[2][5];
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (on[u]) {
                    const unsigned nb5[5] = {C[u].id, C[u].nb(0, -1), C[u].nb(0, 1), C[u].nb(1, -1), C[u].nb(1, 1)};
                    bv[u] = b[C[u].id];
#pragma unroll
                    for (int k = 0; k < 5; ++k) {
                        x5[u][k] = x[nb5[k]];
                        if (FROM_PHI) c5[u][k] = (double)phi[nb5[k]];
                    }
                    if (!FROM_PHI) {
                        c5[u][0] = L.b0[C[u].id];
                        c5[u][1] = L.b0[nb5[2]];
                        c5[u][2] = L.b1[C[u].id];
                        c5[u][3] = L.b1[nb5[4]];
                    }
                }
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (on[u]) {
                    const double f = -(bv[u] - mean);
                    double bl0, bh0, bl1, bh1;
                    if (FROM_PHI) {
                        auto hr = [&](double v) { return h2 + dh * (P.clamp ? fmin(fmax(v, 0.0), 1.0) : v); };
                        const double hc = hr(c5[u][0]);
                        const Cell& Q = C[u];
                        bl0 = Q.wall(0, -1) ? 0.0 : 1.0 / (hr(c5[u][1]) + hc);
                        bh0 = Q.wall(0, 1) ? 0.0 : 1.0 / (hc + hr(c5[u][2]));
                        bl1 = Q.wall(1, -1) ? 0.0 : 1.0 / (hr(c5[u][3]) + hc);
                        bh1 = Q.wall(1, 1) ? 0.0 : 1.0 / (hc + hr(c5[u][4]));
                    } else {
                        bl0 = c5[u][0];
                        bh0 = c5[u][1];
                        bl1 = c5[u][2];
                        bh1 = c5[u][3];
                    }
                    const double xc = x5[u][0];
                    const double ax = (bl0 * (xc - x5[u][1]) - bh0 * (x5[u][2] - xc) + bl1 * (xc - x5[u][3]) -
                                       bh1 * (x5[u][4] - xc)) * ih2;
                    const double r = f - ax;
                    L.r[C[u].id] = S(r);
                    ff += f * f;
                    rr += r * r;
                    const double am = (fabs(bl0 * (xc - x5[u][1])) + fabs(bh0 * (x5[u][2] - xc)) +
                                       fabs(bl1 * (xc - x5[u][3])) + fabs(bh1 * (x5[u][4] - xc))) * ih2;
                    aa += am * am;
                }
        });
        bsum2<NT>(ff, rr, red);
        aa = bsum<NT>(aa, red);
    }

    // Pressure solve for the current b (FP64, mean removed here): returns
    // TPF_OK / TPF_ENOCONV / TPF_ENONFINITE; K.p holds the zero-mean solution.
    // mean: the mean of b (summed by the divergence pass); gauge: remove the
    // mean of the solution (the last stage of a step and a single stage
    // evaluation; inside a step only G p is used, which a constant does not
    // change, and the warm starts combine pressures with weights summing to 1)
    __device__ int poisson(const T* phi, double mean, bool gauge) {
        const S omega = S(0.8);
        build_betas(phi);
        int total = 0, outer = 0, status = TPF_OK;
        double ff = 0.0, rr = 0.0, aa = 0.0;
        // squared rounding level of the explicit residual (16 ulps of |A||x|)
        const double fl2 = (16.0 * 0x1p-53) * (16.0 * 0x1p-53);
        if constexpr (sizeof(T) == 8) {
            residual<false>(phi, mean, ff, rr, aa);
            if (!isfinite(ff) || !isfinite(rr)) status = TPF_ENONFINITE;
            else {
                const int it = pcg<double>(K.p, ff, rr, K.rtol * K.rtol, omega);
                if (it == -2) status = TPF_ENONFINITE;
                else if (it < 0) status = TPF_ENOCONV;
                else total = it;
                outer = 1;
                residual<false>(phi, mean, ff, rr, aa);
            }
        } else {
            status = TPF_ENOCONV;
            for (int o = 0; o < 12; ++o) {
                residual<true>(phi, mean, ff, rr, aa);
                if (!isfinite(ff) || !isfinite(rr)) { status = TPF_ENONFINITE; break; }
                if (ff == 0.0 || rr <= K.rtol * K.rtol * ff || rr <= fl2 * aa) { status = TPF_OK; outer = o; break; }
                S* e = static_cast<S*>(K.ev);
                // aim at the outer tolerance, not below rtol_inner (FP32 depth);
                // an inner solve stopped by maxit still improves the iterate.
                // e starts at 0 (written by the first update, untouched when
                // the solve returns at once)
                const double tin = fmin(0.1, fmax(K.rtol_inner, INNER_MARGIN * K.rtol * sqrt(ff / rr)));
                const int it = pcg<S>(e, rr, rr, tin * tin, omega, true);
                if (it == -2) { status = TPF_ENONFINITE; break; }
                total += it < 0 ? K.maxit : it;
                if (it == 0) continue;
                cells_g(dims(0), [&](const Cell* C, const bool* on) {
                    double pv[UG];
                    S ev[UG];
#pragma unroll
                    for (int u = 0; u < UG; ++u)
                        if (on[u]) {
                            pv[u] = K.p[C[u].id];
                            ev[u] = e[C[u].id];
                        }
#pragma unroll
                    for (int u = 0; u < UG; ++u)
                        if (on[u]) K.p[C[u].id] = pv[u] + (double)ev[u];
                });
                __syncthreads();
            }
        }
        // zero-mean gauge
        if (gauge) {
            double sx = 0.0;
            cells_g(dims(0), [&](const Cell* C, const bool* on) {
                double v[UG];
#pragma unroll
                for (int u = 0; u < UG; ++u) v[u] = on[u] ? K.p[C[u].id] : 0.0;
#pragma unroll
                for (int u = 0; u < UG; ++u)
                    if (on[u]) sx += v[u];
            });
            sx = bsum<NT>(sx, red) / (double)ncell(0);
            cells_g(dims(0), [&](const Cell* C, const bool* on) {
                double v[UG];
#pragma unroll
                for (int u = 0; u < UG; ++u)
                    if (on[u]) v[u] = K.p[C[u].id];
#pragma unroll
                for (int u = 0; u < UG; ++u)
                    if (on[u]) K.p[C[u].id] = v[u] - sx;
            });
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            st->iters = total;
            st->outer = outer;
            st->solves += 1;
            st->outer_total += outer;
            st->inner_total += total;
            st->relres = ff > 0.0 ? sqrt(rr / ff) : 0.0;
        }
        return status;
    }

    // ---------------------------------------------------------- warm starts
    // Pressure warm start of stage s from the pressures of the earlier
    // stages (the rule of the single-case step): stage 2 extrapolates from
    // t - dt/2 and t, stage 3 adds the previous step's stage-3 minus stage-2
    // difference, stage 4 extrapolates from t and t + dt/2.
    __device__ void warm_start(int s, bool valid) {
        double* p = K.p;
        const double* h1 = K.ph[0];
        const double* h2 = K.ph[1];
        const double* h3 = K.ph[2];
        if ((s == 1 || s == 2) && !valid) return;
        if (s == 0) return;
        cells(dims(0), [&](const Cell& C) {
            const unsigned c = C.id;
            if (s == 1) p[c] = 2.0 * p[c] - h2[c];
            else if (s == 2) p[c] = p[c] + h3[c];
            else p[c] = 2.0 * p[c] - h1[c];
        });
        __syncthreads();
    }
    // the history the warm starts of later stages read (stored by the
    // projection pass of stages 1-3)
    __device__ __forceinline__ void record_pressure(int s, unsigned c) const {
        const double* p = K.p;
        if (s == 0) K.ph[0][c] = p[c];
        else if (s == 1) K.ph[1][c] = p[c];
        else if (s == 2) K.ph[2][c] = p[c] - K.ph[1][c];
    }

    // ---------------------------------------------------------- one stage
    // (phi, u) in slot `in`: dphi/dt and du/dt with the RK update of rk, the
    // outputs to slot `out` (and to the accumulator).  Returns a status.
    __device__ int stage(int in, int out, int acc, int yn, const RKArgs& rk) {
        const Phys& P = K.P;
        const Dims d = dims(0);
        const T* phi = static_cast<const T*>(K.y[in][0]);
        const T* u0 = static_cast<const T*>(K.y[in][1]);
        const T* u1 = static_cast<const T*>(K.y[in][2]);
        T* n0 = static_cast<T*>(K.nrm[0]);
        T* n1 = static_cast<T*>(K.nrm[1]);
        T* mu = static_cast<T*>(K.mu);
        T* kap = static_cast<T*>(K.kappa);
        T* r0 = static_cast<T*>(K.rflux[0]);
        T* r1 = static_cast<T*>(K.rflux[1]);
        T* m0 = static_cast<T*>(K.mflux[0]);
        T* m1 = static_cast<T*>(K.mflux[1]);
        T* f0 = static_cast<T*>(K.fs[0]);
        T* f1 = static_cast<T*>(K.fs[1]);
        int* flag = &st->nonfinite;
        // FP32 cases without kappa take the fused pass below (in FP64 its
        // recomputed normals cost the walled kernel variant its registers)
        if (sizeof(T) == 8 || K.need_kappa) {
            cells(d, [&](const Cell& C) { op_cell<T, 2>(P, C, phi, n0, n1, nullptr, K.need_mu ? mu : nullptr); });
            __syncthreads();
            if (K.need_kappa) {
                cells(d, [&](const Cell& C) { op_kappa<T, 2>(P, C, n0, n1, nullptr, kap); });
                __syncthreads();
            }
            cells(d, [&](const Cell& C) {
                op_face<T, 2>(P, C, phi, n0, n1, nullptr, u0, u1, nullptr, r0, r1, nullptr, m0, m1, nullptr);
            });
        } else if constexpr (sizeof(T) == 4) {
            // no kappa (CDI with the energy-based force): the fluxes recompute
            // the normals of c - e_a instead of reading them back, one pass
            // instead of two with the same values
            cells(d, [&](const Cell& C) {
                T g[3] = {T(0), T(0), T(0)};
                const T inv = grad_inv<T, 2>(P, C, phi, g);
                const T f = ld(phi, C.id);
                if (K.need_mu)
                    tpf::st(mu, C.id, T(P.sigma_hat / P.eps) * dpsi(f) - T(P.sigma_hat * P.eps) * lap_at<T, 2>(P, C, phi, f));
                auto nrm = [&](int a, bool lower) -> T {
                    if (!lower) return g[a] * inv;
                    // the cell c - e_a (itself across a wall: the mirror image)
                    const int i = (a == 0 && !C.wall(0, -1)) ? (C.i == 0 ? d.nx - 1 : C.i - 1) : C.i;
                    const int j = (a == 1 && !C.wall(1, -1)) ? (C.j == 0 ? d.ny - 1 : C.j - 1) : C.j;
                    T gm[3] = {T(0), T(0), T(0)};
                    const T im = grad_inv<T, 2>(P, make_cell_w(d, i, j, 0), phi, gm);
                    return gm[a] * im;
                };
                op_face_n<T, 2>(P, C, phi, nrm, u0, u1, nullptr, r0, r1, nullptr, m0, m1, nullptr);
            });
        }
        __syncthreads();
        T* ph_out = static_cast<T*>(K.y[out][0]);
        cells(d, [&](const Cell& C) {
            op_phase<T, 2>(P, rk, C, phi, u0, u1, nullptr, r0, r1, nullptr, kap,
                           static_cast<const T*>(K.y[yn][0]), static_cast<T*>(K.y[acc][0]), ph_out, flag);
            op_momentum<T, 2>(P, C, phi, u0, u1, nullptr, m0, m1, nullptr, mu, kap, f0, f1, nullptr,
                              nullptr, nullptr, nullptr);
        });
        __syncthreads();
        // b = D f*, and the sum of b for the solve's mean
        double bs = 0.0;
        cells(d, [&](const Cell& C) { bs += op_div<T, 2>(P, C, f0, f1, nullptr, K.b); });
        const double mean = bsum<NT>(bs, red) / (double)ncell(0);
        if (!rk.eval_only) warm_start(rk.stage, st->hist_valid != 0);
        const int status = poisson(phi, mean, rk.eval_only || rk.stage == 3);
        if (status != TPF_OK) return status;
        const bool rec = !rk.eval_only && rk.stage < 3;
        cells(d, [&](const Cell& C) {
            op_project<T, 2>(P, rk, C, phi, K.p, f0, f1, nullptr, static_cast<const T*>(K.y[yn][1]),
                             static_cast<const T*>(K.y[yn][2]), nullptr, static_cast<T*>(K.y[acc][1]),
                             static_cast<T*>(K.y[acc][2]), nullptr, static_cast<T*>(K.y[out][1]),
                             static_cast<T*>(K.y[out][2]), nullptr, flag);
            if (rec) record_pressure(rk.stage, C.id);
        });
        __syncthreads();
        return TPF_OK;
    }
};

// One RK4 step of every live case (mode 0), or the projection pressure of
// the current state (mode 1: one stage evaluation, outputs to slot 2).
// Block b owns case order[b].  commit = 0 computes the step without
// advancing the state (used by the tuner).
template <typename T, typename S, int NT, bool W>
__global__ __launch_bounds__(NT) void k_batch_step(const BCase* __restrict__ cases,
                                                   const int* __restrict__ order,
                                                   BState* __restrict__ states,
                                                   const double* __restrict__ dts, int mode,
                                                   int commit) {
    __shared__ double red[2 * (NT / 64)];
    extern __shared__ __align__(16) unsigned char batch_smem[];
    const int q = order[blockIdx.x];
    const BCase& K = cases[q];
    BState* st = states + q;
    if (st->status != TPF_OK) return;
    BatchBlock<T, S, NT, W> B{K, st, red, reinterpret_cast<S*>(batch_smem)};
    const int yn = st->yn, acc = st->acc;
    __syncthreads();
    if (mode == 1) {
        RKArgs rk{0, 1, 0.0, 0.0};
        const int s = B.stage(yn, 2, acc, yn, rk);
        if (threadIdx.x == 0 && s != TPF_OK) st->fails += 1;
        return;
    }
    const double dt = dts[q];
    // slots: inputs y_n, y1, y2, y1; outputs y1, y2, y1 and the accumulator
    const int y1 = 2, y2 = 3;
    const int ins[4] = {yn, y1, y2, y1};
    const int outs[4] = {y1, y2, y1, acc};
    const double wacc[4] = {dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0};
    const double wnext[4] = {0.5 * dt, 0.5 * dt, dt, 0.0};
    int status = TPF_OK;
    for (int s = 0; s < 4 && status == TPF_OK; ++s) {
        RKArgs rk{s, 0, wacc[s], wnext[s]};
        status = B.stage(ins[s], outs[s], acc, yn, rk);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (status == TPF_OK && st->nonfinite) status = TPF_ENONFINITE;
        if (status != TPF_OK) {
            st->status = status;
            st->hist_valid = 0;
        } else if (commit) {
            st->yn = acc;
            st->acc = yn;
            st->t += dt;
            st->step += 1;
            st->hist_valid = 1;
        }
        st->nonfinite = 0;
    }
}

// Diagnostics of every case (one workgroup per case): out[q * 11 + k] with
// the sums and maxima of op_diag.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_batch_diag(const BCase* __restrict__ cases,
                                                   const BState* __restrict__ states,
                                                   double* __restrict__ out) {
    __shared__ double red[2 * (NT / 64)];
    const int q = blockIdx.x;
    const BCase& K = cases[q];
    const int yn = states[q].yn;
    const Dims d{K.nx, K.ny, 1, 0, K.walls};
    double s[ND_SUM] = {0, 0, 0, 0, 0, 0, 0};
    double mx[ND_MAX] = {0.0, 0.0, -1e300, -1e300};
    for (int j = threadIdx.x / 64; j < d.ny; j += NT / 64)
        for (int i = threadIdx.x % 64; i < d.nx; i += 64) {
            double s1[ND_SUM] = {0, 0, 0, 0, 0, 0, 0};
            double m1[ND_MAX] = {0.0, 0.0, -1e300, -1e300};
            op_diag<T, 2>(K.P, make_cell_w(d, i, j, 0), static_cast<const T*>(K.y[yn][0]),
                          static_cast<const T*>(K.y[yn][1]), static_cast<const T*>(K.y[yn][2]), nullptr,
                          K.p, s1, m1);
            for (int k = 0; k < ND_SUM; ++k) s[k] += s1[k];
            for (int k = 0; k < ND_MAX; ++k) mx[k] = fmax(mx[k], m1[k]);
        }
    for (int k = 0; k < ND_SUM; ++k) s[k] = bsum<NT>(s[k], red);
    for (int k = 0; k < ND_MAX; ++k) {
        double v = mx[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        double m = red[0];
        for (int w = 1; w < NT / 64; ++w) m = fmax(m, red[w]);
        __syncthreads();
        mx[k] = m;
    }
    if (threadIdx.x == 0) {
        for (int k = 0; k < ND_SUM; ++k) out[q * (ND_SUM + ND_MAX) + k] = s[k];
        for (int k = 0; k < ND_MAX; ++k) out[q * (ND_SUM + ND_MAX) + ND_SUM + k] = mx[k];
    }
}

}  // namespace tpf
