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
#pragma once
#include <limits>

#include "tpf_internal.hpp"

namespace tpf {

constexpr int BMAXLEV = 10;

// One case of a batch: grid, physics and the addresses of its fields.
struct BCase {
    Phys P;
    int nx, ny, nlev, maxit;
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
    void* pv;           // CG direction (solver precision)
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

template <typename T, typename S, int NT>
struct BatchBlock {
    const BCase& K;
    BState* st;
    double* red;
    S* lds;

    // the cells of a (nx, ny) grid, 64 consecutive x per wave
    template <typename F>
    __device__ __forceinline__ void cells(const Dims& d, F f) const {
        for (int j = threadIdx.x / 64; j < d.ny; j += NT / 64)
            for (int i = threadIdx.x % 64; i < d.nx; i += 64) f(make_cell(d, i, j, 0));
    }

    __device__ __forceinline__ Dims dims(int l) const { return Dims{K.ln[l][0], K.ln[l][1], 1, 0}; }
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
    // clamped linear law; coarser levels: mean of the two fine faces covering
    // each coarse face.  Then the LDS-resident levels receive their copies.
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
            b0[C.id] = S(1) / (hr(C.nb(0, -1)) + hc);
            b1[C.id] = S(1) / (hr(C.nb(1, -1)) + hc);
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

    // ---------------------------------------------------------- V-cycle
    // z = M r on level 0 (r in lev(0).r); the result ends in lev(0).zt.
    __device__ void vcycle(S omega) {
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
            return;
        }
        for (int l = 0; l + 1 < nl; ++l) {
            const BLev<S> L = lev(l);
            cells(L.d, [&](const Cell& C) {            // z = omega r / d
                const unsigned c = C.id;
                const S dg = (L.b0[c] + L.b0[C.nb(0, 1)] + L.b1[c] + L.b1[C.nb(1, 1)]) * L.ih2;
                L.z[c] = omega * L.r[c] / dg;
            });
            __syncthreads();
            cells(L.d, [&](const Cell& C) {            // zt = z + omega (r - A z) / d
                S dg;
                const S az = bapply(L, C, L.z, dg);
                L.zt[C.id] = L.z[C.id] + omega * (L.r[C.id] - az) / dg;
            });
            __syncthreads();
            const BLev<S> Lc = lev(l + 1);
            cells(Lc.d, [&](const Cell& Cc) {          // rc = mean of children of (r - A zt)
                S s = S(0);
                for (int dj = 0; dj < 2; ++dj)
                    for (int di = 0; di < 2; ++di) {
                        const Cell C = make_cell(L.d, 2 * Cc.i + di, 2 * Cc.j + dj, 0);
                        S dg;
                        s += L.r[C.id] - bapply(L, C, L.zt, dg);
                    }
                Lc.r[Cc.id] = s * S(0.25);
            });
            __syncthreads();
        }
        {   // coarsest: fixed damped Jacobi sweeps from zero, result in zt
            const BLev<S> L = lev(nl - 1);
            const int N = ncell(nl - 1);
            const int sweeps = 8 * max(L.d.nx, L.d.ny);
            const S wc = S(0.8);
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
        for (int l = nl - 2; l >= 0; --l) {
            const BLev<S> L = lev(l);
            const BLev<S> Lc = lev(l + 1);
            // Z = zt + P zc, then z = Z + omega (r - A Z) / d, zt = z + omega (r - A z) / d
            cells(L.d, [&](const Cell& C) {
                auto Z = [&](int i, int j) {
                    const int ii = wrapc(i, L.d.nx), jj = wrapc(j, L.d.ny);
                    return L.zt[jj * L.d.nx + ii] + Lc.zt[(jj >> 1) * Lc.d.nx + (ii >> 1)];
                };
                const unsigned c = C.id;
                const S bl0 = L.b0[c], bh0 = L.b0[C.nb(0, 1)];
                const S bl1 = L.b1[c], bh1 = L.b1[C.nb(1, 1)];
                const S zc = Z(C.i, C.j);
                const S az = (bl0 * (zc - Z(C.i - 1, C.j)) - bh0 * (Z(C.i + 1, C.j) - zc) +
                              bl1 * (zc - Z(C.i, C.j - 1)) - bh1 * (Z(C.i, C.j + 1) - zc)) * L.ih2;
                const S dg = (bl0 + bh0 + bl1 + bh1) * L.ih2;
                L.z[c] = zc + omega * (L.r[c] - az) / dg;
            });
            __syncthreads();
            cells(L.d, [&](const Cell& C) {
                S dg;
                const S az = bapply(L, C, L.z, dg);
                L.zt[C.id] = L.z[C.id] + omega * (L.r[C.id] - az) / dg;
            });
            __syncthreads();
        }
    }

    // ---------------------------------------------------------- PCG
    // Solve A x = r0 (initial residual already in lev(0).r, |f|^2 = ff) to
    // |r|^2 <= tol2 ff.  x in precision X.  Returns iterations (>= 0), or -1
    // when maxit was reached, -2 on breakdown with a non-finite value.
    template <typename X>
    __device__ int pcg(X* x, double ff, double rr, double tol2, S omega) {
        if (ff == 0.0 || rr <= tol2 * ff) return 0;
        const BLev<S> L = lev(0);
        S* p = static_cast<S*>(K.pv);
        S* q = static_cast<S*>(K.qv);
        vcycle(omega);
        double rz = 0.0;
        cells(L.d, [&](const Cell& C) {
            const S z = L.zt[C.id];
            p[C.id] = z;
            rz += (double)L.r[C.id] * (double)z;
        });
        rz = bsum<NT>(rz, red);
        for (int it = 0; it < K.maxit; ++it) {
            if (!(rz > 0.0)) return isfinite(rz) ? it : -2;
            double pq = 0.0;
            cells(L.d, [&](const Cell& C) {
                S dg;
                const S a = bapply(L, C, p, dg);
                q[C.id] = a;
                pq += (double)p[C.id] * (double)a;
            });
            pq = bsum<NT>(pq, red);
            if (!(pq > 0.0)) return isfinite(pq) ? it : -2;
            const double alpha = rz / pq;
            double r2 = 0.0;
            cells(L.d, [&](const Cell& C) {
                const unsigned c = C.id;
                x[c] = X((double)x[c] + alpha * (double)p[c]);
                const S rn = S((double)L.r[c] - alpha * (double)q[c]);
                L.r[c] = rn;
                r2 += (double)rn * (double)rn;
            });
            r2 = bsum<NT>(r2, red);
            if (!isfinite(r2)) return -2;
            if (r2 <= tol2 * ff) return it + 1;
            vcycle(omega);
            double rzn = 0.0;
            cells(L.d, [&](const Cell& C) { rzn += (double)L.r[C.id] * (double)L.zt[C.id]; });
            rzn = bsum<NT>(rzn, red);
            const double beta = rzn / rz;
            rz = rzn;
            cells(L.d, [&](const Cell& C) {
                const unsigned c = C.id;
                p[c] = S((double)L.zt[c] + beta * (double)p[c]);
            });
            __syncthreads();
        }
        return -1;
    }

    // r = f - A x with f = -(b - mean) on level 0; FP64 coefficients straight
    // from phi when R64 (the outer residual of the mixed path), else the
    // stored level-0 coefficients.  r stored in precision S.  ff, rr out.
    template <bool FROM_PHI>
    __device__ void residual(const T* phi, double mean, double& ff, double& rr) {
        const BLev<S> L = lev(0);
        const Phys& P = K.P;
        const double h2 = 0.5 * P.rho2, dh = 0.5 * (P.rho1 - P.rho2);
        const double ih2 = 1.0 / (K.lh[0] * K.lh[0]);
        const double* b = K.b;
        const double* x = K.p;
        ff = 0.0;
        rr = 0.0;
        cells(L.d, [&](const Cell& C) {
            const unsigned c = C.id;
            const double f = -(b[c] - mean);
            double ax;
            if (FROM_PHI) {
                auto hr = [&](unsigned q) {
                    const double v = (double)phi[q];
                    return h2 + dh * (P.clamp ? fmin(fmax(v, 0.0), 1.0) : v);
                };
                const double hc = hr(c);
                const double bl0 = 1.0 / (hr(C.nb(0, -1)) + hc), bh0 = 1.0 / (hc + hr(C.nb(0, 1)));
                const double bl1 = 1.0 / (hr(C.nb(1, -1)) + hc), bh1 = 1.0 / (hc + hr(C.nb(1, 1)));
                const double xc = x[c];
                ax = (bl0 * (xc - x[C.nb(0, -1)]) - bh0 * (x[C.nb(0, 1)] - xc) +
                      bl1 * (xc - x[C.nb(1, -1)]) - bh1 * (x[C.nb(1, 1)] - xc)) * ih2;
            } else {
                const double bl0 = L.b0[c], bh0 = L.b0[C.nb(0, 1)];
                const double bl1 = L.b1[c], bh1 = L.b1[C.nb(1, 1)];
                const double xc = x[c];
                ax = (bl0 * (xc - x[C.nb(0, -1)]) - bh0 * (x[C.nb(0, 1)] - xc) +
                      bl1 * (xc - x[C.nb(1, -1)]) - bh1 * (x[C.nb(1, 1)] - xc)) * ih2;
            }
            const double r = f - ax;
            L.r[c] = S(r);
            ff += f * f;
            rr += r * r;
        });
        bsum2<NT>(ff, rr, red);
    }

    // Pressure solve for the current b (FP64, mean removed here): returns
    // TPF_OK / TPF_ENOCONV / TPF_ENONFINITE; K.p holds the zero-mean solution.
    __device__ int poisson(const T* phi) {
        const S omega = S(0.8);
        double mean = 0.0;
        cells(dims(0), [&](const Cell& C) { mean += K.b[C.id]; });
        mean = bsum<NT>(mean, red) / (double)ncell(0);
        build_betas(phi);
        int total = 0, outer = 0, status = TPF_OK;
        double ff = 0.0, rr = 0.0;
        if constexpr (sizeof(T) == 8) {
            residual<false>(phi, mean, ff, rr);
            if (!isfinite(ff) || !isfinite(rr)) status = TPF_ENONFINITE;
            else {
                const int it = pcg<double>(K.p, ff, rr, K.rtol * K.rtol, omega);
                if (it == -2) status = TPF_ENONFINITE;
                else if (it < 0) status = TPF_ENOCONV;
                else total = it;
                outer = 1;
                residual<false>(phi, mean, ff, rr);
            }
        } else {
            status = TPF_ENOCONV;
            for (int o = 0; o < 12; ++o) {
                residual<true>(phi, mean, ff, rr);
                if (!isfinite(ff) || !isfinite(rr)) { status = TPF_ENONFINITE; break; }
                if (ff == 0.0 || rr <= K.rtol * K.rtol * ff) { status = TPF_OK; outer = o; break; }
                S* e = static_cast<S*>(K.ev);
                cells(dims(0), [&](const Cell& C) { e[C.id] = S(0); });
                __syncthreads();
                // aim at the outer tolerance, not below rtol_inner (FP32 depth);
                // an inner solve stopped by maxit still improves the iterate
                const double tin = fmin(0.1, fmax(K.rtol_inner, 0.5 * K.rtol * sqrt(ff / rr)));
                const int it = pcg<S>(e, rr, rr, tin * tin, omega);
                if (it == -2) { status = TPF_ENONFINITE; break; }
                total += it < 0 ? K.maxit : it;
                cells(dims(0), [&](const Cell& C) { K.p[C.id] += (double)e[C.id]; });
                __syncthreads();
            }
        }
        // zero-mean gauge
        double sx = 0.0;
        cells(dims(0), [&](const Cell& C) { sx += K.p[C.id]; });
        sx = bsum<NT>(sx, red) / (double)ncell(0);
        cells(dims(0), [&](const Cell& C) { K.p[C.id] -= sx; });
        __syncthreads();
        if (threadIdx.x == 0) {
            st->iters = total;
            st->outer = outer;
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
    __device__ void record_pressure(int s) {
        const double* p = K.p;
        if (s == 3) return;
        cells(dims(0), [&](const Cell& C) {
            const unsigned c = C.id;
            if (s == 0) K.ph[0][c] = p[c];
            else if (s == 1) K.ph[1][c] = p[c];
            else K.ph[2][c] = p[c] - K.ph[1][c];
        });
        __syncthreads();
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
        cells(d, [&](const Cell& C) { op_cell<T, 2>(P, C, phi, n0, n1, nullptr, K.need_mu ? mu : nullptr); });
        __syncthreads();
        if (K.need_kappa) {
            cells(d, [&](const Cell& C) { op_kappa<T, 2>(P, C, n0, n1, nullptr, kap); });
            __syncthreads();
        }
        cells(d, [&](const Cell& C) {
            op_face<T, 2>(P, C, phi, n0, n1, nullptr, u0, u1, nullptr, r0, r1, nullptr, m0, m1, nullptr);
        });
        __syncthreads();
        T* ph_out = static_cast<T*>(K.y[out][0]);
        cells(d, [&](const Cell& C) {
            op_phase<T, 2>(P, rk, C, phi, u0, u1, nullptr, r0, r1, nullptr, kap,
                           static_cast<const T*>(K.y[yn][0]), static_cast<T*>(K.y[acc][0]), ph_out, flag);
            op_momentum<T, 2>(P, C, phi, u0, u1, nullptr, m0, m1, nullptr, mu, kap, f0, f1, nullptr,
                              nullptr, nullptr, nullptr);
        });
        __syncthreads();
        cells(d, [&](const Cell& C) { (void)op_div<T, 2>(P, C, f0, f1, nullptr, K.b); });
        __syncthreads();
        if (!rk.eval_only) warm_start(rk.stage, st->hist_valid != 0);
        const int status = poisson(phi);
        if (status != TPF_OK) return status;
        if (!rk.eval_only) record_pressure(rk.stage);
        cells(d, [&](const Cell& C) {
            op_project<T, 2>(P, rk, C, phi, K.p, f0, f1, nullptr, static_cast<const T*>(K.y[yn][1]),
                             static_cast<const T*>(K.y[yn][2]), nullptr, static_cast<T*>(K.y[acc][1]),
                             static_cast<T*>(K.y[acc][2]), nullptr, static_cast<T*>(K.y[out][1]),
                             static_cast<T*>(K.y[out][2]), nullptr, flag);
        });
        __syncthreads();
        return TPF_OK;
    }
};

// One RK4 step of every live case (mode 0), or the projection pressure of
// the current state (mode 1: one stage evaluation, outputs to slot 2).
// Block b owns case order[b].  commit = 0 computes the step without
// advancing the state (used by the tuner).
template <typename T, typename S, int NT>
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
    BatchBlock<T, S, NT> B{K, st, red, reinterpret_cast<S*>(batch_smem)};
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
    const Dims d{K.nx, K.ny, 1, 0};
    double s[ND_SUM] = {0, 0, 0, 0, 0, 0, 0};
    double mx[ND_MAX] = {0.0, 0.0, -1e300, -1e300};
    for (int j = threadIdx.x / 64; j < d.ny; j += NT / 64)
        for (int i = threadIdx.x % 64; i < d.nx; i += 64) {
            double s1[ND_SUM] = {0, 0, 0, 0, 0, 0, 0};
            double m1[ND_MAX] = {0.0, 0.0, -1e300, -1e300};
            op_diag<T, 2>(K.P, make_cell(d, i, j, 0), static_cast<const T*>(K.y[yn][0]),
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
