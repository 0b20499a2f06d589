// Backward-Euler step of the phase-field equation (Eq. 1) with the ISODI
// regularisation of Table 1, solved by Newton's method.
//
// ISODI differs from the Sun-Beckermann model only in the factor of its
// curvature term: phi (1 - phi) / eps, the equilibrium value of |grad phi|,
// in place of |grad phi| itself (the paragraph after Table 1).  That factor is
// a polynomial in phi, so the residual of a fully implicit step is a smooth
// function of phi with a Jacobian that is cheap to apply.  With the face
// velocity u held fixed over the step of size dt, one step solves
//
//   F(phi) = phi - phi_old - dt R(phi) = 0,
//   R(phi) = -D(u A phi) + gamma [eps L phi - psi'(phi)/eps + phi (1 - phi) kappa(phi)],
//
// kappa = -sum_a C_a n_a, n_a = C_a phi / s, s = sqrt(|C phi|^2 + delta^2), the
// same discrete operators as the explicit stage.  Newton: J(phi) x = -F(phi),
// phi += x, until max |F| <= tol, where
//
//   J v = c v + dt D(u A v) - dt gamma eps L v + dt gamma phi (1 - phi) sum_a C_a dn_a,
//   c   = 1 + dt gamma [psi''(phi)/eps - (1 - 2 phi) kappa],
//   dn_a = (C_a v - n_a (n . C v)) / s            (derivative of the normal;
//          s floored at 1e-10 / h here, see k_imp_normals).
//
// J is not symmetric (transport, and the curvature term), so each Newton
// system is solved by BiCGStab with a Jacobi (diagonal) right preconditioner
// M = c + 2 dim dt gamma eps / h^2, to a relative residual eta that follows
// the progress of Newton (Eisenstat and Walker's second choice: loose while
// ||F|| is large, tight as it falls, never tighter than newton_tol needs), or
// a fixed krylov_rtol; the step is then shortened by halving until ||F||_2
// decreases (Armijo).
//
// Every field is FP64 and every kernel is one thread per cell on the
// z-chunked tiling of the stage kernels; reductions write per-block partials
// that one single-block kernel sums in a fixed order (deterministic), and
// the scalars of the iteration stay on the device, so the host only reads
// them back to test convergence.
#include <algorithm>
#include <cmath>
#include <vector>

#include "tpf_internal.hpp"

namespace tpf {

// scalars of the Newton / BiCGStab iteration (device)
struct ImpScal {
    double rho, alpha, omega, beta;
    double rr0;     // ||b||^2 of the current Newton system (b = -F)
    double rr;      // ||r||^2 of the current Krylov residual
    double tol2;    // stop when rr <= tol2 rr0
    double fmax;    // max |F| at the current Newton iterate (NaN if F is not finite)
    int done, iters, breakdown, pad;
};
static_assert(sizeof(ImpScal) <= 256, "ImpScal must fit its 256-byte slot");

enum { IMP_INIT = 0, IMP_ALPHA = 1, IMP_OMEGA = 2, IMP_RHO = 3 };

constexpr int FIN_T = 256;

// Write NS block sums and NM block maxima to partials[q * nb + block].
template <int NS, int NM>
__device__ __forceinline__ void imp_partials(double (&s)[NS], double (&m)[NM > 0 ? NM : 1], double* partials) {
    block_sum<NS>(s);
    if constexpr (NM > 0) block_max<NM>(m);
    if (thread_linear() == 0) {
        const int nb = nblocks_linear(), b = block_linear();
#pragma unroll
        for (int q = 0; q < NS; ++q) partials[(long)q * nb + b] = s[q];
#pragma unroll
        for (int q = 0; q < NM; ++q) partials[(long)(NS + q) * nb + b] = m[q];
    }
}

// ------------------------------------------------------------------ Newton-level kernels
// n_a = C_a phi / s at every cell, and the 1/s of the normal's derivative
// with s floored at SJ_FLOOR per cell width: where |C phi| is below that, the
// exact derivative (up to 1/delta) holds only for changes of phi far smaller
// than a Newton correction, and the bounded one steers Newton better.  F
// itself always uses the exact normals, so the root does not change.
constexpr double SJ_FLOOR = 1e-10;

template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_imp_normals(Dims d, int kz, Phys P, const double* __restrict__ phi,
                                                       double* __restrict__ n0, double* __restrict__ n1,
                                                       double* __restrict__ n2, double* __restrict__ sinv) {
    const double floor2 = (SJ_FLOOR * P.inv_h) * (SJ_FLOOR * P.inv_h);
    for_cells_zchunk(d, kz, [&](const Cell& C) {
        double g[3] = {0.0, 0.0, 0.0};
        const double inv = grad_inv<double, DIM>(P, C, phi, g);
        st(n0, C.id, g[0] * inv);
        st(n1, C.id, g[1] * inv);
        if (DIM == 3) st(n2, C.id, g[2] * inv);
        double gg = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) gg += g[a] * g[a];
        st(sinv, C.id, 1.0 / sqrt(gg + P.delta2 + floor2));
    });
}

// F at every cell; the Newton system's right-hand side b = -F goes to r and
// rhat (BiCGStab's shadow residual), the pointwise Jacobian part c to cdiag;
// block partials of sum F^2 and max |F|
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_imp_residual(
    Dims d, int kz, Phys P, double dt, const double* __restrict__ phi, const double* __restrict__ phi_old,
    const double* __restrict__ u0, const double* __restrict__ u1, const double* __restrict__ u2,
    const double* __restrict__ n0, const double* __restrict__ n1, const double* __restrict__ n2,
    double* __restrict__ r, double* __restrict__ rhat, double* __restrict__ cdiag, double* __restrict__ partials) {
    const double* u[3] = {u0, u1, u2};
    const double* n[3] = {n0, n1, n2};
    double s[1] = {0.0}, m[1] = {0.0};
    for_cells_zchunk(d, kz, [&](const Cell& C) {
        const unsigned c = C.id;
        const double f = ld(phi, c);
        const double ih = P.inv_h, ih2 = 0.5 * P.inv_h;
        double adv = 0.0, lap = 0.0, divn = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const unsigned cp = C.off(a, 1), cm = C.off(a, -1);
            const double fp = ld(phi, cp), fm = ld(phi, cm);
            adv += (ld(u[a], cp) * (0.5 * (f + fp)) - ld(u[a], c) * (0.5 * (fm + f))) * ih;
            lap += ((fp - f) * ih - (f - fm) * ih) * ih;
            divn += (ld(n[a], cp) - ld(n[a], cm)) * ih2;
        }
        const double kap = -divn;
        const double rhs = -adv + P.gamma * (P.eps * lap - dpsi(f) / P.eps + f * (1.0 - f) * kap);
        const double F = f - ld(phi_old, c) - dt * rhs;
        st(r, c, -F);
        st(rhat, c, -F);
        const double d2psi = 1.0 - 6.0 * f + 6.0 * f * f;
        st(cdiag, c, 1.0 + dt * P.gamma * (d2psi / P.eps - (1.0 - 2.0 * f) * kap));
        s[0] += F * F;
        m[0] = fmax(m[0], fabs(F));
    });
    imp_partials<1, 1>(s, m, partials);
}

// phi += lam x
__global__ __launch_bounds__(BLOCK) void k_imp_update(Dims d, int kz, double lam, double* __restrict__ phi,
                                                      const double* __restrict__ x) {
    for_cells_zchunk(d, kz, [&](const Cell& C) { st(phi, C.id, ld(phi, C.id) + lam * ld(x, C.id)); });
}

// Start of step n > 0 of a call: phi_old holds phi_{n-1} and phi holds phi_n.
// phi_old = phi_n, and the Newton start phi = 2 phi_n - phi_{n-1} (linear
// extrapolation in time, O(dt^2) from the root instead of O(dt)).
__global__ __launch_bounds__(BLOCK) void k_imp_predict(Dims d, int kz, double* __restrict__ phi,
                                                       double* __restrict__ phi_old) {
    for_cells_zchunk(d, kz, [&](const Cell& C) {
        const double cur = ld(phi, C.id);
        st(phi, C.id, 2.0 * cur - ld(phi_old, C.id));
        st(phi_old, C.id, cur);
    });
}

// ------------------------------------------------------------------ Jacobian-vector product
// dn_a = (C_a w - n_a (n . C w)) / s
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_imp_dn(Dims d, int kz, Phys P, const ImpScal* __restrict__ sc,
                                                  const double* __restrict__ w, const double* __restrict__ n0,
                                                  const double* __restrict__ n1, const double* __restrict__ n2,
                                                  const double* __restrict__ sinv, double* __restrict__ dn0,
                                                  double* __restrict__ dn1, double* __restrict__ dn2) {
    if (sc->done) return;
    const double* n[3] = {n0, n1, n2};
    double* dn[3] = {dn0, dn1, dn2};
    for_cells_zchunk(d, kz, [&](const Cell& C) {
        const unsigned c = C.id;
        const double ih2 = 0.5 * P.inv_h;
        double cw[3] = {0.0, 0.0, 0.0}, nc[3] = {0.0, 0.0, 0.0}, ncw = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            cw[a] = (ld(w, C.off(a, 1)) - ld(w, C.off(a, -1))) * ih2;
            nc[a] = ld(n[a], c);
            ncw += nc[a] * cw[a];
        }
        const double si = ld(sinv, c);
#pragma unroll
        for (int a = 0; a < DIM; ++a) st(dn[a], c, si * (cw[a] - nc[a] * ncw));
    });
}

// out = J w.  MODE 0: partial <rhat, out> (other = rhat); MODE 1: partials
// <out, s> and <out, out> (other = s)
template <int DIM, int MODE>
__global__ __launch_bounds__(BLOCK) void k_imp_apply(
    Dims d, int kz, Phys P, double dt, const ImpScal* __restrict__ sc, const double* __restrict__ phi,
    const double* __restrict__ u0, const double* __restrict__ u1, const double* __restrict__ u2,
    const double* __restrict__ cdiag, const double* __restrict__ w, const double* __restrict__ dn0,
    const double* __restrict__ dn1, const double* __restrict__ dn2, const double* __restrict__ other,
    double* __restrict__ out, double* __restrict__ partials) {
    if (sc->done) return;
    const double* u[3] = {u0, u1, u2};
    const double* dn[3] = {dn0, dn1, dn2};
    double s[2] = {0.0, 0.0}, m[1] = {0.0};
    for_cells_zchunk(d, kz, [&](const Cell& C) {
        const unsigned c = C.id;
        const double ih = P.inv_h, ih2 = 0.5 * P.inv_h;
        const double wc = ld(w, c), f = ld(phi, c);
        double adv = 0.0, lap = 0.0, ddn = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const unsigned cp = C.off(a, 1), cm = C.off(a, -1);
            const double wp = ld(w, cp), wm = ld(w, cm);
            adv += (ld(u[a], cp) * (0.5 * (wc + wp)) - ld(u[a], c) * (0.5 * (wm + wc))) * ih;
            lap += ((wp - wc) * ih - (wc - wm) * ih) * ih;
            ddn += (ld(dn[a], cp) - ld(dn[a], cm)) * ih2;
        }
        const double gdt = dt * P.gamma;
        const double jw = ld(cdiag, c) * wc + dt * adv - gdt * P.eps * lap + gdt * f * (1.0 - f) * ddn;
        st(out, c, jw);
        const double o = ld(other, c);
        s[0] += o * jw;
        if (MODE == 1) s[1] += jw * jw;
    });
    imp_partials<2, 0>(s, m, partials);
}

// ------------------------------------------------------------------ BiCGStab vector updates
// p = r (first iteration) or r + beta (p - omega v); phat = p / M
__global__ __launch_bounds__(BLOCK) void k_imp_dir(Dims d, int kz, double mshift, const ImpScal* __restrict__ sc,
                                                   const double* __restrict__ r, double* __restrict__ p,
                                                   const double* __restrict__ v, const double* __restrict__ cdiag,
                                                   double* __restrict__ phat) {
    if (sc->done) return;
    const bool first = sc->iters == 0;
    const double beta = sc->beta, om = sc->omega;
    for_cells_zchunk(d, kz, [&](const Cell& C) {
        const unsigned c = C.id;
        double pn;
        if (first) pn = ld(r, c);
        else pn = ld(r, c) + beta * (ld(p, c) - om * ld(v, c));
        st(p, c, pn);
        st(phat, c, pn / (ld(cdiag, c) + mshift));
    });
}

// s = r - alpha v (in place of r); shat = s / M
__global__ __launch_bounds__(BLOCK) void k_imp_half(Dims d, int kz, double mshift, const ImpScal* __restrict__ sc,
                                                    double* __restrict__ r, const double* __restrict__ v,
                                                    const double* __restrict__ cdiag, double* __restrict__ shat) {
    if (sc->done) return;
    const double alpha = sc->alpha;
    for_cells_zchunk(d, kz, [&](const Cell& C) {
        const unsigned c = C.id;
        const double sv = ld(r, c) - alpha * ld(v, c);
        st(r, c, sv);
        st(shat, c, sv / (ld(cdiag, c) + mshift));
    });
}

// x += alpha phat + omega shat (x = 0 before the first iteration);
// r = s - omega t; partials <rhat, r>, <r, r>
__global__ __launch_bounds__(BLOCK) void k_imp_step(Dims d, int kz, const ImpScal* __restrict__ sc,
                                                    double* __restrict__ x, const double* __restrict__ phat,
                                                    const double* __restrict__ shat, double* __restrict__ r,
                                                    const double* __restrict__ t, const double* __restrict__ rhat,
                                                    double* __restrict__ partials) {
    if (sc->done) return;
    const double alpha = sc->alpha, om = sc->omega;
    const bool first = sc->iters == 0;
    double s[2] = {0.0, 0.0}, m[1] = {0.0};
    for_cells_zchunk(d, kz, [&](const Cell& C) {
        const unsigned c = C.id;
        const double x0 = first ? 0.0 : ld(x, c);
        st(x, c, x0 + alpha * ld(phat, c) + om * ld(shat, c));
        const double rn = ld(r, c) - om * ld(t, c);
        st(r, c, rn);
        s[0] += ld(rhat, c) * rn;
        s[1] += rn * rn;
    });
    imp_partials<2, 0>(s, m, partials);
}

// ------------------------------------------------------------------ scalar updates
// Sums (and for IMP_INIT the maximum) of the block partials in a fixed order,
// then the scalar recurrences of Newton / BiCGStab.
__global__ __launch_bounds__(FIN_T) void k_imp_finalize(int nb, int op, double tol2,
                                                        const double* __restrict__ partials,
                                                        ImpScal* __restrict__ sc) {
    if (op != IMP_INIT && sc->done) return;
    double v[2] = {0.0, 0.0}, m[1] = {0.0};
    for (int i = threadIdx.x; i < nb; i += FIN_T) {
        v[0] += partials[i];
        if (op == IMP_INIT) m[0] = fmax(m[0], partials[(long)nb + i]);
        else v[1] += partials[(long)nb + i];
    }
    block_sum<2>(v);
    block_max<1>(m);
    if (threadIdx.x != 0) return;
    if (op == IMP_INIT) {
        const double ff = v[0];
        sc->rr0 = ff;
        sc->rr = ff;
        sc->rho = ff;
        sc->tol2 = tol2;
        sc->fmax = isfinite(ff) ? m[0] : NAN;
        sc->alpha = 1.0;
        sc->omega = 1.0;
        sc->beta = 0.0;
        sc->iters = 0;
        sc->breakdown = 0;
        sc->done = !(ff > 0.0) || !isfinite(ff);
    } else if (op == IMP_ALPHA) {
        const double rv = v[0];
        if (!(rv != 0.0) || !isfinite(rv)) {
            sc->done = 1;
            sc->breakdown = 1;
        } else {
            sc->alpha = sc->rho / rv;
        }
    } else if (op == IMP_OMEGA) {
        const double ts = v[0], tt = v[1];
        // t = 0 only when s = 0: x += alpha phat is then exact, and omega = 0
        // ends the iteration after the update
        sc->omega = (tt > 0.0 && isfinite(tt) && isfinite(ts)) ? ts / tt : 0.0;
    } else {
        const double rho_n = v[0], rr = v[1];
        sc->rr = rr;
        sc->iters += 1;
        if (!isfinite(rr) || !isfinite(rho_n)) {
            sc->done = 1;
            sc->breakdown = 1;
        } else if (rr <= sc->tol2 * sc->rr0) {
            sc->done = 1;
        } else if (sc->omega == 0.0 || rho_n == 0.0) {
            sc->done = 1;
            sc->breakdown = 1;
        } else {
            sc->beta = (rho_n / sc->rho) * (sc->alpha / sc->omega);
            sc->rho = rho_n;
        }
    }
}

// ------------------------------------------------------------------ host side
namespace {

struct ImpFields {
    double* phi;        // current iterate (the state slot)
    double* phi_old;
    const double* u[3];
    double* n[3];
    double* sinv;
    double* cdiag;
    double* dn[3];
    double *x, *r, *rhat, *p, *v, *phat, *shat, *t;
};

ImpFields imp_fields(tpf_ctx* c) {
    ImpFields F{};
    F.phi = (double*)c->phi[c->s_yn];
    F.phi_old = (double*)c->phi[c->s_y1];
    for (int a = 0; a < 3; ++a) {
        const int on = a < c->dim;
        F.u[a] = (const double*)(on ? c->u[a][c->s_yn] : c->u[0][c->s_yn]);
        F.n[a] = (double*)(on ? c->nrm[a] : c->nrm[0]);
        F.dn[a] = (double*)(on ? c->rflux[a] : c->rflux[0]);
    }
    F.sinv = (double*)c->mu;
    F.cdiag = (double*)c->kappa;
    F.x = (double*)c->phi[c->s_y2];
    F.r = (double*)c->phi[c->s_acc];
    F.rhat = c->b;
    F.p = (double*)c->mflux[0];
    F.v = (double*)c->mflux[1];
    F.phat = (double*)c->fs[0];
    F.shat = (double*)c->fs[1];
    F.t = (double*)c->force[0];
    return F;
}

struct Launch {
    tpf_ctx* c;
    Dims d;
    Phys P;
    int kz;
    dim3 grid;
    int nb;
    double N;     // cells
};

template <int DIM>
hipError_t newton_residual(const Launch& L, const ImpFields& F, double dt, double tol2, ImpScal* sc) {
    tpf_ctx* c = L.c;
    prof_begin(c, PC_IMP_NORMALS, L.N * 8.0 * (2 + DIM));
    k_imp_normals<DIM><<<L.grid, dim3(BX, BY), 0, c->stream>>>(L.d, L.kz, L.P, F.phi, F.n[0], F.n[1], F.n[2], F.sinv);
    prof_end(c);
    prof_begin(c, PC_IMP_RESIDUAL, L.N * 8.0 * (5 + 2 * DIM));
    k_imp_residual<DIM><<<L.grid, dim3(BX, BY), 0, c->stream>>>(L.d, L.kz, L.P, dt, F.phi, F.phi_old, F.u[0],
                                                                F.u[1], F.u[2], F.n[0], F.n[1], F.n[2], F.r,
                                                                F.rhat, F.cdiag, c->partials);
    prof_end(c);
    prof_begin(c, PC_IMP_FINALIZE, 0.0);
    k_imp_finalize<<<1, FIN_T, 0, c->stream>>>(L.nb, IMP_INIT, tol2, c->partials, sc);
    prof_end(c);
    return hipGetLastError();
}

// J w -> out (dn is scratch)
template <int DIM, int MODE>
void jvp(const Launch& L, const ImpFields& F, double dt, const ImpScal* sc, const double* w,
         const double* other, double* out) {
    tpf_ctx* c = L.c;
    prof_begin(c, PC_IMP_DN, L.N * 8.0 * (2 + 2 * DIM));
    k_imp_dn<DIM><<<L.grid, dim3(BX, BY), 0, c->stream>>>(L.d, L.kz, L.P, sc, w, F.n[0], F.n[1], F.n[2], F.sinv,
                                                   F.dn[0], F.dn[1], F.dn[2]);
    prof_end(c);
    prof_begin(c, PC_IMP_APPLY, L.N * 8.0 * (5 + 2 * DIM));
    k_imp_apply<DIM, MODE><<<L.grid, dim3(BX, BY), 0, c->stream>>>(L.d, L.kz, L.P, dt, sc, F.phi, F.u[0], F.u[1],
                                                            F.u[2], F.cdiag, w, F.dn[0], F.dn[1], F.dn[2],
                                                            other, out, c->partials);
    prof_end(c);
}

void fin(const Launch& L, int op, double tol2, ImpScal* sc) {
    prof_begin(L.c, PC_IMP_FINALIZE, 0.0);
    k_imp_finalize<<<1, FIN_T, 0, L.c->stream>>>(L.nb, op, tol2, L.c->partials, sc);
    prof_end(L.c);
}

// one BiCGStab iteration (every kernel returns at once when sc->done)
template <int DIM>
void bicgstab_iteration(const Launch& L, const ImpFields& F, double dt, double mshift, ImpScal* sc) {
    tpf_ctx* c = L.c;
    prof_begin(c, PC_IMP_VECTOR, L.N * 8.0 * 6);
    k_imp_dir<<<L.grid, dim3(BX, BY), 0, c->stream>>>(L.d, L.kz, mshift, sc, F.r, F.p, F.v, F.cdiag, F.phat);
    prof_end(c);
    jvp<DIM, 0>(L, F, dt, sc, F.phat, F.rhat, F.v);
    fin(L, IMP_ALPHA, 0.0, sc);
    prof_begin(c, PC_IMP_VECTOR, L.N * 8.0 * 5);
    k_imp_half<<<L.grid, dim3(BX, BY), 0, c->stream>>>(L.d, L.kz, mshift, sc, F.r, F.v, F.cdiag, F.shat);
    prof_end(c);
    jvp<DIM, 1>(L, F, dt, sc, F.shat, F.r, F.t);
    fin(L, IMP_OMEGA, 0.0, sc);
    prof_begin(c, PC_IMP_VECTOR, L.N * 8.0 * 8);
    k_imp_step<<<L.grid, dim3(BX, BY), 0, c->stream>>>(L.d, L.kz, sc, F.x, F.phat, F.shat, F.r, F.t, F.rhat,
                                                c->partials);
    prof_end(c);
    fin(L, IMP_RHO, 0.0, sc);
}

// launches and bytes issued per profiling class so far
struct ProfSnap {
    long n[NPROF];
    double b[NPROF];
};
void snapshot(const tpf_ctx* c, ProfSnap& o) {
    for (int q = 0; q < NPROF; ++q) {
        o.n[q] = c->prof_issued[q];
        o.b[q] = c->prof_issued_bytes[q];
    }
}

tpf_status read_scal(tpf_ctx* c, ImpScal* host) {
    const hipError_t e = fetch_bytes(c, c->imp_scal, sizeof(ImpScal), host);
    return e == hipSuccess ? TPF_OK : hip_fail(e, "implicit step scalars");
}

template <int DIM>
tpf_status implicit_steps(tpf_ctx* c, double dt, int nsteps, const tpf_implicit_opts& o, tpf_implicit_info* info) {
    const ImpFields F = imp_fields(c);
    Launch L{c, dims_of(c->n), phys_of(c), c->stage_kz, zchunk_grid(c->n, c->stage_kz), 0, (double)c->N};
    L.nb = (int)L.grid.x;
    ImpScal* sc = (ImpScal*)c->imp_scal;
    const double mshift = 2.0 * DIM * dt * L.P.gamma * L.P.eps * L.P.inv_h * L.P.inv_h;
    // fixed forcing term, or 0: adaptive (set per Newton iteration below)
    const double tol2 = o.krylov_rtol * o.krylov_rtol;
    const bool adaptive = o.krylov_rtol == 0.0;
    const size_t bytes = (size_t)c->N * 8;
    const int chunk = 4;   // BiCGStab iterations queued between convergence checks
    const int LS_MAX = 10;  // halvings of the Newton step in the line search
    std::vector<ProfSnap> snaps((size_t)o.krylov_maxit + chunk);
    for (int n = 0; n < nsteps; ++n) {
        hipError_t e;
        if (n == 0) {
            e = hipMemcpyAsync(F.phi_old, F.phi, bytes, hipMemcpyDeviceToDevice, c->stream);
        } else {
            prof_begin(c, PC_IMP_VECTOR, L.N * 8.0 * 4);
            k_imp_predict<<<L.grid, dim3(BX, BY), 0, c->stream>>>(L.d, L.kz, F.phi, F.phi_old);
            prof_end(c);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return hip_fail(e, "implicit step start");
        int newton = 0, krylov = 0;
        double eta_prev = 0.1, fn_prev = 0.0, eta2 = 0.0;
        tpf_status st = TPF_OK;
        // F and the Newton system at the current iterate
        ImpScal h;
        e = newton_residual<DIM>(L, F, dt, tol2, sc);
        if (e != hipSuccess) st = hip_fail(e, "implicit residual");
        if (st == TPF_OK) st = read_scal(c, &h);
        double fmax = st == TPF_OK ? h.fmax : 0.0;
        for (; st == TPF_OK; ++newton) {
            fmax = h.fmax;
            if (!std::isfinite(fmax)) {
                set_error("non-finite residual in the implicit phase-field step; phi rolled back");
                st = TPF_ENONFINITE;
                break;
            }
            if (fmax <= o.newton_tol) break;
            if (newton == o.newton_maxit) {
                set_error("implicit phase-field step: Newton did not reach newton_tol within newton_maxit "
                          "iterations; phi rolled back");
                st = TPF_ENOCONV;
                break;
            }
            const double ff = h.rr0;
            if (adaptive) {
                // Eisenstat-Walker choice 2 (gamma 0.9, exponent (1 + sqrt 5)/2)
                // with their safeguard, capped at 0.1, and floored where a
                // linear residual of 0.1 newton_tol in 2-norm (hence in max
                // norm) is already met
                const double fn = std::sqrt(ff), ex = 1.6180339887498949;
                double eta = 0.1;
                if (newton > 0) {
                    eta = 0.9 * std::pow(fn / fn_prev, ex);
                    const double sg = 0.9 * std::pow(eta_prev, ex);
                    if (sg > 0.1) eta = std::max(eta, sg);
                }
                eta = std::max(std::min(eta, 0.1), std::min(0.5, 0.1 * o.newton_tol / fn));
                eta_prev = eta;
                fn_prev = fn;
                eta2 = eta * eta;
                e = hipMemcpyAsync(&sc->tol2, &eta2, sizeof(double), hipMemcpyHostToDevice, c->stream);
                if (e != hipSuccess) { st = hip_fail(e, "implicit forcing term"); break; }
            }
            int done = h.done, queued = 0;
            for (int it = 0; !done && it < o.krylov_maxit; it += chunk) {
                const int k = std::min(chunk, o.krylov_maxit - it);
                for (int q = 0; q < k; ++q, ++queued) {
                    snapshot(c, snaps[queued]);
                    bicgstab_iteration<DIM>(L, F, dt, mshift, sc);
                }
                if ((e = hipGetLastError()) != hipSuccess) break;
                if ((st = read_scal(c, &h)) != TPF_OK) break;
                done = h.done;
            }
            if (e != hipSuccess) { st = hip_fail(e, "implicit Krylov solve"); break; }
            if (st != TPF_OK) break;
            // iterations queued after convergence returned at once: they count
            // in the timed total but not as working launches or bytes
            if (h.iters < queued) {
                ProfSnap now;
                snapshot(c, now);
                for (int q = 0; q < NPROF; ++q) {
                    c->prof_noop[q] += now.n[q] - snaps[h.iters].n[q];
                    c->prof_noop_bytes[q] += now.b[q] - snaps[h.iters].b[q];
                }
            }
            if (h.iters == 0) {
                set_error("implicit phase-field step: BiCGStab broke down in its first iteration; phi rolled back");
                st = TPF_ENOCONV;
                break;
            }
            krylov += h.iters;
            // backtracking on ||F||_2: accept phi + lam x once
            // ||F(phi + lam x)|| <= (1 - 1e-4 lam) ||F(phi)||, halving lam up
            // to LS_MAX times (the last trial is kept).  Each trial evaluates
            // F and sets up the next Newton system at the trial point.
            double lam = 1.0;
            for (int bt = 0;; ++bt) {
                prof_begin(c, PC_IMP_VECTOR, L.N * 8.0 * 3);
                // phi_k + lam x  ->  phi_k + (lam / 2) x
                const double coef = bt == 0 ? 1.0 : -0.5 * lam;
                k_imp_update<<<L.grid, dim3(BX, BY), 0, c->stream>>>(L.d, L.kz, coef, F.phi, F.x);
                prof_end(c);
                if (bt > 0) lam *= 0.5;     // phi now holds phi_k + lam x
                e = newton_residual<DIM>(L, F, dt, tol2, sc);
                if (e != hipSuccess) { st = hip_fail(e, "implicit residual"); break; }
                if ((st = read_scal(c, &h)) != TPF_OK) break;
                const double lim = (1.0 - 1e-4 * lam) * (1.0 - 1e-4 * lam) * ff;
                if ((std::isfinite(h.rr0) && h.rr0 <= lim) || bt == LS_MAX) break;
            }
        }
        if (info) {
            info->newton_iters = newton;
            info->krylov_iters = krylov;
            info->residual = fmax;
            info->newton_total += newton;
            info->krylov_total += krylov;
        }
        if (st != TPF_OK) {
            (void)hipMemcpyAsync(F.phi, F.phi_old, bytes, hipMemcpyDeviceToDevice, c->stream);
            (void)hipStreamSynchronize(c->stream);
            return st;
        }
    }
    return TPF_OK;
}

}  // namespace
}  // namespace tpf

using namespace tpf;

extern "C" tpf_status tpf_implicit_phase_step(tpf_ctx* c, double dt, int32_t nsteps, const tpf_implicit_opts* opts,
                                              tpf_implicit_info* info) {
    if (!c) { set_error("ctx is NULL"); return TPF_EINVAL; }
    if (c->P.model != TPF_ISODI) {
        set_error("the implicit phase-field step is defined for the ISODI model");
        return TPF_EINVAL;
    }
    if (c->mixed) { set_error("the implicit phase-field step needs an FP64 context"); return TPF_EINVAL; }
    if (c->walls) { set_error("the implicit phase-field step needs a periodic box (params.walls = 0)"); return TPF_EINVAL; }
    if (!(dt >= 0.0) || !std::isfinite(dt) || nsteps < 0) {
        set_error("dt must be finite and >= 0, nsteps >= 0");
        return TPF_EINVAL;
    }
    tpf_implicit_opts o{};
    if (opts) o = *opts;
    if (!(o.newton_tol >= 0.0) || !(o.krylov_rtol >= 0.0 && o.krylov_rtol < 1.0) || o.newton_maxit < 0 ||
        o.krylov_maxit < 0) {
        set_error("newton_tol >= 0, 0 <= krylov_rtol < 1, newton_maxit >= 0, krylov_maxit >= 0");
        return TPF_EINVAL;
    }
    if (o.newton_tol == 0.0) o.newton_tol = 1e-12;
    if (o.newton_maxit == 0) o.newton_maxit = 30;
    if (o.krylov_maxit == 0) o.krylov_maxit = 400;
    if (info) *info = tpf_implicit_info{};
    if (nsteps == 0) return TPF_OK;
    // the step changes phi: the stored projection pressure no longer belongs
    // to the state
    c->p_valid = 0;
    return c->dim == 2 ? implicit_steps<2>(c, dt, nsteps, o, info) : implicit_steps<3>(c, dt, nsteps, o, info);
}
