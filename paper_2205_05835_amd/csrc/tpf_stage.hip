// Stage kernels: everything in one RK4 stage evaluation except the pressure
// solve.  One thread per cell; each kernel reads its operands straight from
// HBM with x-contiguous (coalesced) rows, neighbours reused through L1/L2.
//
// Discrete operators on the staggered periodic grid (Sec. 3):
//   A_a q[c] = (q[c-e_a] + q[c])/2,  G_a q[c] = (q[c] - q[c-e_a])/h,
//   D F[c] = sum_a (F_a[c+e_a] - F_a[c])/h,  C_a q[c] = (q[c+e_a]-q[c-e_a])/(2h)
#include "tpf_internal.hpp"

namespace tpf {

// ------------------------------------------------------------------ normals, mu
// n_a = C_a phi / sqrt(|C phi|^2 + delta^2)  (Table 1 caption, regularised)
// mu = (sigma_hat/eps) psi'(phi) - sigma_hat eps L phi   (Eq. 2)
template <typename T, int DIM>
__global__ __launch_bounds__(BLOCK) void k_cell(Dims d, Phys P, const T* __restrict__ phi,
                                                T* __restrict__ n0, T* __restrict__ n1,
                                                T* __restrict__ n2, T* __restrict__ mu) {
    Cell C;
    if (!cell_of_thread(d, C)) return;
    const unsigned c = C.id;
    const T f = phi[c];
    const T ih = T(P.inv_h), ih2 = T(0.5 * P.inv_h);
    T g[3] = {T(0), T(0), T(0)};
    T gg = T(0), lap = T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const T fp = phi[C.off(a, 1)], fm = phi[C.off(a, -1)];
        g[a] = (fp - fm) * ih2;
        gg += g[a] * g[a];
        lap += ((fp - f) * ih - (f - fm) * ih) * ih;
    }
    const T inv = T(1) / sqrt(gg + T(P.delta2));
    n0[c] = g[0] * inv;
    n1[c] = g[1] * inv;
    if (DIM == 3) n2[c] = g[2] * inv;
    if (mu) mu[c] = T(P.sigma_hat / P.eps) * dpsi(f) - T(P.sigma_hat * P.eps) * lap;
}

// kappa = - sum_a C_a n_a   (Eq. 3)
template <typename T, int DIM>
__global__ __launch_bounds__(BLOCK) void k_kappa(Dims d, Phys P, const T* __restrict__ n0,
                                                 const T* __restrict__ n1,
                                                 const T* __restrict__ n2, T* __restrict__ kappa) {
    Cell C;
    if (!cell_of_thread(d, C)) return;
    const T* n[3] = {n0, n1, n2};
    const T ih2 = T(0.5 * P.inv_h);
    T s = T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) s += (n[a][C.off(a, 1)] - n[a][C.off(a, -1)]) * ih2;
    kappa[C.id] = -s;
}

// ------------------------------------------------------------------ face fluxes
// CDI flux r_a = gamma [eps G_a phi - A_a(phi (1 - phi) n_a)]  (Table 1)
// mass flux m_a = rho_a u_a - (rho1 - rho2) r_a  (CDI; r = 0 otherwise)
template <typename T, int DIM>
__global__ __launch_bounds__(BLOCK) void k_face(Dims d, Phys P, const T* __restrict__ phi,
                                                const T* __restrict__ n0, const T* __restrict__ n1,
                                                const T* __restrict__ n2, const T* __restrict__ u0,
                                                const T* __restrict__ u1, const T* __restrict__ u2,
                                                T* __restrict__ r0, T* __restrict__ r1,
                                                T* __restrict__ r2, T* __restrict__ m0,
                                                T* __restrict__ m1, T* __restrict__ m2) {
    Cell C;
    if (!cell_of_thread(d, C)) return;
    const T* n[3] = {n0, n1, n2};
    const T* u[3] = {u0, u1, u2};
    T* r[3] = {r0, r1, r2};
    T* m[3] = {m0, m1, m2};
    const unsigned c = C.id;
    const T f = phi[c];
    const bool cdi = P.model == MODEL_CDI;
    const T drho = T(P.rho1 - P.rho2);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const unsigned cm = C.off(a, -1);
        const T fm = phi[cm];
        const T rho_f = T(0.5) * (rho_of(P, fm) + rho_of(P, f));
        T ra = T(0);
        if (cdi) {
            const T wm = fm * (T(1) - fm) * n[a][cm];
            const T wc = f * (T(1) - f) * n[a][c];
            ra = T(P.gamma) * (T(P.eps) * ((f - fm) * T(P.inv_h)) - T(0.5) * (wm + wc));
            r[a][c] = ra;
        }
        m[a][c] = rho_f * u[a][c] - drho * ra;
    }
}

// ------------------------------------------------------------------ phase field
// dphi/dt = -D(u A phi) + g   (Eq. 1), g of Table 1; then the RK4 update.
template <typename T, int DIM>
__global__ __launch_bounds__(BLOCK) void k_phase(Dims d, Phys P, RKArgs rk,
                                                 const T* __restrict__ phi,
                                                 const T* __restrict__ u0, const T* __restrict__ u1,
                                                 const T* __restrict__ u2, const T* __restrict__ r0,
                                                 const T* __restrict__ r1, const T* __restrict__ r2,
                                                 const T* __restrict__ kappa,
                                                 const T* __restrict__ yn, T* __restrict__ acc,
                                                 T* __restrict__ ynext, int* __restrict__ flags) {
    Cell C;
    if (!cell_of_thread(d, C)) return;
    const T* u[3] = {u0, u1, u2};
    const T* r[3] = {r0, r1, r2};
    const unsigned c = C.id;
    const T f = phi[c];
    const T ih = T(P.inv_h);
    T adv = T(0), g = T(0), lap = T(0), gg = T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const unsigned cp = C.off(a, 1), cm = C.off(a, -1);
        const T fp = phi[cp], fm = phi[cm];
        const T jhi = u[a][cp] * (T(0.5) * (f + fp));
        const T jlo = u[a][c] * (T(0.5) * (fm + f));
        adv += (jhi - jlo) * ih;
        if (P.model == MODEL_CDI) {
            g += (r[a][cp] - r[a][c]) * ih;
        } else {
            lap += ((fp - f) * ih - (f - fm) * ih) * ih;
            const T ga = (fp - fm) * T(0.5 * P.inv_h);
            gg += ga * ga;
        }
    }
    if (P.model != MODEL_CDI) {
        const T base = T(P.eps) * lap - dpsi(f) / T(P.eps);
        const T curv = (P.model == MODEL_SB) ? T(P.eps) * sqrt(gg) * kappa[c]
                                             : f * (T(1) - f) * kappa[c];
        g = T(P.gamma) * (base + curv);
    }
    const T k = -adv + g;
    if (rk.eval_only) {
        ynext[c] = k;
        return;
    }
    const T y0 = yn[c];
    const T a_new = (rk.stage == 0 ? y0 : acc[c]) + T(rk.wacc) * k;
    acc[c] = a_new;
    if (rk.stage < 3) ynext[c] = y0 + T(rk.wnext) * k;
    else if (!isfinite(a_new)) flags[0] = 1;
}

// ------------------------------------------------------------------ momentum
// f*_a = (-N_a + V_a + F_a) / rho_a on face (c, a).
//   N_a: velocity form of div(m (x) u) with arithmetic-mean fluxes on the u_a
//        control volume, minus u_a A_a(D m)
//   V_a: divergence of the full viscous stress eta (grad u + grad u^T); edge
//        viscosity = mean of the four cells around the edge
//   F_a: surface tension -- EB: A_a(mu) G_a phi (Eq. 4, + sign on the RHS);
//        CSF: sigma A_a(kappa) G_a phi;  LCSF: sigma_hat A_a(kappa)
//        A_a(phi(1-phi)) G_a phi (Eq. 11)
template <typename T, int DIM>
__global__ __launch_bounds__(BLOCK) void k_momentum(
    Dims d, Phys P, const T* __restrict__ phi, const T* __restrict__ u0,
    const T* __restrict__ u1, const T* __restrict__ u2, const T* __restrict__ m0,
    const T* __restrict__ m1, const T* __restrict__ m2, const T* __restrict__ mu,
    const T* __restrict__ kappa, T* __restrict__ f0, T* __restrict__ f1, T* __restrict__ f2,
    T* __restrict__ F0, T* __restrict__ F1, T* __restrict__ F2) {
    Cell C;
    if (!cell_of_thread(d, C)) return;
    const T* u[3] = {u0, u1, u2};
    const T* m[3] = {m0, m1, m2};
    T* fs[3] = {f0, f1, f2};
    T* Fo[3] = {F0, F1, F2};
    const unsigned c = C.id;
    const T ih = T(P.inv_h);
    const T f = phi[c];
    const T eta_c = visc_of(P, f);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const unsigned cp = C.off(a, 1), cm = C.off(a, -1);
        const T fm = phi[cm];
        const T eta_m = visc_of(P, fm);
        const T uac = u[a][c];
        // ---- advection
        T adv = T(0), dm_c = T(0), dm_m = T(0);
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            T hi, lo;
            if (b == a) {
                hi = (T(0.5) * (m[a][c] + m[a][cp])) * (T(0.5) * (uac + u[a][cp]));
                lo = (T(0.5) * (m[a][cm] + m[a][c])) * (T(0.5) * (u[a][cm] + uac));
            } else {
                const unsigned cpb = C.off(b, 1), cmb = C.off(b, -1), cmapb = C.off2(a, -1, b, 1);
                hi = (T(0.5) * (m[b][cpb] + m[b][cmapb])) * (T(0.5) * (uac + u[a][cpb]));
                lo = (T(0.5) * (m[b][c] + m[b][cm])) * (T(0.5) * (u[a][cmb] + uac));
            }
            adv += (hi - lo) * ih;
            dm_c += (m[b][C.off(b, 1)] - m[b][c]) * ih;
            // (c - e_a) + e_b: back to c itself when b == a
            dm_m += (m[b][b == a ? c : C.off2(a, -1, b, 1)] - m[b][cm]) * ih;
        }
        const T N = adv - uac * (T(0.5) * (dm_m + dm_c));
        // ---- viscous stress
        T V = T(0);
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            T hi, lo;
            if (b == a) {
                hi = T(2) * eta_c * ((u[a][cp] - uac) * ih);
                lo = T(2) * eta_m * ((uac - u[a][cm]) * ih);
            } else {
                const unsigned cpb = C.off(b, 1), cmb = C.off(b, -1);
                const unsigned cmapb = C.off2(a, -1, b, 1), cmamb = C.off2(a, -1, b, -1);
                const T e_pb = visc_of(P, phi[cpb]), e_mapb = visc_of(P, phi[cmapb]);
                const T e_mb = visc_of(P, phi[cmb]), e_mamb = visc_of(P, phi[cmamb]);
                const T eta_hi = T(0.25) * (eta_c + eta_m + e_pb + e_mapb);
                const T eta_lo = T(0.25) * (e_mb + e_mamb + eta_c + eta_m);
                hi = eta_hi * ((u[a][cpb] - uac) * ih + (u[b][cpb] - u[b][cmapb]) * ih);
                lo = eta_lo * ((uac - u[a][cmb]) * ih + (u[b][c] - u[b][cm]) * ih);
            }
            V += (hi - lo) * ih;
        }
        // ---- surface tension
        const T gphi = (f - fm) * ih;
        T F;
        if (P.force == FORCE_EB) {
            F = (T(0.5) * (mu[cm] + mu[c])) * gphi;
        } else if (P.force == FORCE_CSF) {
            F = T(P.sigma) * (T(0.5) * (kappa[cm] + kappa[c])) * gphi;
        } else {
            F = T(P.sigma_hat) * (T(0.5) * (kappa[cm] + kappa[c])) *
                (T(0.5) * (fm * (T(1) - fm) + f * (T(1) - f))) * gphi;
        }
        if (Fo[0]) Fo[a][c] = F;
        const T rho_f = T(0.5) * (rho_of(P, fm) + rho_of(P, f));
        fs[a][c] = (-N + V + F) * (T(1) / rho_f);
    }
}

// ------------------------------------------------------------------ D f* (FP64)
template <typename T, int DIM>
__global__ __launch_bounds__(BLOCK) void k_div(Dims d, Phys P, const T* __restrict__ f0,
                                               const T* __restrict__ f1,
                                               const T* __restrict__ f2, double* __restrict__ b,
                                               double* __restrict__ partials) {
    Cell C;
    double v[1] = {0.0};
    if (cell_of_thread(d, C)) {
        const T* fs[3] = {f0, f1, f2};
        const unsigned c = C.id;
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a)
            s += ((double)fs[a][C.off(a, 1)] - (double)fs[a][c]) * P.inv_h;
        b[c] = s;
        v[0] = s;
    }
    block_partials<1>(v, partials);
}

// ------------------------------------------------------------------ projection
// du_a/dt = f*_a - beta_a G_a p, then the RK4 update of u_a.
template <typename T, int DIM>
__global__ __launch_bounds__(BLOCK) void k_project(Dims d, Phys P, RKArgs rk,
                                                   const T* __restrict__ phi,
                                                   const double* __restrict__ p,
                                                   const T* __restrict__ f0, const T* __restrict__ f1,
                                                   const T* __restrict__ f2, const T* yn0,
                                                   const T* yn1, const T* yn2, T* acc0, T* acc1,
                                                   T* acc2, T* nx0, T* nx1, T* nx2,
                                                   int* __restrict__ flags) {
    Cell C;
    if (!cell_of_thread(d, C)) return;
    const T* fs[3] = {f0, f1, f2};
    const T* yn[3] = {yn0, yn1, yn2};
    T* acc[3] = {acc0, acc1, acc2};
    T* nx[3] = {nx0, nx1, nx2};
    const unsigned c = C.id;
    const T f = phi[c];
    const double pc = p[c];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const unsigned cm = C.off(a, -1);
        const double rho_f = 0.5 * ((double)rho_of(P, phi[cm]) + (double)rho_of(P, f));
        const double gp = (pc - p[cm]) * P.inv_h;
        const T k = T((double)fs[a][c] - gp / rho_f);
        if (rk.eval_only) {
            nx[a][c] = k;
            continue;
        }
        const T y0 = yn[a][c];
        const T a_new = (rk.stage == 0 ? y0 : acc[a][c]) + T(rk.wacc) * k;
        acc[a][c] = a_new;
        if (rk.stage < 3) nx[a][c] = y0 + T(rk.wnext) * k;
        else if (!isfinite(a_new)) flags[0] = 1;
    }
}

// ------------------------------------------------------------------ init / convert
// phi = [1 + tanh(s/2eps)]/2, s = (1 - q)/|grad q| with q = |x / a| (first-order
// signed distance to the ellipse/ellipsoid, exact for circles and spheres)
template <typename T, int DIM>
__global__ __launch_bounds__(BLOCK) void k_init_droplet(Dims d, double h, double eps, double c0,
                                                        double c1, double c2, double a0, double a1,
                                                        double a2, T* __restrict__ phi) {
    Cell C;
    if (!cell_of_thread(d, C)) return;
    const double cen[3] = {c0, c1, c2}, ax[3] = {a0, a1, a2};
    const int v[3] = {C.i, C.j, C.k};
    const int nn[3] = {d.nx, d.ny, d.nz};
    double q2 = 0.0, g2 = 0.0, amin = ax[0];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double L = nn[a] * h;
        double x = (v[a] + 0.5) * h - cen[a];
        x -= L * floor(x / L + 0.5);
        q2 += (x / ax[a]) * (x / ax[a]);
        g2 += x * x / (ax[a] * ax[a] * ax[a] * ax[a]);
        amin = fmin(amin, ax[a]);
    }
    const double q = sqrt(q2);
    const double s = (q2 == 0.0) ? amin : (1.0 - q) * q / sqrt(g2);
    phi[C.id] = T(0.5 * (1.0 + tanh(s / (2.0 * eps))));
}

template <typename T>
__global__ void k_convert_in(long N, const double* __restrict__ src, T* __restrict__ dst) {
    long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < N) dst[q] = T(src[q]);
}
template <typename T>
__global__ void k_convert_out(long N, const T* __restrict__ src, double* __restrict__ dst) {
    long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < N) dst[q] = (double)src[q];
}
template <typename T>
__global__ void k_fill(long N, T* __restrict__ dst, T v) {
    long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < N) dst[q] = v;
}

// ------------------------------------------------------------------ diagnostics
// Per-block partials: [0] sum phi, [1] KE density, [2] SE density, [3] sum p
// (phi>0.99), [4] count in, [5] sum p (phi<0.01), [6] count out; maxima:
// [7] |u_cell|, [8] |D u|, [9] -min phi, [10] max phi.
constexpr int ND_SUM = 7, ND_MAX = 4;

template <typename T, int DIM>
__global__ __launch_bounds__(BLOCK) void k_diag(Dims d, Phys P, const T* __restrict__ phi,
                                                const T* __restrict__ u0, const T* __restrict__ u1,
                                                const T* __restrict__ u2,
                                                const double* __restrict__ p,
                                                double* __restrict__ part) {
    Cell C;
    double s[ND_SUM] = {0, 0, 0, 0, 0, 0, 0};
    double mx[ND_MAX] = {0.0, 0.0, -1e300, -1e300};
    if (cell_of_thread(d, C)) {
        const T* u[3] = {u0, u1, u2};
        const unsigned c = C.id;
        const double f = (double)phi[c];
        double sp2 = 0.0, kin = 0.0, g2 = 0.0, div = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const unsigned cp = C.off(a, 1), cm = C.off(a, -1);
            const double ua = (double)u[a][c], uap = (double)u[a][cp];
            const double ub = 0.5 * (ua + uap);
            sp2 += ub * ub;
            const double fm = (double)phi[cm];
            const double rf = 0.5 * ((double)rho_of(P, fm) + (double)rho_of(P, f));
            kin += 0.5 * rf * ua * ua;
            const double g = (f - fm) * P.inv_h;
            g2 += g * g;
            div += (uap - ua) * P.inv_h;
        }
        s[0] = f;
        s[1] = kin;
        s[2] = (P.sigma_hat / P.eps) * psi(f) + 0.5 * P.sigma_hat * P.eps * g2;
        if (p) {
            if (f > 0.99) { s[3] = p[c]; s[4] = 1.0; }
            if (f < 0.01) { s[5] = p[c]; s[6] = 1.0; }
        }
        mx[0] = sqrt(sp2);
        mx[1] = fabs(div);
        mx[2] = -f;
        mx[3] = f;
    }
    block_sum<ND_SUM>(s);
    block_max<ND_MAX>(mx);
    if (thread_linear() == 0) {
        const int b = block_linear(), nb = nblocks_linear();
        for (int q = 0; q < ND_SUM; ++q) part[(long)q * nb + b] = s[q];
        for (int q = 0; q < ND_MAX; ++q) part[(long)(ND_SUM + q) * nb + b] = mx[q];
    }
}

__global__ __launch_bounds__(BLOCK) void k_diag_final(int nb, const double* __restrict__ part,
                                                      double* __restrict__ out) {
    double s[ND_SUM] = {0, 0, 0, 0, 0, 0, 0};
    double mx[ND_MAX] = {0.0, 0.0, -1e300, -1e300};
    for (int b = thread_linear(); b < nb; b += BLOCK) {
        for (int q = 0; q < ND_SUM; ++q) s[q] += part[(long)q * nb + b];
        for (int q = 0; q < ND_MAX; ++q) mx[q] = fmax(mx[q], part[(long)(ND_SUM + q) * nb + b]);
    }
    block_sum<ND_SUM>(s);
    block_max<ND_MAX>(mx);
    if (thread_linear() == 0) {
        for (int q = 0; q < ND_SUM; ++q) out[q] = s[q];
        for (int q = 0; q < ND_MAX; ++q) out[ND_SUM + q] = mx[q];
    }
}

// ================================================================== launchers

template <typename T>
static inline T* tp(void* p) { return static_cast<T*>(p); }
template <typename T>
static inline const T* ctp(const void* p) { return static_cast<const T*>(p); }

template <typename T, int DIM>
static hipError_t stage_fields_impl(tpf_ctx* c, const void* phi_s) {
    const Phys P = phys_of(c);
    const Dims d = dims_of(c->n);
    const dim3 g = grid_of(c->n), b(BX, BY);
    const bool need_mu = c->P.force == FORCE_EB;
    const bool need_kappa = c->P.model != MODEL_CDI || c->P.force != FORCE_EB;
    prof_begin(c, PC_CELL, (double)c->N * c->tsz * (1 + DIM + (need_mu ? 1 : 0)));
    k_cell<T, DIM><<<g, b, 0, c->stream>>>(d, P, ctp<T>(phi_s), tp<T>(c->nrm[0]), tp<T>(c->nrm[1]),
                                           tp<T>(c->nrm[2]), need_mu ? tp<T>(c->mu) : nullptr);
    prof_end(c);
    if (need_kappa) {
        prof_begin(c, PC_KAPPA, (double)c->N * c->tsz * (DIM + 1));
        k_kappa<T, DIM><<<g, b, 0, c->stream>>>(d, P, ctp<T>(c->nrm[0]), ctp<T>(c->nrm[1]),
                                                ctp<T>(c->nrm[2]), tp<T>(c->kappa));
        prof_end(c);
    }
    return hipGetLastError();
}

template <typename T, int DIM>
static hipError_t face_impl(tpf_ctx* c, const void* phi_s, const void* const u_s[3]) {
    const Phys P = phys_of(c);
    const Dims d = dims_of(c->n);
    const dim3 g = grid_of(c->n), b(BX, BY);
    const int cdi = c->P.model == MODEL_CDI;
    prof_begin(c, PC_FACE, (double)c->N * c->tsz * (1 + DIM * (cdi ? 4 : 2)));
    k_face<T, DIM><<<g, b, 0, c->stream>>>(
        d, P, ctp<T>(phi_s), ctp<T>(c->nrm[0]), ctp<T>(c->nrm[1]), ctp<T>(c->nrm[2]),
        ctp<T>(u_s[0]), ctp<T>(u_s[1]), ctp<T>(u_s[2]), tp<T>(c->rflux[0]), tp<T>(c->rflux[1]),
        tp<T>(c->rflux[2]), tp<T>(c->mflux[0]), tp<T>(c->mflux[1]), tp<T>(c->mflux[2]));
    prof_end(c);
    return hipGetLastError();
}

hipError_t launch_stage_fields(tpf_ctx* c, const void* phi_s, const void* const u_s[3]) {
    hipError_t e;
    if (c->mixed) {
        e = c->dim == 2 ? stage_fields_impl<float, 2>(c, phi_s) : stage_fields_impl<float, 3>(c, phi_s);
        if (e != hipSuccess) return e;
        return c->dim == 2 ? face_impl<float, 2>(c, phi_s, u_s) : face_impl<float, 3>(c, phi_s, u_s);
    }
    e = c->dim == 2 ? stage_fields_impl<double, 2>(c, phi_s) : stage_fields_impl<double, 3>(c, phi_s);
    if (e != hipSuccess) return e;
    return c->dim == 2 ? face_impl<double, 2>(c, phi_s, u_s) : face_impl<double, 3>(c, phi_s, u_s);
}

template <typename T, int DIM>
static hipError_t phase_impl(tpf_ctx* c, const void* phi_s, const void* const u_s[3],
                             const RKArgs& rk, void* out) {
    const Phys P = phys_of(c);
    const dim3 g = grid_of(c->n), b(BX, BY);
    const int cdi = c->P.model == MODEL_CDI;
    T* yn = tp<T>(c->phi[c->s_yn]);
    T* acc = tp<T>(c->phi[c->s_acc]);
    prof_begin(c, PC_PHASE, (double)c->N * c->tsz * (1 + DIM + (cdi ? DIM : 1) + (rk.eval_only ? 1 : 3 + (rk.stage < 3))));
    k_phase<T, DIM><<<g, b, 0, c->stream>>>(
        dims_of(c->n), P, rk, ctp<T>(phi_s), ctp<T>(u_s[0]), ctp<T>(u_s[1]), ctp<T>(u_s[2]),
        ctp<T>(c->rflux[0]), ctp<T>(c->rflux[1]), ctp<T>(c->rflux[2]), ctp<T>(c->kappa), yn, acc,
        tp<T>(out), c->flags);
    prof_end(c);
    return hipGetLastError();
}

hipError_t launch_phase_update(tpf_ctx* c, const void* phi_s, const void* const u_s[3],
                               const RKArgs& rk, void* out) {
    if (c->mixed)
        return c->dim == 2 ? phase_impl<float, 2>(c, phi_s, u_s, rk, out)
                           : phase_impl<float, 3>(c, phi_s, u_s, rk, out);
    return c->dim == 2 ? phase_impl<double, 2>(c, phi_s, u_s, rk, out)
                       : phase_impl<double, 3>(c, phi_s, u_s, rk, out);
}

template <typename T, int DIM>
static hipError_t mom_impl(tpf_ctx* c, const void* phi_s, const void* const u_s[3], int want_force) {
    const Phys P = phys_of(c);
    const dim3 g = grid_of(c->n), b(BX, BY);
    prof_begin(c, PC_MOM, (double)c->N * c->tsz * (1 + 3 * DIM + 1));
    k_momentum<T, DIM><<<g, b, 0, c->stream>>>(
        dims_of(c->n), P, ctp<T>(phi_s), ctp<T>(u_s[0]), ctp<T>(u_s[1]), ctp<T>(u_s[2]),
        ctp<T>(c->mflux[0]), ctp<T>(c->mflux[1]), ctp<T>(c->mflux[2]), ctp<T>(c->mu),
        ctp<T>(c->kappa), tp<T>(c->fs[0]), tp<T>(c->fs[1]), tp<T>(c->fs[2]),
        want_force ? tp<T>(c->force[0]) : nullptr, tp<T>(c->force[1]), tp<T>(c->force[2]));
    prof_end(c);
    return hipGetLastError();
}

hipError_t launch_momentum(tpf_ctx* c, const void* phi_s, const void* const u_s[3], int want_force) {
    if (c->mixed)
        return c->dim == 2 ? mom_impl<float, 2>(c, phi_s, u_s, want_force)
                           : mom_impl<float, 3>(c, phi_s, u_s, want_force);
    return c->dim == 2 ? mom_impl<double, 2>(c, phi_s, u_s, want_force)
                       : mom_impl<double, 3>(c, phi_s, u_s, want_force);
}

template <typename T, int DIM>
static hipError_t div_impl(tpf_ctx* c) {
    const Phys P = phys_of(c);
    const dim3 g = grid_of(c->n), b(BX, BY);
    prof_begin(c, PC_DIV, (double)c->N * (c->tsz * DIM + 8));
    k_div<T, DIM><<<g, b, 0, c->stream>>>(dims_of(c->n), P, ctp<T>(c->fs[0]), ctp<T>(c->fs[1]),
                                          ctp<T>(c->fs[2]), c->b, c->partials);
    prof_end(c);
    return hipGetLastError();
}

hipError_t launch_divergence(tpf_ctx* c) {
    hipError_t e;
    if (c->mixed) e = c->dim == 2 ? div_impl<float, 2>(c) : div_impl<float, 3>(c);
    else e = c->dim == 2 ? div_impl<double, 2>(c) : div_impl<double, 3>(c);
    if (e != hipSuccess) return e;
    return launch_finalize(c, (int)nblocks_of(c->n), 1, FIN_MEAN);
}

template <typename T, int DIM>
static hipError_t proj_impl(tpf_ctx* c, const void* phi_s, const RKArgs& rk, void* const out[3]) {
    const Phys P = phys_of(c);
    const dim3 g = grid_of(c->n), b(BX, BY);
    const int yn = c->s_yn, ac = c->s_acc;
    prof_begin(c, PC_PROJ, (double)c->N * (c->tsz * (1 + DIM + (rk.eval_only ? DIM : DIM * (3 + (rk.stage < 3)))) + 8));
    k_project<T, DIM><<<g, b, 0, c->stream>>>(
        dims_of(c->n), P, rk, ctp<T>(phi_s), c->p, ctp<T>(c->fs[0]), ctp<T>(c->fs[1]),
        ctp<T>(c->fs[2]), ctp<T>(c->u[0][yn]), ctp<T>(c->u[1][yn]), ctp<T>(c->u[2][yn]),
        tp<T>(c->u[0][ac]), tp<T>(c->u[1][ac]), tp<T>(c->u[2][ac]), tp<T>(out[0]), tp<T>(out[1]),
        tp<T>(out[2]), c->flags);
    prof_end(c);
    return hipGetLastError();
}

hipError_t launch_project_update(tpf_ctx* c, const void* phi_s, const RKArgs& rk, void* const out[3]) {
    if (c->mixed)
        return c->dim == 2 ? proj_impl<float, 2>(c, phi_s, rk, out) : proj_impl<float, 3>(c, phi_s, rk, out);
    return c->dim == 2 ? proj_impl<double, 2>(c, phi_s, rk, out) : proj_impl<double, 3>(c, phi_s, rk, out);
}

hipError_t launch_init_droplet(tpf_ctx* c, const double center[3], const double axes[3]) {
    const dim3 g = grid_of(c->n), b(BX, BY);
    const Dims d = dims_of(c->n);
    void* dst = c->phi[c->s_yn];
    const double eps = c->P.eps;
#define TPF_INIT(T, D)                                                                        \
    k_init_droplet<T, D><<<g, b, 0, c->stream>>>(d, c->h, eps, center[0], center[1], center[2], \
                                                 axes[0], axes[1], axes[2], tp<T>(dst))
    if (c->mixed) { if (c->dim == 2) TPF_INIT(float, 2); else TPF_INIT(float, 3); }
    else { if (c->dim == 2) TPF_INIT(double, 2); else TPF_INIT(double, 3); }
#undef TPF_INIT
    return hipGetLastError();
}

hipError_t launch_convert_in(tpf_ctx* c, const double* src, void* dst) {
    const int bs = 256;
    const unsigned nb = (unsigned)((c->N + bs - 1) / bs);
    if (c->mixed) k_convert_in<float><<<nb, bs, 0, c->stream>>>(c->N, src, tp<float>(dst));
    else k_convert_in<double><<<nb, bs, 0, c->stream>>>(c->N, src, tp<double>(dst));
    return hipGetLastError();
}

hipError_t launch_convert_out(tpf_ctx* c, const void* src, double* dst) {
    const int bs = 256;
    const unsigned nb = (unsigned)((c->N + bs - 1) / bs);
    if (c->mixed) k_convert_out<float><<<nb, bs, 0, c->stream>>>(c->N, ctp<float>(src), dst);
    else k_convert_out<double><<<nb, bs, 0, c->stream>>>(c->N, ctp<double>(src), dst);
    return hipGetLastError();
}

hipError_t launch_zero_state(tpf_ctx* c, void* dst) {
    const int bs = 256;
    const unsigned nb = (unsigned)((c->N + bs - 1) / bs);
    if (c->mixed) k_fill<float><<<nb, bs, 0, c->stream>>>(c->N, tp<float>(dst), 0.0f);
    else k_fill<double><<<nb, bs, 0, c->stream>>>(c->N, tp<double>(dst), 0.0);
    return hipGetLastError();
}

template <typename T, int DIM>
static hipError_t diag_impl(tpf_ctx* c, const void* phi, const void* const u[3], const double* p) {
    const Phys P = phys_of(c);
    const dim3 g = grid_of(c->n), b(BX, BY);
    k_diag<T, DIM><<<g, b, 0, c->stream>>>(dims_of(c->n), P, ctp<T>(phi), ctp<T>(u[0]),
                                           ctp<T>(u[1]), ctp<T>(u[2]), p, c->diag_part);
    k_diag_final<<<1, BLOCK, 0, c->stream>>>((int)nblocks_of(c->n), c->diag_part, c->diag_out);
    return hipGetLastError();
}

hipError_t launch_diagnostics(tpf_ctx* c, const void* phi, const void* const u[3], const double* p) {
    if (c->mixed)
        return c->dim == 2 ? diag_impl<float, 2>(c, phi, u, p) : diag_impl<float, 3>(c, phi, u, p);
    return c->dim == 2 ? diag_impl<double, 2>(c, phi, u, p) : diag_impl<double, 3>(c, phi, u, p);
}

}  // namespace tpf
