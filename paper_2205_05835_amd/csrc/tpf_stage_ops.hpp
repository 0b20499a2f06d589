// Per-cell bodies of the stage operators, shared by the one-thread-per-cell
// kernels of the single-case step and the block-stride loops of the batched
// persistent step.  Each op_* computes the outputs of one cell C.
//
// Discrete operators on the staggered grid (Sec. 3):
//   A_a q[c] = (q[c-e_a] + q[c])/2,  G_a q[c] = (q[c] - q[c-e_a])/h,
//   D F[c] = sum_a (F_a[c+e_a] - F_a[c])/h,  C_a q[c] = (q[c+e_a]-q[c-e_a])/(2h)
//
// Each axis is periodic or closed by free-slip walls at both ends (cells
// with wall bits, tpf_index.hpp).  A free-slip wall is a mirror plane of the
// solution: across it a cell field reads its even image (Cell::off), the
// component of the normal along the wall's axis its odd image, and a face
// field normal to the wall is 0 on the wall faces.  The bodies write 0 to
// the face outputs that lie on a wall (fluxes, f*, the velocity update), so
// the wall faces of u stay as they were set.
#pragma once
#include "tpf_device.hpp"

namespace tpf {

struct RKArgs {
    int stage;        // 0..3
    int eval_only;    // 1: write the derivative to out instead of updating
    double wacc;      // acc (+)= wacc * k
    double wnext;     // ynext = yn + wnext * k (stages 0-2)
};

// ------------------------------------------------------------------ normals, mu
// central gradient g = C phi at cell Q and 1 / sqrt(|g|^2 + delta^2)
template <typename T, int DIM>
__device__ __forceinline__ T grad_inv(const Phys& P, const Cell& Q, const T* __restrict__ phi, T (&g)[3]) {
    const T ih2 = T(0.5 * P.inv_h);
    T gg = T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        g[a] = (ld(phi, Q.off(a, 1)) - ld(phi, Q.off(a, -1))) * ih2;
        gg += g[a] * g[a];
    }
    return rsqrt_of(gg + T(P.delta2));
}

// L phi at cell C (5- or 7-point)
template <typename T, int DIM>
__device__ __forceinline__ T lap_at(const Phys& P, const Cell& C, const T* __restrict__ phi, T f) {
    const T ih = T(P.inv_h);
    T lap = T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const T fp = ld(phi, C.off(a, 1)), fm = ld(phi, C.off(a, -1));
        lap += ((fp - f) * ih - (f - fm) * ih) * ih;
    }
    return lap;
}

// n_a = C_a phi / sqrt(|C phi|^2 + delta^2)  (Table 1 caption, regularised)
// mu = (sigma_hat/eps) psi'(phi) - sigma_hat eps L phi   (Eq. 2)
template <typename T, int DIM>
__device__ __forceinline__ void op_cell(const Phys& P, const Cell& C, const T* __restrict__ phi,
                                                T* __restrict__ n0, T* __restrict__ n1,
                                                T* __restrict__ n2, T* __restrict__ mu) {
    const unsigned c = C.id;
    const T f = ld(phi, c);
    T g[3] = {T(0), T(0), T(0)};
    const T inv = grad_inv<T, DIM>(P, C, phi, g);
    st(n0, c, g[0] * inv);
    st(n1, c, g[1] * inv);
    if (DIM == 3) st(n2, c, g[2] * inv);
    if (mu) st(mu, c, T(P.sigma_hat / P.eps) * dpsi(f) - T(P.sigma_hat * P.eps) * lap_at<T, DIM>(P, C, phi, f));
}

// kappa = - sum_a C_a n_a   (Eq. 3)
template <typename T, int DIM>
__device__ __forceinline__ void op_kappa(const Phys& P, const Cell& C, const T* __restrict__ n0,
                                                 const T* __restrict__ n1,
                                                 const T* __restrict__ n2, T* __restrict__ kappa) {
    const T* n[3] = {n0, n1, n2};
    const T ih2 = T(0.5 * P.inv_h);
    T s = T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        // n_a is odd across a wall normal to a: its image there is -n_a(c)
        const T np = ld(n[a], C.off(a, 1)), nm = ld(n[a], C.off(a, -1));
        s += ((C.wall(a, 1) ? -np : np) - (C.wall(a, -1) ? -nm : nm)) * ih2;
    }
    st(kappa, C.id, -s);
}

// ------------------------------------------------------------------ face fluxes
// CDI flux r_a = gamma [eps G_a phi - A_a(phi (1 - phi) n_a)]  (Table 1)
// mass flux m_a = rho_a u_a - (rho1 - rho2) r_a  (CDI; r = 0 otherwise)
// nrm(a, lower): component a of the normal at c (lower = false) or at the
// cell c - e_a reads (lower = true)
template <typename T, int DIM, typename N>
__device__ __forceinline__ void op_face_n(const Phys& P, const Cell& C, const T* __restrict__ phi, N nrm,
                                          const T* __restrict__ u0, const T* __restrict__ u1,
                                          const T* __restrict__ u2, T* __restrict__ r0, T* __restrict__ r1,
                                          T* __restrict__ r2, T* __restrict__ m0, T* __restrict__ m1,
                                          T* __restrict__ m2) {
    const T* u[3] = {u0, u1, u2};
    T* r[3] = {r0, r1, r2};
    T* m[3] = {m0, m1, m2};
    const unsigned c = C.id;
    const T f = ld(phi, c);
    const bool cdi = P.model == MODEL_CDI;
    const T drho = T(P.rho1 - P.rho2);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const unsigned cm = C.off(a, -1);
        const T fm = ld(phi, cm);
        const T rho_f = T(0.5) * (rho_of(P, fm) + rho_of(P, f));
        const bool shut = C.wall(a, -1);   // face on a wall: no flux
        T ra = T(0);
        if (cdi) {
            const T wm = fm * (T(1) - fm) * nrm(a, true);
            const T wc = f * (T(1) - f) * nrm(a, false);
            ra = shut ? T(0) : T(P.gamma) * (T(P.eps) * ((f - fm) * T(P.inv_h)) - T(0.5) * (wm + wc));
            st(r[a], c, ra);
        }
        st(m[a], c, shut ? T(0) : rho_f * ld(u[a], c) - drho * ra);
    }
}

// the same with the normals read from the stored n_a
template <typename T, int DIM>
__device__ __forceinline__ void op_face(const Phys& P, const Cell& C, const T* __restrict__ phi,
                                                const T* __restrict__ n0, const T* __restrict__ n1,
                                                const T* __restrict__ n2, const T* __restrict__ u0,
                                                const T* __restrict__ u1, const T* __restrict__ u2,
                                                T* __restrict__ r0, T* __restrict__ r1,
                                                T* __restrict__ r2, T* __restrict__ m0,
                                                T* __restrict__ m1, T* __restrict__ m2) {
    const T* n[3] = {n0, n1, n2};
    auto nrm = [&](int a, bool lower) { return ld(n[a], lower ? C.off(a, -1) : C.id); };
    op_face_n<T, DIM>(P, C, phi, nrm, u0, u1, u2, r0, r1, r2, m0, m1, m2);
}

// ------------------------------------------------------------------ field access
// The phase and momentum bodies read their neighbour values through an
// accessor: G (global memory, a Cell's offsets) here, or one that serves the
// in-plane neighbours of a z-plane from an LDS tile.  f is one of the field
// ids below; a, b are axes and s, t in {-1, +1}.
enum { F_PHI = 0, F_U0, F_U1, F_U2, F_M0, F_M1, F_M2, F_MU, F_KAP, F_R0, F_R1, F_R2, F_NF };

// the axis a face field is normal to (u_a, m_a, r_a), or -1 for a cell field
__device__ __forceinline__ int normal_of(int f) {
    return (f >= F_U0 && f <= F_U2) ? f - F_U0
         : (f >= F_M0 && f <= F_M2) ? f - F_M0
         : (f >= F_R0 && f <= F_R2) ? f - F_R0 : -1;
}

template <typename T>
struct GAcc {
    const Cell& C;
    const T* p[F_NF];
    // A face field normal to axis n, read dn faces above the cell's own lower
    // n-face (dn in -1..1), is 0 on a wall face: the lower face of the first
    // cell (dn = 0 there, dn = -1 from the second cell), the upper face of
    // the last (dn = +1).  (From the first cell dn = -1 is past the wall; it
    // feeds only the wall face's own outputs, which are written as 0.)
    __device__ __forceinline__ bool shut(int f, int dn) const {
        const int n = normal_of(f);
        if (n < 0) return false;
        if (dn > 0) return C.wall(n, 1);
        return C.wall(n, -1) || (dn < 0 && C.second(n));
    }
    // (the load is unconditional and the wall test a select: the loads of a
    // body stay free to be issued together)
    __device__ __forceinline__ T c(int f) const {
        const T v = ld(p[f], C.id);
        return shut(f, 0) ? T(0) : v;
    }
    __device__ __forceinline__ T nb(int f, int a, int s) const {
        const T v = ld(p[f], C.off(a, s));
        return shut(f, a == normal_of(f) ? s : 0) ? T(0) : v;
    }
    __device__ __forceinline__ T nb2(int f, int a, int s, int b, int t) const {
        const int n = normal_of(f);
        const T v = ld(p[f], C.off2(a, s, b, t));
        return shut(f, (a == n ? s : 0) + (b == n ? t : 0)) ? T(0) : v;
    }
    // the cell's own value of a field outside the table (the RK state y_n
    // and accumulator of the phase update)
    __device__ __forceinline__ T own(const T* __restrict__ q, int) const { return ld(q, C.id); }
};

// ------------------------------------------------------------------ phase field
// dphi/dt = -D(u A phi) + g   (Eq. 1), g of Table 1; then the RK4 update.
// KM, KF: the model and force when the caller knows them at compile time
// (-1: read from P)
template <typename T, int DIM, typename Acc, int KM = -1>
__device__ __forceinline__ void op_phase_g(const Phys& P, const RKArgs& rk, const Cell& C, const Acc& G,
                                           const T* __restrict__ yn, T* __restrict__ acc,
                                           T* __restrict__ ynext, int* __restrict__ flags) {
    const int model = KM >= 0 ? KM : P.model;
    const unsigned c = C.id;
    const T f = G.c(F_PHI);
    const T ih = T(P.inv_h);
    T adv = T(0), g = T(0), lap = T(0), gg = T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const T fp = G.nb(F_PHI, a, 1), fm = G.nb(F_PHI, a, -1);
        const T jhi = G.nb(F_U0 + a, a, 1) * (T(0.5) * (f + fp));
        const T jlo = G.c(F_U0 + a) * (T(0.5) * (fm + f));
        adv += (jhi - jlo) * ih;
        if (model == MODEL_CDI) {
            g += (G.nb(F_R0 + a, a, 1) - G.c(F_R0 + a)) * ih;
        } else {
            lap += ((fp - f) * ih - (f - fm) * ih) * ih;
            const T ga = (fp - fm) * T(0.5 * P.inv_h);
            gg += ga * ga;
        }
    }
    if (model != MODEL_CDI) {
        const T base = T(P.eps) * lap - dpsi(f) / T(P.eps);
        const T curv = (model == MODEL_SB) ? T(P.eps) * sqrt(gg) * G.c(F_KAP)
                                             : f * (T(1) - f) * G.c(F_KAP);
        g = T(P.gamma) * (base + curv);
    }
    const T k = -adv + g;
    if (rk.eval_only) {
        stn(ynext, c, k);
        return;
    }
    const T y0 = G.own(yn, 0);
    const T a_new = (rk.stage == 0 ? y0 : G.own(acc, 1)) + T(rk.wacc) * k;
    stn(acc, c, a_new);
    if (rk.stage < 3) stn(ynext, c, y0 + T(rk.wnext) * k);
    else if (!isfinite(a_new)) flags[0] = 1;
}

template <typename T, int DIM>
__device__ __forceinline__ void op_phase(const Phys& P, const RKArgs& rk, const Cell& C,
                                                 const T* __restrict__ phi,
                                                 const T* __restrict__ u0, const T* __restrict__ u1,
                                                 const T* __restrict__ u2, const T* __restrict__ r0,
                                                 const T* __restrict__ r1, const T* __restrict__ r2,
                                                 const T* __restrict__ kappa,
                                                 const T* __restrict__ yn, T* __restrict__ acc,
                                                 T* __restrict__ ynext, int* __restrict__ flags) {
    const GAcc<T> G{C, {phi, u0, u1, u2, nullptr, nullptr, nullptr, nullptr, kappa, r0, r1, r2}};
    op_phase_g<T, DIM>(P, rk, C, G, yn, acc, ynext, flags);
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
template <typename T, int DIM, typename Acc, int KF = -1>
__device__ __forceinline__ void op_momentum_g(const Phys& P, const Cell& C, const Acc& G, T* __restrict__ f0,
                                              T* __restrict__ f1, T* __restrict__ f2, T* __restrict__ F0,
                                              T* __restrict__ F1, T* __restrict__ F2) {
    const int force = KF >= 0 ? KF : P.force;
    T* fs[3] = {f0, f1, f2};
    T* Fo[3] = {F0, F1, F2};
    const unsigned c = C.id;
    const T ih = T(P.inv_h);
    const T v2 = T(P.visc2), dv = T(P.visc1 - P.visc2);
    const T f = G.c(F_PHI);
    const T clc = clamp01(P, f);
    // h D m at c, shared by the faces of c
    T dmc = T(0);
#pragma unroll
    for (int b = 0; b < DIM; ++b) dmc += G.nb(F_M0 + b, b, 1) - G.c(F_M0 + b);
    // The sums below are the terms of N_a, V_a and F_a with the factors 1/2,
    // 1/4 and 1/h of the averages and differences taken out: N_a = Nh / h,
    // V_a = Vh2 / h^2, F_a = Fh / h.
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const T fm = G.nb(F_PHI, a, -1);
        const T clm = clamp01(P, fm);
        const T uac = G.c(F_U0 + a), uap = G.nb(F_U0 + a, a, 1), uam = G.nb(F_U0 + a, a, -1);
        // ---- advection: fluxes are products of two-point sums (x 1/4)
        const T mac = G.c(F_M0 + a), mam = G.nb(F_M0 + a, a, -1);
        T adv4 = (mac + G.nb(F_M0 + a, a, 1)) * (uac + uap) - (mam + mac) * (uam + uac);
        T dmm = mac - mam;      // h D m at c - e_a
        // ---- viscous stress (x 1/h^2); edge viscosity v2 + dv/4 (sum of four clamped phi)
        T vh2 = T(2) * ((v2 + dv * clc) * (uap - uac) - (v2 + dv * clm) * (uac - uam));
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            if (b == a) continue;
            const T uapb = G.nb(F_U0 + a, b, 1), uamb = G.nb(F_U0 + a, b, -1);
            const T mbc = G.c(F_M0 + b), mbm = G.nb(F_M0 + b, a, -1), mbmp = G.nb2(F_M0 + b, a, -1, b, 1);
            adv4 += (G.nb(F_M0 + b, b, 1) + mbmp) * (uac + uapb) - (mbc + mbm) * (uamb + uac);
            dmm += mbmp - mbm;
            const T cc = clc + clm;
            const T e_hi = v2 + T(0.25) * dv * (cc + clamp01(P, G.nb(F_PHI, b, 1)) + clamp01(P, G.nb2(F_PHI, a, -1, b, 1)));
            const T e_lo = v2 + T(0.25) * dv * (cc + clamp01(P, G.nb(F_PHI, b, -1)) + clamp01(P, G.nb2(F_PHI, a, -1, b, -1)));
            vh2 += e_hi * ((uapb - uac) + (G.nb(F_U0 + b, b, 1) - G.nb2(F_U0 + b, a, -1, b, 1))) -
                   e_lo * ((uac - uamb) + (G.c(F_U0 + b) - G.nb(F_U0 + b, a, -1)));
        }
        const T nh = T(0.25) * adv4 - T(0.5) * uac * (dmm + dmc);
        // ---- surface tension (x 1/h)
        const T gh = f - fm;
        T fh;
        if (force == FORCE_EB) {
            fh = T(0.5) * (G.nb(F_MU, a, -1) + G.c(F_MU)) * gh;
        } else if (force == FORCE_CSF) {
            fh = T(0.5 * P.sigma) * (G.nb(F_KAP, a, -1) + G.c(F_KAP)) * gh;
        } else {
            fh = T(0.25 * P.sigma_hat) * (G.nb(F_KAP, a, -1) + G.c(F_KAP)) *
                 (fm * (T(1) - fm) + f * (T(1) - f)) * gh;
        }
        const bool shut = C.wall(a, -1);   // face on a wall: f* = 0
        if (Fo[0]) stn(Fo[a], c, shut ? T(0) : fh * ih);
        const T rho_f = T(P.rho2) + T(0.5 * (P.rho1 - P.rho2)) * (clm + clc);
        stn(fs[a], c, shut ? T(0) : quot((fh - nh) * ih + vh2 * (ih * ih), rho_f));
    }
}

template <typename T, int DIM>
__device__ __forceinline__ void op_momentum(const Phys& P, const Cell& C, const T* __restrict__ phi, const T* __restrict__ u0,
    const T* __restrict__ u1, const T* __restrict__ u2, const T* __restrict__ m0,
    const T* __restrict__ m1, const T* __restrict__ m2, const T* __restrict__ mu,
    const T* __restrict__ kappa, T* __restrict__ f0, T* __restrict__ f1, T* __restrict__ f2,
    T* __restrict__ F0, T* __restrict__ F1, T* __restrict__ F2) {
    const GAcc<T> G{C, {phi, u0, u1, u2, m0, m1, m2, mu, kappa, nullptr, nullptr, nullptr}};
    op_momentum_g<T, DIM>(P, C, G, f0, f1, f2, F0, F1, F2);
}

// ------------------------------------------------------------------ D f* (FP64)
template <typename T, int DIM>
__device__ __forceinline__ double op_div(const Phys& P, const Cell& C, const T* __restrict__ f0,
                                         const T* __restrict__ f1, const T* __restrict__ f2,
                                         double* __restrict__ b) {
    const T* fs[3] = {f0, f1, f2};
    const unsigned c = C.id;
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double hi = C.wall(a, 1) ? 0.0 : (double)ld(fs[a], C.off(a, 1));
        const double lo = C.wall(a, -1) ? 0.0 : (double)ld(fs[a], c);
        s += (hi - lo) * P.inv_h;
    }
    b[c] = s;
    return s;
}

// ------------------------------------------------------------------ projection
// du_a/dt = f*_a - beta_a G_a p, then the RK4 update of u_a.
template <typename T, int DIM>
__device__ __forceinline__ void op_project(const Phys& P, const RKArgs& rk, const Cell& C,
                                                   const T* __restrict__ phi,
                                                   const double* __restrict__ p,
                                                   const T* __restrict__ f0, const T* __restrict__ f1,
                                                   const T* __restrict__ f2, const T* yn0,
                                                   const T* yn1, const T* yn2, T* acc0, T* acc1,
                                                   T* acc2, T* nx0, T* nx1, T* nx2,
                                                   int* __restrict__ flags) {
    const T* fs[3] = {f0, f1, f2};
    const T* yn[3] = {yn0, yn1, yn2};
    T* acc[3] = {acc0, acc1, acc2};
    T* nx[3] = {nx0, nx1, nx2};
    const unsigned c = C.id;
    const T f = ld(phi, c);
    const double pc = ld(p, c);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const unsigned cm = C.off(a, -1);
        const double rho_f = 0.5 * ((double)rho_of(P, ld(phi, cm)) + (double)rho_of(P, f));
        const double gp = (pc - ld(p, cm)) * P.inv_h;
        const T k = C.wall(a, -1) ? T(0) : T((double)ld(fs[a], c) - gp / rho_f);   // wall face: u stays
        if (rk.eval_only) {
            stn(nx[a], c, k);
            continue;
        }
        const T y0 = ld(yn[a], c);
        const T a_new = (rk.stage == 0 ? y0 : ld(acc[a], c)) + T(rk.wacc) * k;
        stn(acc[a], c, a_new);
        if (rk.stage < 3) stn(nx[a], c, y0 + T(rk.wnext) * k);
        else if (!isfinite(a_new)) flags[0] = 1;
    }
}

// ------------------------------------------------------------------ initial droplet
// phi = [1 + tanh(s/2eps)]/2, s = (1 - q)/|grad q| with q = |x / a| (first-order
// signed distance to the ellipse/ellipsoid, exact for circles and spheres);
// the nearest periodic image along periodic axes, none across walled ones
template <typename T, int DIM>
__device__ __forceinline__ void op_init_droplet(const Dims& d, const Cell& C, double h, double eps, double c0,
                                                        double c1, double c2, double a0, double a1,
                                                        double a2, T* __restrict__ phi) {
    const double cen[3] = {c0, c1, c2}, ax[3] = {a0, a1, a2};
    const int v[3] = {C.i, C.j, C.k};
    const int nn[3] = {d.nx, d.ny, d.nz};
    double q2 = 0.0, g2 = 0.0, amin = ax[0];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double L = nn[a] * h;
        double x = (v[a] + 0.5) * h - cen[a];
        if (!((d.walls >> a) & 1)) x -= L * floor(x / L + 0.5);
        q2 += (x / ax[a]) * (x / ax[a]);
        g2 += x * x / (ax[a] * ax[a] * ax[a] * ax[a]);
        amin = fmin(amin, ax[a]);
    }
    const double q = sqrt(q2);
    const double s = (q2 == 0.0) ? amin : (1.0 - q) * q / sqrt(g2);
    phi[C.id] = T(0.5 * (1.0 + tanh(s / (2.0 * eps))));
}

// ------------------------------------------------------------------ diagnostics
// Per-block partials: [0] sum phi, [1] KE density, [2] SE density, [3] sum p
// (phi>0.99), [4] count in, [5] sum p (phi<0.01), [6] count out; maxima:
// [7] |u_cell|, [8] |D u|, [9] -min phi, [10] max phi.
constexpr int ND_SUM = 7, ND_MAX = 4;

template <typename T, int DIM>
__device__ __forceinline__ void op_diag(const Phys& P, const Cell& C, const T* __restrict__ phi,
                                        const T* __restrict__ u0, const T* __restrict__ u1,
                                        const T* __restrict__ u2, const double* __restrict__ p,
                                        double (&s)[ND_SUM], double (&mx)[ND_MAX]) {
    const T* u[3] = {u0, u1, u2};
    const unsigned c = C.id;
    const double f = (double)phi[c];
    double sp2 = 0.0, kin = 0.0, g2 = 0.0, div = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const unsigned cp = C.off(a, 1), cm = C.off(a, -1);
        const double ua = C.wall(a, -1) ? 0.0 : (double)u[a][c];
        const double uap = C.wall(a, 1) ? 0.0 : (double)u[a][cp];
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

}  // namespace tpf
