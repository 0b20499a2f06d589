// Reverse-mode derivative of the step: the transpose of every stage operator,
// hand written, plus the RK4 reverse sweep over a tape of stage states.  It
// covers 2D and 3D grids, the three phase-field models of Table 1 and the
// three surface forces (Eq. 4, CSF, Eq. 11).
//
// One stage maps y = (phi, u) to (dphi/dt, du/dt) (Eq. 1 with g of Table 1;
// momentum with the chosen force; projection).  Given the cotangents
// (l_dphi, l_du) of its outputs, stage_vjp returns the cotangents of phi and
// u and adds those of sigma and eps.  Discrete transposes used throughout
// (periodic grid, plain sums as inner products):
//   D^T = -G,  G^T = -D,  A_a^T q[c] = (q[c] + q[c+e_a])/2,  C_a^T = -C_a,
//   L^T = L, and the viscous operator V(eta, .) is symmetric.
// Projection: du = f* - beta G p with D(beta G p) = D f*.  With
//   q solving D(beta G q) = D(beta l_du):
//   l_f* = l_du - G q,   l_rho_a = -beta_a l_f*_a du_a.
// Curvature kappa = -sum_a C_a n_a (Eq. 3) gives l_n_a += C_a l_kappa.
// All cotangents are FP64 whatever the state precision T.
#include <cmath>
#include <cstring>

#include "tpf_internal.hpp"

namespace tpf {

struct AdjFields {
    const double* ldphi;   // cotangent of dphi/dt (cell)
    const double* ldu[3];  // cotangent of du/dt (faces)
    const double* p;       // stage pressure
    const double* q;       // adjoint pressure
    double* lX[3];         // cotangent of X = -N + V + F (faces)
    double* lrho[3];       // cotangent of the face density
    double* lr[3];         // cotangent of the CDI flux (faces)
    double* lg[3];         // cotangent of the central gradient g (cells)
    double* lmu;           // cotangent of mu (cells; energy-based force)
    double* ldm;           // cotangent of D m (cells)
    double* leta;          // cotangent of the viscosity (cells)
    double* lkap;          // cotangent of kappa (cells)
    double* dm;            // D m of the forward stage (cells)
    double* outphi;        // stage cotangent of phi (cells)
    double* outu[3];       // stage cotangent of u (faces)
};

template <typename T>
struct Fwd {
    const T* phi;
    const T* u[3];
    const T* n[3];
    const T* mu;
    const T* kappa;
    const T* m[3];
    const T* f[3];
};

__device__ __forceinline__ double clamp_slope(const Phys& P, double f) {
    return (!P.clamp || (f >= 0.0 && f <= 1.0)) ? 1.0 : 0.0;
}
__device__ __forceinline__ double rho_d(const Phys& P, double f) {
    const double g = P.clamp ? fmin(fmax(f, 0.0), 1.0) : f;
    return P.rho2 + (P.rho1 - P.rho2) * g;
}
__device__ __forceinline__ double eta_d(const Phys& P, double f) {
    const double g = P.clamp ? fmin(fmax(f, 0.0), 1.0) : f;
    return P.visc2 + (P.visc1 - P.visc2) * g;
}
__device__ __forceinline__ double wfun(double f) { return f * (1.0 - f); }
// psi''(phi) = 1 - 6 phi + 6 phi^2  (Eq. 2)
__device__ __forceinline__ double d2psi(double f) { return 1.0 - 6.0 * f + 6.0 * f * f; }
__device__ __forceinline__ bool needs_kappa(const Phys& P) {
    return P.model != MODEL_CDI || P.force != FORCE_EB;
}
// the cell at C + (di, dj, dk), each shift in {-1, 0, 1}
__device__ __forceinline__ Cell shifted(const Dims& d, const Cell& C, int di, int dj, int dk) {
    return make_cell(d, wrapc(C.i + di, d.nx), wrapc(C.j + dj, d.ny), wrapc(C.k + dk, d.nz));
}
__device__ __forceinline__ Cell shifted_ab(const Dims& d, const Cell& C, int a, int sa, int b, int sb) {
    int s[3] = {0, 0, 0};
    s[a] += sa;
    s[b] += sb;
    return shifted(d, C, s[0], s[1], s[2]);
}

// ------------------------------------------------------------------ rhs of the adjoint solve
// b = D(beta l_du) in FP64, block sums for the mean
template <typename T, int DIM>
__global__ __launch_bounds__(BLOCK) void k_adj_rhs(Dims d, Phys P, const T* __restrict__ phi, AdjFields A,
                                                   double* __restrict__ b, double* __restrict__ partials) {
    Cell C;
    double v[1] = {0.0};
    if (cell_of_thread(d, C)) {
        const unsigned c = C.id;
        const double rc = rho_d(P, (double)phi[c]);
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const unsigned cp = C.off(a, 1), cm = C.off(a, -1);
            const double hi = A.ldu[a][cp] / (0.5 * (rc + rho_d(P, (double)phi[cp])));
            const double lo = A.ldu[a][c] / (0.5 * (rho_d(P, (double)phi[cm]) + rc));
            s += (hi - lo) * P.inv_h;
        }
        b[c] = s;
        v[0] = s;
    }
    block_partials<1>(v, partials);
}

// ------------------------------------------------------------------ P1: projection and f* = X beta
template <typename T, int DIM>
__global__ __launch_bounds__(BLOCK) void k_adj_proj(Dims d, Phys P, Fwd<T> F, AdjFields A) {
    Cell C;
    if (!cell_of_thread(d, C)) return;
    const unsigned c = C.id;
    const double fc = (double)F.phi[c];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const unsigned cm = C.off(a, -1);
        const double beta = 1.0 / (0.5 * (rho_d(P, (double)F.phi[cm]) + rho_d(P, fc)));
        const double lf = A.ldu[a][c] - (A.q[c] - A.q[cm]) * P.inv_h;
        const double du = (double)F.f[a][c] - beta * (A.p[c] - A.p[cm]) * P.inv_h;
        A.lX[a][c] = lf * beta;
        A.lrho[a][c] = -beta * lf * du;
    }
}

// ------------------------------------------------------------------ P2: cell cotangents
// lambda_mu = A^T(l_X G phi) (energy-based force); lambda_kappa from the CSF
// or LCSF force and from the SB or ISODI right-hand side; lambda_Dm =
// A^T(l_X u); lambda_eta from the symmetric viscous form; D m of the forward
// stage; parameter partials (sigma, eps) of the force and of g.
template <typename T, int DIM>
__global__ __launch_bounds__(BLOCK) void k_adj_cell1(Dims d, Phys P, Fwd<T> F, AdjFields A,
                                                     double* __restrict__ partials) {
    Cell C;
    double v[2] = {0.0, 0.0};
    if (cell_of_thread(d, C)) {
        const unsigned c = C.id;
        const double ih = P.inv_h;
        auto ph = [&](unsigned q) { return (double)F.phi[q]; };
        auto U = [&](int a, unsigned q) { return (double)F.u[a][q]; };
        const double fc = ph(c);
        const bool lcsf = P.force == FORCE_LCSF;
        double sgx = 0.0, sgxw = 0.0, ldm = 0.0, lap = 0.0, gg = 0.0, dmf = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const unsigned cp = C.off(a, 1), cm = C.off(a, -1);
            const double fp = ph(cp), fm = ph(cm);
            const double g_lo = (fc - fm) * ih, g_hi = (fp - fc) * ih;
            sgx += 0.5 * (A.lX[a][c] * g_lo + A.lX[a][cp] * g_hi);
            ldm += 0.5 * (A.lX[a][c] * U(a, c) + A.lX[a][cp] * U(a, cp));
            lap += (g_hi - g_lo) * ih;
            const double ga = (fp - fm) * (0.5 * ih);
            gg += ga * ga;
            dmf += ((double)F.m[a][cp] - (double)F.m[a][c]) * ih;
            if (P.force != FORCE_EB) {
                // face (c, a): F_a = sigma A(kappa) G phi  or  sigma_hat A(kappa) A(w) G phi
                const double kf = 0.5 * ((double)F.kappa[cm] + (double)F.kappa[c]);
                const double w_lo = 0.5 * (wfun(fm) + wfun(fc));
                if (lcsf) {
                    const double w_hi = 0.5 * (wfun(fc) + wfun(fp));
                    sgxw += 0.5 * (A.lX[a][c] * w_lo * g_lo + A.lX[a][cp] * w_hi * g_hi);
                    v[0] += 6.0 * A.lX[a][c] * kf * w_lo * g_lo;
                } else {
                    v[0] += A.lX[a][c] * kf * g_lo;
                }
            }
        }
        // viscous: d<w, V(eta, u)>/d eta_c with w = l_X.  Cell part: the normal
        // stresses; edge part: each edge viscosity is the mean of the four
        // cells around the edge, and the edges of cell c in the (a, b) plane
        // are the lower (a, b) corners of c, c + e_a, c + e_b, c + e_a + e_b
        double leta = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const unsigned cp = C.off(a, 1);
            const double su = (U(a, cp) - U(a, c)) * ih;
            const double sw = (A.lX[a][cp] - A.lX[a][c]) * ih;
            leta -= 2.0 * su * sw;
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
            for (int b = a + 1; b < DIM; ++b)
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const Cell Q = shifted_ab(d, C, a, k & 1, b, k >> 1);
                    const unsigned q = Q.id, qmb = Q.off(b, -1), qma = Q.off(a, -1);
                    const double gu = (U(a, q) - U(a, qmb)) * ih + (U(b, q) - U(b, qma)) * ih;
                    const double gw = (A.lX[a][q] - A.lX[a][qmb]) * ih + (A.lX[b][q] - A.lX[b][qma]) * ih;
                    leta -= 0.25 * gu * gw;
                }
        A.ldm[c] = ldm;
        A.leta[c] = leta;
        A.dm[c] = dmf;
        const double dp = (double)dpsi(fc);
        if (P.force == FORCE_EB) {
            // mu = (sigma_hat / eps) psi'(phi) - sigma_hat eps L phi,  sigma_hat = 6 sigma
            A.lmu[c] = sgx;
            v[0] += sgx * 6.0 * (dp / P.eps - P.eps * lap);
            v[1] += sgx * (-P.sigma_hat * dp / (P.eps * P.eps) - P.sigma_hat * lap);
        }
        if (needs_kappa(P)) {
            const double ld = A.ldphi[c];
            double lk = 0.0;
            if (P.force == FORCE_CSF) lk += P.sigma * sgx;
            if (lcsf) lk += P.sigma_hat * sgxw;
            if (P.model == MODEL_SB) lk += P.gamma * P.eps * sqrt(gg) * ld;
            if (P.model == MODEL_ISODI) lk += P.gamma * wfun(fc) * ld;
            A.lkap[c] = lk;
        }
        if (P.model != MODEL_CDI) {
            // g = gamma [eps L phi - psi'(phi)/eps + curv], curv = eps |C phi| kappa (SB)
            // or phi (1 - phi) kappa (ISODI)
            double de = lap + dp / (P.eps * P.eps);
            if (P.model == MODEL_SB) de += sqrt(gg) * (double)F.kappa[c];
            v[1] += A.ldphi[c] * P.gamma * de;
        }
    }
    block_partials<2>(v, partials);
}

// ------------------------------------------------------------------ P3: face cotangents
// advection (l_N = -l_X), viscous V(eta, l_X), mass flux, phase-field flux
template <typename T, int DIM>
__global__ __launch_bounds__(BLOCK) void k_adj_face(Dims d, Phys P, Fwd<T> F, AdjFields A,
                                                    double* __restrict__ partials) {
    Cell C;
    double v[2] = {0.0, 0.0};
    if (cell_of_thread(d, C)) {
        const unsigned c = C.id;
        const double ih = P.inv_h;
        auto ph = [&](unsigned q) { return (double)F.phi[q]; };
        auto U = [&](int a, unsigned q) { return (double)F.u[a][q]; };
        auto M = [&](int a, unsigned q) { return (double)F.m[a][q]; };
        auto lN = [&](int a, unsigned q) { return -A.lX[a][q]; };
        auto W = [&](int e, unsigned q) { return A.lX[e][q]; };
        auto eta = [&](unsigned q) { return eta_d(P, ph(q)); };
        const double fc = ph(c);
        const double drho = P.rho1 - P.rho2;
        const double eta_c = eta(c);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const unsigned cp = C.off(a, 1), cm = C.off(a, -1);
            const double eta_m = eta(cm);
            double lm = 0.0, lu = 0.0;
            // cell terms Phi_aa(q) = Mc(q) Uc(q) at q = c and q = c - e_a
            {
                const double lphi_c = (lN(a, c) - lN(a, cp)) * ih;     // Phi_aa(c)
                const double lphi_m = (lN(a, cm) - lN(a, c)) * ih;     // Phi_aa(c - e_a)
                const double Uc_c = 0.5 * (U(a, c) + U(a, cp)), Uc_m = 0.5 * (U(a, cm) + U(a, c));
                const double Mc_c = 0.5 * (M(a, c) + M(a, cp)), Mc_m = 0.5 * (M(a, cm) + M(a, c));
                lm += 0.5 * (lphi_c * Uc_c + lphi_m * Uc_m);
                lu += 0.5 * (lphi_c * Mc_c + lphi_m * Mc_m);
            }
            double V = (2.0 * eta_c * (W(a, cp) - W(a, c)) * ih - 2.0 * eta_m * (W(a, c) - W(a, cm)) * ih) * ih;
#pragma unroll
            for (int b = 0; b < DIM; ++b) {
                if (b == a) continue;
                const unsigned cpb = C.off(b, 1), cmb = C.off(b, -1);
                // edge terms.  Edge E(q) is the lower corner of q in the (a, b)
                // plane.  Phi_ba(E(q)) = Mb_b(E(q)) Ub_a(E(q)) enters N_a[q - e_b]
                // with +1/h and N_a[q] with -1/h; Phi_ab(E(q)) = Mb_a(E(q)) Ub_b(E(q))
                // enters N_b[q - e_a] with +1/h and N_b[q] with -1/h.
                //   Mb_b(E(q)) = (m_b[q] + m_b[q - e_a]) / 2,  Ub_a(E(q)) = (u_a[q - e_b] + u_a[q]) / 2
                //   Mb_a(E(q)) = (m_a[q] + m_a[q - e_b]) / 2,  Ub_b(E(q)) = (u_b[q - e_a] + u_b[q]) / 2
                const unsigned cpb_ma = C.off2(b, 1, a, -1);           // c + e_b - e_a
                {
                    // u_a[c] sits in Ub_a(E(c)) and Ub_a(E(c + e_b))
                    const double lP_c = (lN(a, cmb) - lN(a, c)) * ih;      // Phi_ba(E(c))
                    const double lP_p = (lN(a, c) - lN(a, cpb)) * ih;      // Phi_ba(E(c + e_b))
                    const double Mb_c = 0.5 * (M(b, c) + M(b, cm));
                    const double Mb_p = 0.5 * (M(b, cpb) + M(b, cpb_ma));
                    lu += 0.5 * (lP_c * Mb_c + lP_p * Mb_p);
                    // m_a[c] sits in Mb_a(E(c)) and Mb_a(E(c + e_b))
                    const double lQ_c = (lN(b, cm) - lN(b, c)) * ih;       // Phi_ab(E(c))
                    const double lQ_p = (lN(b, cpb_ma) - lN(b, cpb)) * ih; // Phi_ab(E(c + e_b))
                    const double Ub_c = 0.5 * (U(b, cm) + U(b, c));
                    const double Ub_p = 0.5 * (U(b, cpb_ma) + U(b, cpb));
                    lm += 0.5 * (lQ_c * Ub_c + lQ_p * Ub_p);
                }
                // viscous V_a(eta, l_X)[c], edge part (the operator is symmetric)
                {
                    const unsigned cmamb = C.off2(a, -1, b, -1);
                    const double eta_hi = 0.25 * (eta_c + eta_m + eta(cpb) + eta(cpb_ma));
                    const double eta_lo = 0.25 * (eta(cmb) + eta(cmamb) + eta_c + eta_m);
                    const double hi = eta_hi * ((W(a, cpb) - W(a, c)) * ih + (W(b, cpb) - W(b, cpb_ma)) * ih);
                    const double lo = eta_lo * ((W(a, c) - W(a, cmb)) * ih + (W(b, c) - W(b, cm)) * ih);
                    V += (hi - lo) * ih;
                }
            }
            lu += V;
            // - u_a A_a(D m):  l_u += l_X A_a(Dm);  l_m_a += -G_a(l_Dm)
            lu += A.lX[a][c] * 0.5 * (A.dm[cm] + A.dm[c]);
            lm += -(A.ldm[c] - A.ldm[cm]) * ih;
            // mass flux m_a = rho_a u_a - (rho1 - rho2) r_a
            const double rho_f = 0.5 * (rho_d(P, ph(cm)) + rho_d(P, fc));
            lu += rho_f * lm;
            A.lrho[a][c] += U(a, c) * lm;
            // phase field: J_a = u_a A_a phi, dphi = -D J (+ D r for CDI)
            const double lJ = (A.ldphi[c] - A.ldphi[cm]) * ih;
            lu += lJ * 0.5 * (ph(cm) + fc);
            if (P.model == MODEL_CDI) {
                const double lra = -drho * lm - lJ;
                A.lr[a][c] = lra;
                // r_a = gamma [eps G_a phi - ...]:  d r / d eps = gamma G_a phi
                v[1] += lra * P.gamma * (fc - ph(cm)) * ih;
            }
            A.outu[a][c] = lu;
        }
    }
    block_partials<2>(v, partials);
}

// ------------------------------------------------------------------ P4: phi cotangent (all but C^T l_g)
template <typename T, int DIM>
__global__ __launch_bounds__(BLOCK) void k_adj_cell2(Dims d, Phys P, Fwd<T> F, AdjFields A) {
    Cell C;
    if (!cell_of_thread(d, C)) return;
    const unsigned c = C.id;
    const double ih = P.inv_h;
    auto ph = [&](unsigned q) { return (double)F.phi[q]; };
    auto kap = [&](unsigned q) { return (double)F.kappa[q]; };
    auto mu = [&](unsigned q) { return (double)F.mu[q]; };
    const bool cdi = P.model == MODEL_CDI, kap_on = needs_kappa(P);
    const double fc = ph(c), wc = wfun(fc);
    const double ld = A.ldphi[c];
    double lphi = 0.0, lrho_c = 0.0, llap_mu = 0.0, llap_d = 0.0, lw = 0.0, gg = 0.0;
    double lwn[3] = {0.0, 0.0, 0.0}, g[3] = {0.0, 0.0, 0.0}, ln[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const unsigned cp = C.off(a, 1), cm = C.off(a, -1);
        const double fp = ph(cp), fm = ph(cm);
        const double* lX = A.lX[a];
        lrho_c += 0.5 * (A.lrho[a][c] + A.lrho[a][cp]);
        // surface force F_a = coef_a G_a phi: G_a^T of l_X coef_a
        if (P.force == FORCE_EB) {
            lphi += (lX[c] * 0.5 * (mu(cm) + mu(c)) - lX[cp] * 0.5 * (mu(c) + mu(cp))) * ih;
            llap_mu += ((A.lmu[cp] - A.lmu[c]) * ih - (A.lmu[c] - A.lmu[cm]) * ih) * ih;
        } else {
            const double k_lo = 0.5 * (kap(cm) + kap(c)), k_hi = 0.5 * (kap(c) + kap(cp));
            double co_lo, co_hi;
            if (P.force == FORCE_CSF) {
                co_lo = P.sigma * k_lo;
                co_hi = P.sigma * k_hi;
            } else {
                const double w_lo = 0.5 * (wfun(fm) + wc), w_hi = 0.5 * (wc + wfun(fp));
                co_lo = P.sigma_hat * k_lo * w_lo;
                co_hi = P.sigma_hat * k_hi * w_hi;
                // A_a^T of the cotangent of A_a(w)
                lw += 0.5 * (lX[c] * P.sigma_hat * k_lo * (fc - fm) * ih +
                             lX[cp] * P.sigma_hat * k_hi * (fp - fc) * ih);
            }
            lphi += (lX[c] * co_lo - lX[cp] * co_hi) * ih;
        }
        // phase-field flux J: A_a^T of l_J u_a
        const double lJ_c = (ld - A.ldphi[cm]) * ih, lJ_p = (A.ldphi[cp] - ld) * ih;
        lphi += 0.5 * (lJ_c * (double)F.u[a][c] + lJ_p * (double)F.u[a][cp]);
        if (cdi) {
            // CDI flux: gamma eps G_a phi, and - gamma A_a(w n_a)
            lphi += P.gamma * P.eps * (A.lr[a][c] - A.lr[a][cp]) * ih;
            lwn[a] = -P.gamma * 0.5 * (A.lr[a][c] + A.lr[a][cp]);
        } else {
            llap_d += ((A.ldphi[cp] - ld) * ih - (ld - A.ldphi[cm]) * ih) * ih;
        }
        g[a] = (fp - fm) * (0.5 * ih);
        gg += g[a] * g[a];
        // kappa = - sum_a C_a n_a
        if (kap_on) ln[a] += (A.lkap[cp] - A.lkap[cm]) * (0.5 * ih);
    }
    lphi += (P.rho1 - P.rho2) * clamp_slope(P, fc) * lrho_c;
    lphi += (P.visc1 - P.visc2) * clamp_slope(P, fc) * A.leta[c];
    if (P.force == FORCE_EB)
        lphi += (P.sigma_hat / P.eps) * d2psi(fc) * A.lmu[c] - P.sigma_hat * P.eps * llap_mu;
    if (P.force == FORCE_LCSF) lphi += (1.0 - 2.0 * fc) * lw;
    if (cdi) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            s += lwn[a] * (double)F.n[a][c];
            ln[a] += lwn[a] * wc;
        }
        lphi += (1.0 - 2.0 * fc) * s;
    } else {
        // g = gamma [eps L phi - psi'(phi)/eps + curv]
        lphi += P.gamma * (P.eps * llap_d - d2psi(fc) / P.eps * ld);
        if (P.model == MODEL_ISODI) lphi += P.gamma * kap(c) * (1.0 - 2.0 * fc) * ld;
    }
    // normals n = g / sqrt(g.g + delta^2): l_g = s (l_n - n (n . l_n))
    const double s = 1.0 / sqrt(gg + P.delta2);
    double dot = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) dot += g[a] * s * ln[a];
    double lg[3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) lg[a] = s * (ln[a] - g[a] * s * dot);
    // SB: curv = eps |g| kappa; its gradient g/|g| (taken as 0 where g = 0)
    if (P.model == MODEL_SB && gg > 0.0) {
        const double k = P.gamma * P.eps * kap(c) * ld / sqrt(gg);
#pragma unroll
        for (int a = 0; a < DIM; ++a) lg[a] += k * g[a];
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) A.lg[a][c] = lg[a];
    A.outphi[c] = lphi;
}

// ------------------------------------------------------------------ P5: C_a^T of l_g
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_adj_cell3(Dims d, Phys P, AdjFields A) {
    Cell C;
    if (!cell_of_thread(d, C)) return;
    const unsigned c = C.id;
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) s -= (A.lg[a][C.off(a, 1)] - A.lg[a][C.off(a, -1)]) * (0.5 * P.inv_h);
    A.outphi[c] += s;
}

// ------------------------------------------------------------------ small vector kernels
// out = a x + b y (any of x, y may alias out)
__global__ void k_axpby(long N, double a, const double* x, double b, const double* y,
                        double* out) {
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < N; q += (long)gridDim.x * blockDim.x)
        out[q] = a * x[q] + (y ? b * y[q] : 0.0);
}

// grad[k] += sum of the block partials of region k (fixed order)
__global__ __launch_bounds__(256) void k_adj_grad(int nb, long stride, const double* __restrict__ partials,
                                                  double* __restrict__ grad) {
    __shared__ double red[2][4];
    const int t = threadIdx.x;
    double v[2] = {0.0, 0.0};
    for (int k = 0; k < 2; ++k)
        for (int b = t; b < nb; b += 256) v[k] += partials[k * stride + b];
    for (int k = 0; k < 2; ++k)
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_down(v[k], o, 64);
    if ((t & 63) == 0) {
        red[0][t >> 6] = v[0];
        red[1][t >> 6] = v[1];
    }
    __syncthreads();
    if (t == 0)
        for (int k = 0; k < 2; ++k) grad[k] += (red[k][0] + red[k][1]) + (red[k][2] + red[k][3]);
}

template <typename T>
__global__ void k_copy_state(long N, const T* __restrict__ src, T* __restrict__ dst) {
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < N; q += (long)gridDim.x * blockDim.x)
        dst[q] = src[q];
}

static unsigned vb(long N) { return (unsigned)std::min<long>((N + 255) / 256, 8192); }

// ================================================================== host side

// Adjoint scratch: FP64 fields of adj_stride doubles each, in this order
// (S = 1 + dim state fields, dim face fields per group), then the two
// parameter-gradient accumulators.
struct AdjLayout {
    int lam;    // S: cotangent of y_{n+1} (phi, u)
    int acc;    // S: cotangent of y_n being accumulated
    int lk;     // S: cotangent of the stage derivative k_s
    int ly;     // S: cotangent of the stage input Y_s
    int lx, lrho, lr, lg;      // dim each
    int lmu, ldm, leta, lkap, dm;
    int pst;    // stage pressure (single-stage adjoint)
    int q;      // last adjoint pressure (warm start of the next adjoint solve)
    int count;
};
static AdjLayout adj_layout(int dim) {
    AdjLayout L;
    const int S = 1 + dim;
    int k = 0;
    L.lam = k; k += S;
    L.acc = k; k += S;
    L.lk = k; k += S;
    L.ly = k; k += S;
    L.lx = k; k += dim;
    L.lrho = k; k += dim;
    L.lr = k; k += dim;
    L.lg = k; k += dim;
    L.lmu = k++;
    L.ldm = k++;
    L.leta = k++;
    L.lkap = k++;
    L.dm = k++;
    L.pst = k++;
    L.q = k++;
    L.count = k;
    return L;
}

static double* af(tpf_ctx* c, int k) { return c->adj + (long)k * c->adj_stride; }
static double* grad_acc(tpf_ctx* c) { return af(c, adj_layout(c->dim).count); }

static tpf_status adjoint_supported(const tpf_ctx* c) {
    if (!c) { set_error("ctx is NULL"); return TPF_EINVAL; }
    if (!c->adj || adj_layout(c->dim).count != adj_fields(c->dim)) {
        set_error("the context was created without the adjoint scratch (tpf_params.adjoint = 1)");
        return TPF_EINVAL;
    }
    return TPF_OK;
}

static size_t stage_tape_bytes(const tpf_ctx* c) {
    return (size_t)(1 + c->dim) * align256((size_t)c->N * c->tsz) + align256((size_t)c->N * 8);
}

template <typename T>
static Fwd<T> fwd_of(tpf_ctx* c, const void* phi, const void* const u[3]) {
    Fwd<T> F;
    F.phi = static_cast<const T*>(phi);
    for (int a = 0; a < 3; ++a) {
        const bool on = a < c->dim;
        F.u[a] = on ? static_cast<const T*>(u[a]) : nullptr;
        F.n[a] = on ? static_cast<const T*>(c->nrm[a]) : nullptr;
        F.m[a] = on ? static_cast<const T*>(c->mflux[a]) : nullptr;
        F.f[a] = on ? static_cast<const T*>(c->fs[a]) : nullptr;
    }
    F.mu = static_cast<const T*>(c->mu);
    F.kappa = static_cast<const T*>(c->kappa);
    return F;
}

// Transpose of one stage evaluation at (phi_s, u_s) with stage pressure p_s:
// (l_dphi, l_du) -> (out_phi, out_u); parameter cotangents added to the
// accumulators after the scratch fields.
template <typename T, int DIM>
static tpf_status stage_vjp_t(tpf_ctx* c, const void* phi_s, const void* const u_s[3], const double* p_s,
                              const double* const lk[4], double* const out[4]) {
    const AdjLayout L = adj_layout(DIM);
    const Phys P = phys_of(c);
    const Dims d = dims_of(c->n);
    const dim3 g = grid_of(c->n), b(BX, BY);
    const int nb = (int)nblocks_of(c->n);
    const void* u3[3] = {u_s[0], u_s[1], DIM == 3 ? u_s[2] : u_s[1]};
    AdjFields A{};
    A.ldphi = lk[0];
    for (int a = 0; a < DIM; ++a) {
        A.ldu[a] = lk[1 + a];
        A.lX[a] = af(c, L.lx + a);
        A.lrho[a] = af(c, L.lrho + a);
        A.lr[a] = af(c, L.lr + a);
        A.lg[a] = af(c, L.lg + a);
        A.outu[a] = out[1 + a];
    }
    A.p = p_s;
    A.q = c->p;
    A.lmu = af(c, L.lmu);
    A.ldm = af(c, L.ldm);
    A.leta = af(c, L.leta);
    A.lkap = af(c, L.lkap);
    A.dm = af(c, L.dm);
    A.outphi = out[0];
    // forward intermediates: normals, mu or kappa, CDI and mass fluxes, f*
    hipError_t e = launch_stage_fields(c, phi_s, u3);
    if (e == hipSuccess) e = launch_momentum(c, phi_s, u3, 0);
    // adjoint pressure: D(beta G q) = D(beta l_du), zero mean; warm start:
    // the adjoint pressure of the previous stage in the sweep
    if (e == hipSuccess)
        k_adj_rhs<T, DIM><<<g, b, 0, c->stream>>>(d, P, static_cast<const T*>(phi_s), A, c->b, c->partials);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = launch_finalize(c, nb, 1, FIN_MEAN);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->p, af(c, L.q), (size_t)c->N * 8, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint stage setup");
    int it = 0, outer = 0;
    double rr = 0.0;
    tpf_status st = poisson_solve(c, phi_s, &it, &rr, &outer);
    if (st != TPF_OK) return st;
    e = hipMemcpyAsync(af(c, L.q), c->p, (size_t)c->N * 8, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint pressure copy");
    const Fwd<T> F = fwd_of<T>(c, phi_s, u_s);
    double* grad = grad_acc(c);
    k_adj_proj<T, DIM><<<g, b, 0, c->stream>>>(d, P, F, A);
    k_adj_cell1<T, DIM><<<g, b, 0, c->stream>>>(d, P, F, A, c->partials);
    k_adj_grad<<<1, 256, 0, c->stream>>>(nb, nb, c->partials, grad);
    k_adj_face<T, DIM><<<g, b, 0, c->stream>>>(d, P, F, A, c->partials);
    k_adj_grad<<<1, 256, 0, c->stream>>>(nb, nb, c->partials, grad);
    k_adj_cell2<T, DIM><<<g, b, 0, c->stream>>>(d, P, F, A);
    k_adj_cell3<DIM><<<g, b, 0, c->stream>>>(d, P, A);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "adjoint stage kernels");
    return TPF_OK;
}

static tpf_status stage_vjp(tpf_ctx* c, const void* phi_s, const void* const u_s[3], const double* p_s,
                            const double* const lk[4], double* const out[4]) {
    if (c->mixed)
        return c->dim == 2 ? stage_vjp_t<float, 2>(c, phi_s, u_s, p_s, lk, out)
                           : stage_vjp_t<float, 3>(c, phi_s, u_s, p_s, lk, out);
    return c->dim == 2 ? stage_vjp_t<double, 2>(c, phi_s, u_s, p_s, lk, out)
                       : stage_vjp_t<double, 3>(c, phi_s, u_s, p_s, lk, out);
}

static tpf_status vec_in(tpf_ctx* c, double* dst, const double* src, int on_device) {
    hipError_t e = hipMemcpyAsync(dst, src, (size_t)c->N * 8,
                                  on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream);
    return e == hipSuccess ? TPF_OK : hip_fail(e, "cotangent copy in");
}
static tpf_status vec_out(tpf_ctx* c, double* dst, const double* src, int on_device) {
    hipError_t e = hipMemcpyAsync(dst, src, (size_t)c->N * 8,
                                  on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream);
    return e == hipSuccess ? TPF_OK : hip_fail(e, "cotangent copy out");
}

// zero the parameter accumulators and the adjoint-pressure warm start
static tpf_status zero_grad(tpf_ctx* c) {
    hipError_t e = hipMemsetAsync(grad_acc(c), 0, 2 * sizeof(double), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(af(c, adj_layout(c->dim).q), 0, (size_t)c->N * 8, c->stream);
    return e == hipSuccess ? TPF_OK : hip_fail(e, "gradient reset");
}

static tpf_status add_grad(tpf_ctx* c, double* grad_params) {
    double g[2] = {0.0, 0.0};
    hipError_t e = hipMemcpyAsync(g, grad_acc(c), sizeof(g), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "gradient readback");
    if (grad_params) {
        grad_params[0] += g[0];
        grad_params[1] += g[1];
    }
    return TPF_OK;
}

}  // namespace tpf

using namespace tpf;

extern "C" {

tpf_status tpf_adjoint_tape_bytes(const tpf_ctx* c, int32_t nsteps, size_t* bytes) {
    tpf_status st = adjoint_supported(c);
    if (st != TPF_OK) return st;
    if (nsteps < 0 || !bytes) { set_error("nsteps >= 0 and bytes required"); return TPF_EINVAL; }
    *bytes = (size_t)nsteps * 4 * stage_tape_bytes(c);
    return TPF_OK;
}

tpf_status tpf_stage_adjoint(tpf_ctx* c, const double* lphi, const double* lu0, const double* lu1,
                             const double* lu2, double* gphi, double* gu0, double* gu1, double* gu2,
                             double grad_params[2], int32_t on_device) {
    tpf_status st = adjoint_supported(c);
    if (st != TPF_OK) return st;
    const int S = 1 + c->dim;
    const double* lin[4] = {lphi, lu0, lu1, lu2};
    double* gout[4] = {gphi, gu0, gu1, gu2};
    for (int k = 0; k < S; ++k)
        if (!lin[k] || !gout[k]) { set_error("NULL cotangent"); return TPF_EINVAL; }
    const AdjLayout L = adj_layout(c->dim);
    st = eval_current(c, 0);
    if (st != TPF_OK) return st;
    hipError_t e = hipMemcpyAsync(af(c, L.pst), c->p, (size_t)c->N * 8, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(e, "stage pressure copy");
    for (int k = 0; k < S && st == TPF_OK; ++k) st = vec_in(c, af(c, L.lk + k), lin[k], on_device);
    if (st == TPF_OK) st = zero_grad(c);
    if (st != TPF_OK) return st;
    const void* u[3] = {c->u[0][c->s_yn], c->u[1][c->s_yn], c->dim == 3 ? c->u[2][c->s_yn] : nullptr};
    const double* lk[4] = {};
    double* out[4] = {};
    for (int k = 0; k < S; ++k) {
        lk[k] = af(c, L.lk + k);
        out[k] = af(c, L.ly + k);
    }
    st = stage_vjp(c, c->phi[c->s_yn], u, af(c, L.pst), lk, out);
    if (st != TPF_OK) return st;
    for (int k = 0; k < S && st == TPF_OK; ++k) st = vec_out(c, gout[k], out[k], on_device);
    if (st != TPF_OK) return st;
    c->p_valid = 0;
    c->hist2_valid = 0;
    return add_grad(c, grad_params);
}

tpf_status tpf_step_adjoint(tpf_ctx* c, void* tape, size_t tape_bytes, double dt, int32_t nsteps,
                            double* gphi, double* gu0, double* gu1, double* gu2, int32_t on_device,
                            double grad_params[2]) {
    tpf_status st = adjoint_supported(c);
    if (st != TPF_OK) return st;
    const int S = 1 + c->dim;
    double* gio[4] = {gphi, gu0, gu1, gu2};
    for (int k = 0; k < S; ++k)
        if (!gio[k]) { set_error("NULL cotangent"); return TPF_EINVAL; }
    if (!(dt > 0) || nsteps < 0) { set_error("dt must be > 0 and nsteps >= 0"); return TPF_EINVAL; }
    const size_t sb = stage_tape_bytes(c);
    if (!tape || tape_bytes < (size_t)nsteps * 4 * sb) {
        set_error("tape too small: need tpf_adjoint_tape_bytes()");
        return TPF_ENOMEM;
    }
    char* T = static_cast<char*>(tape);
    // forward: record every stage input and pressure
    st = advance(c, dt, nsteps, T, sb);
    if (st != TPF_OK) return st;
    const AdjLayout L = adj_layout(c->dim);
    for (int k = 0; k < S && st == TPF_OK; ++k) st = vec_in(c, af(c, L.lam + k), gio[k], on_device);
    if (st == TPF_OK) st = zero_grad(c);
    if (st != TPF_OK) return st;
    const long N = c->N;
    const size_t fT = align256((size_t)N * c->tsz);
    const double wlam[4] = {dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0};
    const double wnext[4] = {dt / 2.0, dt / 2.0, dt, 0.0};
    double *lam[4] = {}, *acc[4] = {}, *lk[4] = {}, *ly[4] = {};
    for (int k = 0; k < S; ++k) {
        lam[k] = af(c, L.lam + k);
        acc[k] = af(c, L.acc + k);
        lk[k] = af(c, L.lk + k);
        ly[k] = af(c, L.ly + k);
    }
    const double* clk[4] = {lk[0], lk[1], lk[2], lk[3]};
    for (int n = nsteps - 1; n >= 0; --n) {
        // y_{n+1} = y_n + sum_s wlam[s] k_s,  Y_{s+1} = y_n + wnext[s] k_s
        for (int k = 0; k < S; ++k) k_axpby<<<vb(N), 256, 0, c->stream>>>(N, 1.0, lam[k], 0.0, nullptr, acc[k]);
        for (int s = 3; s >= 0; --s) {
            for (int k = 0; k < S; ++k)
                k_axpby<<<vb(N), 256, 0, c->stream>>>(N, wlam[s], lam[k], wnext[s], s < 3 ? ly[k] : nullptr, lk[k]);
            const char* rec = T + ((size_t)n * 4 + s) * sb;
            const void* u[3] = {rec + fT, rec + 2 * fT, c->dim == 3 ? rec + 3 * fT : nullptr};
            st = stage_vjp(c, rec, u, reinterpret_cast<const double*>(rec + (size_t)S * fT), clk, ly);
            if (st != TPF_OK) return st;
            for (int k = 0; k < S; ++k) k_axpby<<<vb(N), 256, 0, c->stream>>>(N, 1.0, acc[k], 1.0, ly[k], acc[k]);
        }
        for (int k = 0; k < S; ++k) k_axpby<<<vb(N), 256, 0, c->stream>>>(N, 1.0, acc[k], 0.0, nullptr, lam[k]);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "adjoint sweep");
    for (int k = 0; k < S && st == TPF_OK; ++k) st = vec_out(c, gio[k], lam[k], on_device);
    if (st != TPF_OK) return st;
    c->p_valid = 0;
    c->hist2_valid = 0;
    return add_grad(c, grad_params);
}

// ------------------------------------------------------------------ checkpoints
struct CkptHeader {
    int64_t magic, N, dim, tsz, step;
    double t, mass0;
};
static const int64_t CKPT_MAGIC = 0x74706663706b7431LL;

tpf_status tpf_checkpoint_bytes(const tpf_ctx* c, size_t* bytes) {
    if (!c || !bytes) { set_error("NULL argument"); return TPF_EINVAL; }
    *bytes = 256 + (size_t)(1 + c->dim) * align256((size_t)c->N * c->tsz) + align256((size_t)c->N * 8);
    return TPF_OK;
}

tpf_status tpf_save_checkpoint(tpf_ctx* c, void* dst) {
    if (!c || !dst) { set_error("NULL argument"); return TPF_EINVAL; }
    CkptHeader h{CKPT_MAGIC, c->N, c->dim, (int64_t)c->tsz, c->step, c->t, c->mass0};
    char* D = static_cast<char*>(dst);
    const size_t fT = align256((size_t)c->N * c->tsz);
    hipError_t e = hipMemcpyAsync(D, &h, sizeof(h), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(D + 256, c->phi[c->s_yn], (size_t)c->N * c->tsz, hipMemcpyDeviceToDevice, c->stream);
    for (int a = 0; a < c->dim && e == hipSuccess; ++a)
        e = hipMemcpyAsync(D + 256 + (1 + a) * fT, c->u[a][c->s_yn], (size_t)c->N * c->tsz, hipMemcpyDeviceToDevice,
                           c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(D + 256 + (1 + c->dim) * fT, c->p, (size_t)c->N * 8, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "checkpoint save");
    return TPF_OK;
}

tpf_status tpf_load_checkpoint(tpf_ctx* c, const void* src) {
    if (!c || !src) { set_error("NULL argument"); return TPF_EINVAL; }
    const char* S = static_cast<const char*>(src);
    CkptHeader h{};
    hipError_t e = hipMemcpyAsync(&h, S, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "checkpoint header");
    if (h.magic != CKPT_MAGIC || h.N != c->N || h.dim != c->dim || h.tsz != (int64_t)c->tsz) {
        set_error("checkpoint does not belong to a context of this shape and precision");
        return TPF_EINVAL;
    }
    const size_t fT = align256((size_t)c->N * c->tsz);
    e = hipMemcpyAsync(c->phi[c->s_yn], S + 256, (size_t)c->N * c->tsz, hipMemcpyDeviceToDevice, c->stream);
    for (int a = 0; a < c->dim && e == hipSuccess; ++a)
        e = hipMemcpyAsync(c->u[a][c->s_yn], S + 256 + (1 + a) * fT, (size_t)c->N * c->tsz, hipMemcpyDeviceToDevice,
                           c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->p, S + 256 + (1 + c->dim) * fT, (size_t)c->N * 8, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "checkpoint load");
    c->t = h.t;
    c->step = h.step;
    c->mass0 = h.mass0;
    c->p_valid = 0;
    c->hist2_valid = 0;
    return TPF_OK;
}

}  // extern "C"
