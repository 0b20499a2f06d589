// Reverse-mode derivative of the step (2D, CDI phase field, energy-based
// force): the transpose of every stage operator, hand written, plus the RK4
// reverse sweep over a tape of stage states.
//
// One stage maps y = (phi, u) to (dphi/dt, du/dt) (Eq. 1 with the CDI flux of
// Table 1; momentum with the force of Eq. 4 and mu of Eq. 2; projection).
// Given the cotangents (l_dphi, l_du) of its outputs, stage_vjp returns the
// cotangents of phi and u and adds those of sigma and eps.  Discrete
// transposes used throughout (periodic grid, plain sums as inner products):
//   D^T = -G,  G^T = -D,  A_a^T q[c] = (q[c] + q[c+e_a])/2,  C_a^T = -C_a,
//   L^T = L, and the viscous operator V(eta, .) is symmetric.
// Projection: du = f* - beta G p with D(beta G p) = D f*.  With
//   q solving D(beta G q) = D(beta l_du):
//   l_f* = l_du - G q,   l_rho_a = -beta_a l_f*_a du_a.
// All cotangents are FP64 whatever the state precision T.
#include <cmath>
#include <cstring>

#include "tpf_internal.hpp"

namespace tpf {

struct AdjFields {
    const double* ldphi;   // cotangent of dphi/dt (cell)
    const double* ldu0;    // cotangent of du/dt (faces)
    const double* ldu1;
    const double* p;       // stage pressure
    const double* q;       // adjoint pressure
    double* lX0;           // cotangent of X = -N + V + F (faces)
    double* lX1;
    double* lrho0;         // cotangent of the face density
    double* lrho1;
    double* lr0;           // cotangent of the CDI flux (faces)
    double* lr1;
    double* lmu;           // cotangent of mu (cells)
    double* ldm;           // cotangent of D m (cells)
    double* leta;          // cotangent of the viscosity (cells)
    double* lg0;           // cotangent of the central gradient g (cells)
    double* lg1;
    double* outphi;        // stage cotangent of phi (cells)
    double* outu0;         // stage cotangent of u (faces)
    double* outu1;
};

template <typename T>
struct Fwd {
    const T* phi;
    const T* u0;
    const T* u1;
    const T* n0;
    const T* n1;
    const T* mu;
    const T* m0;
    const T* m1;
    const T* f0;
    const T* f1;
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

// ------------------------------------------------------------------ rhs of the adjoint solve
// b = D(beta l_du) in FP64, block sums for the mean
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_adj_rhs(Dims d, Phys P, const T* __restrict__ phi,
                                                   const double* __restrict__ l0, const double* __restrict__ l1,
                                                   double* __restrict__ b, double* __restrict__ partials) {
    Cell C;
    double v[1] = {0.0};
    if (cell_of_thread(d, C)) {
        const double* l[2] = {l0, l1};
        auto bl = [&](int a, unsigned c) {     // beta_a l_a at face (c, a)
            const Cell Q = make_cell(d, c % d.nx, c / d.nx, 0);
            const double rf = 0.5 * (rho_d(P, (double)phi[Q.off(a, -1)]) + rho_d(P, (double)phi[c]));
            return l[a][c] / rf;
        };
        double s = 0.0;
        for (int a = 0; a < 2; ++a) s += (bl(a, C.off(a, 1)) - bl(a, C.id)) * P.inv_h;
        b[C.id] = s;
        v[0] = s;
    }
    block_partials<1>(v, partials);
}

// ------------------------------------------------------------------ P1: projection and f* = X beta
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_adj_proj(Dims d, Phys P, Fwd<T> F, AdjFields A) {
    Cell C;
    if (!cell_of_thread(d, C)) return;
    const unsigned c = C.id;
    const double* ldu[2] = {A.ldu0, A.ldu1};
    const T* fs[2] = {F.f0, F.f1};
    double* lX[2] = {A.lX0, A.lX1};
    double* lrho[2] = {A.lrho0, A.lrho1};
    const double fc = (double)F.phi[c];
    for (int a = 0; a < 2; ++a) {
        const unsigned cm = C.off(a, -1);
        const double beta = 1.0 / (0.5 * (rho_d(P, (double)F.phi[cm]) + rho_d(P, fc)));
        const double lf = ldu[a][c] - (A.q[c] - A.q[cm]) * P.inv_h;
        const double du = (double)fs[a][c] - beta * (A.p[c] - A.p[cm]) * P.inv_h;
        lX[a][c] = lf * beta;
        lrho[a][c] = -beta * lf * du;
    }
}

// ------------------------------------------------------------------ P2: mu, D m and viscosity cotangents
// lambda_mu = A^T(l_X G phi) (energy-based force); lambda_Dm = A^T(l_X u);
// lambda_eta from the symmetric viscous form; parameter partials of mu.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_adj_cell1(Dims d, Phys P, Fwd<T> F, AdjFields A,
                                                     double* __restrict__ partials) {
    Cell C;
    double v[2] = {0.0, 0.0};
    if (cell_of_thread(d, C)) {
        const unsigned c = C.id;
        const double ih = P.inv_h;
        const double* lX[2] = {A.lX0, A.lX1};
        const T* u[2] = {F.u0, F.u1};
        auto ph = [&](unsigned q) { return (double)F.phi[q]; };
        double lmu = 0.0, ldm = 0.0, lap = 0.0;
        const double fc = ph(c);
        for (int a = 0; a < 2; ++a) {
            const unsigned cp = C.off(a, 1), cm = C.off(a, -1);
            const double g_lo = (fc - ph(cm)) * ih, g_hi = (ph(cp) - fc) * ih;
            lmu += 0.5 * (lX[a][c] * g_lo + lX[a][cp] * g_hi);
            ldm += 0.5 * (lX[a][c] * (double)u[a][c] + lX[a][cp] * (double)u[a][cp]);
            lap += (g_hi - g_lo) * ih;
        }
        // viscous: d<w, V(eta, u)>/d eta_c with w = l_X
        double leta = 0.0;
        for (int a = 0; a < 2; ++a) {
            const unsigned cp = C.off(a, 1);
            const double su = ((double)u[a][cp] - (double)u[a][c]) * ih;
            const double sw = (lX[a][cp] - lX[a][c]) * ih;
            leta -= 2.0 * su * sw;
        }
        // the four corners of cell c: E(c), E(c+e0), E(c+e1), E(c+e0+e1); the
        // corner E(q) is shared by q, q-e0, q-e1, q-e0-e1
        auto gam = [&](unsigned q, const Cell& Q, bool useX) {
            const unsigned q0m = Q.off(1, -1);   // q - e1 (for u0)
            const unsigned q1m = Q.off(0, -1);   // q - e0 (for u1)
            if (useX) return (lX[0][q] - lX[0][q0m]) * ih + (lX[1][q] - lX[1][q1m]) * ih;
            return ((double)u[0][q] - (double)u[0][q0m]) * ih + ((double)u[1][q] - (double)u[1][q1m]) * ih;
        };
        const int cx[4] = {0, 1, 0, 1}, cy[4] = {0, 0, 1, 1};
        for (int k = 0; k < 4; ++k) {
            const int i = wrapc(C.i + cx[k], d.nx), j = wrapc(C.j + cy[k], d.ny);
            const Cell Q = make_cell(d, i, j, 0);
            leta -= 0.25 * gam(Q.id, Q, false) * gam(Q.id, Q, true);
        }
        A.lmu[c] = lmu;
        A.ldm[c] = ldm;
        A.leta[c] = leta;
        // mu = (6 sigma / eps) psi'(phi) - 6 sigma eps L phi
        const double dp = (double)dpsi(fc);
        v[0] = lmu * 6.0 * (dp / P.eps - P.eps * lap);
        v[1] = lmu * (-P.sigma_hat * dp / (P.eps * P.eps) - P.sigma_hat * lap);
    }
    block_partials<2>(v, partials);
}

// ------------------------------------------------------------------ P3: face cotangents
// advection (l_N = -l_X), viscous V(eta, l_X), mass flux, phase-field flux
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_adj_face(Dims d, Phys P, Fwd<T> F, AdjFields A,
                                                    double* __restrict__ partials) {
    Cell C;
    double v[2] = {0.0, 0.0};
    if (cell_of_thread(d, C)) {
        const unsigned c = C.id;
        const double ih = P.inv_h;
        const double* lX[2] = {A.lX0, A.lX1};
        const T* u[2] = {F.u0, F.u1};
        const T* m[2] = {F.m0, F.m1};
        double* lrho[2] = {A.lrho0, A.lrho1};
        double* lr[2] = {A.lr0, A.lr1};
        double* outu[2] = {A.outu0, A.outu1};
        auto ph = [&](unsigned q) { return (double)F.phi[q]; };
        auto U = [&](int a, unsigned q) { return (double)u[a][q]; };
        auto M = [&](int a, unsigned q) { return (double)m[a][q]; };
        auto lN = [&](int a, unsigned q) { return -lX[a][q]; };
        const double fc = ph(c);
        const double drho = P.rho1 - P.rho2;
        for (int a = 0; a < 2; ++a) {
            const int b = 1 - a;
            const unsigned cp = C.off(a, 1), cm = C.off(a, -1);
            const unsigned cpb = C.off(b, 1), cmb = C.off(b, -1);
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
            // corner terms.  Corner E(q) is the lower corner of q in the (a, b)
            // plane.  Phi_ba(E(q)) = Mb_b(E(q)) Ub_a(E(q)) enters N_a[q - e_b]
            // with +1/h and N_a[q] with -1/h; Phi_ab(E(q)) = Mb_a(E(q)) Ub_b(E(q))
            // enters N_b[q - e_a] with +1/h and N_b[q] with -1/h.
            //   Mb_b(E(q)) = (m_b[q] + m_b[q - e_a]) / 2,  Ub_a(E(q)) = (u_a[q - e_b] + u_a[q]) / 2
            //   Mb_a(E(q)) = (m_a[q] + m_a[q - e_b]) / 2,  Ub_b(E(q)) = (u_b[q - e_a] + u_b[q]) / 2
            {
                // u_a[c] sits in Ub_a(E(c)) and Ub_a(E(c + e_b))
                const unsigned cpb_ma = C.off2(b, 1, a, -1);           // c + e_b - e_a
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
            // - u_a A_a(D m):  l_u += l_X A_a(Dm);  l_m_a += -G_a(l_Dm)
            {
                auto dm = [&](unsigned q) {
                    const Cell Q = make_cell(d, q % d.nx, q / d.nx, 0);
                    double s = 0.0;
                    for (int e = 0; e < 2; ++e) s += (M(e, Q.off(e, 1)) - M(e, q)) * ih;
                    return s;
                };
                lu += lX[a][c] * 0.5 * (dm(cm) + dm(c));
                lm += -(A.ldm[c] - A.ldm[cm]) * ih;
            }
            // viscous V_a(eta, l_X)[c] (the operator is symmetric)
            {
                auto eta = [&](unsigned q) { return eta_d(P, ph(q)); };
                auto W = [&](int e, unsigned q) { return lX[e][q]; };
                const double eta_c = eta(c), eta_m = eta(cm);
                double V = 0.0;
                V += (2.0 * eta_c * (W(a, cp) - W(a, c)) * ih - 2.0 * eta_m * (W(a, c) - W(a, cm)) * ih) * ih;
                const unsigned cmapb = C.off2(a, -1, b, 1), cmamb = C.off2(a, -1, b, -1);
                const double eta_hi = 0.25 * (eta_c + eta_m + eta(cpb) + eta(cmapb));
                const double eta_lo = 0.25 * (eta(cmb) + eta(cmamb) + eta_c + eta_m);
                const double hi = eta_hi * ((W(a, cpb) - W(a, c)) * ih + (W(b, cpb) - W(b, cmapb)) * ih);
                const double lo = eta_lo * ((W(a, c) - W(a, cmb)) * ih + (W(b, c) - W(b, cm)) * ih);
                V += (hi - lo) * ih;
                lu += V;
            }
            // mass flux m_a = rho_a u_a - (rho1 - rho2) r_a
            const double rho_f = 0.5 * (rho_d(P, ph(cm)) + rho_d(P, fc));
            lu += rho_f * lm;
            lrho[a][c] += U(a, c) * lm;
            // phase field: J_a = u_a A_a phi, dphi = -D J + D r
            const double lJ = (A.ldphi[c] - A.ldphi[cm]) * ih;
            lu += lJ * 0.5 * (ph(cm) + fc);
            const double lra = -drho * lm - lJ;
            lr[a][c] = lra;
            outu[a][c] = lu;
            // r_a = gamma [eps G_a phi - ...]:  d r / d eps = gamma G_a phi
            v[1] += lra * P.gamma * (fc - ph(cm)) * ih;
        }
    }
    block_partials<2>(v, partials);
}

// ------------------------------------------------------------------ P4: phi cotangent (all but the normals)
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_adj_cell2(Dims d, Phys P, Fwd<T> F, AdjFields A) {
    Cell C;
    if (!cell_of_thread(d, C)) return;
    const unsigned c = C.id;
    const double ih = P.inv_h;
    const double* lX[2] = {A.lX0, A.lX1};
    const double* lrho[2] = {A.lrho0, A.lrho1};
    const double* lr[2] = {A.lr0, A.lr1};
    const T* u[2] = {F.u0, F.u1};
    const T* n[2] = {F.n0, F.n1};
    auto ph = [&](unsigned q) { return (double)F.phi[q]; };
    auto mu = [&](unsigned q) { return (double)F.mu[q]; };
    const double fc = ph(c);
    double lphi = 0.0;
    double lrho_c = 0.0, llap = 0.0, lwn[2], g[2], gg = 0.0;
    for (int a = 0; a < 2; ++a) {
        const unsigned cp = C.off(a, 1), cm = C.off(a, -1);
        lrho_c += 0.5 * (lrho[a][c] + lrho[a][cp]);
        // energy-based force: G_a^T of l_X A_a(mu)
        lphi += (lX[a][c] * 0.5 * (mu(cm) + mu(c)) - lX[a][cp] * 0.5 * (mu(c) + mu(cp))) * ih;
        llap += ((A.lmu[cp] - A.lmu[c]) * ih - (A.lmu[c] - A.lmu[cm]) * ih) * ih;
        // phase-field flux J: A_a^T of l_J u_a
        const double lJ_c = (A.ldphi[c] - A.ldphi[cm]) * ih, lJ_p = (A.ldphi[cp] - A.ldphi[c]) * ih;
        lphi += 0.5 * (lJ_c * (double)u[a][c] + lJ_p * (double)u[a][cp]);
        // CDI flux: gamma eps G_a phi
        lphi += P.gamma * P.eps * (lr[a][c] - lr[a][cp]) * ih;
        // - gamma A_a(w n_a): cotangent of (w n_a) at the cell
        lwn[a] = -P.gamma * 0.5 * (lr[a][c] + lr[a][cp]);
        g[a] = (ph(cp) - ph(cm)) * (0.5 * ih);
        gg += g[a] * g[a];
    }
    lphi += (P.rho1 - P.rho2) * clamp_slope(P, fc) * lrho_c;
    lphi += (P.visc1 - P.visc2) * clamp_slope(P, fc) * A.leta[c];
    // mu = (sigma_hat/eps) psi'(phi) - sigma_hat eps L phi;  psi'' = 1 - 6 phi + 6 phi^2
    lphi += (P.sigma_hat / P.eps) * (1.0 - 6.0 * fc + 6.0 * fc * fc) * A.lmu[c] - P.sigma_hat * P.eps * llap;
    const double w = fc * (1.0 - fc);
    const double nn[2] = {(double)n[0][c], (double)n[1][c]};
    lphi += (1.0 - 2.0 * fc) * (lwn[0] * nn[0] + lwn[1] * nn[1]);
    // normals n = g / sqrt(g.g + delta^2): l_g = s (l_n - n (n . l_n)), l_n = l_wn w
    const double s = 1.0 / sqrt(gg + P.delta2);
    const double ln0 = lwn[0] * w, ln1 = lwn[1] * w;
    const double m0 = g[0] * s, m1 = g[1] * s;
    const double dot = m0 * ln0 + m1 * ln1;
    A.lg0[c] = s * (ln0 - m0 * dot);
    A.lg1[c] = s * (ln1 - m1 * dot);
    A.outphi[c] = lphi;
}

// ------------------------------------------------------------------ P5: C_a^T of l_g
__global__ __launch_bounds__(BLOCK) void k_adj_cell3(Dims d, Phys P, AdjFields A) {
    Cell C;
    if (!cell_of_thread(d, C)) return;
    const unsigned c = C.id;
    const double* lg[2] = {A.lg0, A.lg1};
    double s = 0.0;
    for (int a = 0; a < 2; ++a) s -= (lg[a][C.off(a, 1)] - lg[a][C.off(a, -1)]) * (0.5 * P.inv_h);
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

// adjoint scratch fields (each adj_stride doubles)
enum {
    AF_LAM = 0,      // 3: cotangent of y_{n+1} (phi, u0, u1)
    AF_ACC = 3,      // 3: cotangent of y_n being accumulated
    AF_LK = 6,       // 3: cotangent of the stage derivative k_s
    AF_LY = 9,       // 3: cotangent of the stage input Y_s
    AF_LX = 12,      // 2
    AF_LRHO = 14,    // 2
    AF_LR = 16,      // 2
    AF_LG = 18,      // 2
    AF_LMU = 20,
    AF_LDM = 21,
    AF_LETA = 22,
    AF_PST = 23,     // stage pressure (single-stage adjoint)
    AF_Q = 24,       // last adjoint pressure (warm start of the next adjoint solve)
    AF_GRAD = 26     // two accumulators after the fields
};
static_assert(AF_PST < ADJ_FIELDS, "adjoint scratch layout");

static double* af(tpf_ctx* c, int k) { return c->adj + (long)k * c->adj_stride; }

static tpf_status adjoint_supported(const tpf_ctx* c) {
    if (!c) { set_error("ctx is NULL"); return TPF_EINVAL; }
    if (c->dim != 2 || c->P.model != TPF_CDI || c->P.force != TPF_EB || !c->adj) {
        set_error("the adjoint covers 2D cases with the CDI model and the energy-based force");
        return TPF_EINVAL;
    }
    return TPF_OK;
}

static size_t stage_tape_bytes(const tpf_ctx* c) {
    return 3 * align256((size_t)c->N * c->tsz) + align256((size_t)c->N * 8);
}

template <typename T>
static Fwd<T> fwd_of(tpf_ctx* c, const void* phi, const void* const u[2]) {
    return Fwd<T>{static_cast<const T*>(phi), static_cast<const T*>(u[0]), static_cast<const T*>(u[1]),
                  static_cast<const T*>(c->nrm[0]), static_cast<const T*>(c->nrm[1]),
                  static_cast<const T*>(c->mu), static_cast<const T*>(c->mflux[0]),
                  static_cast<const T*>(c->mflux[1]), static_cast<const T*>(c->fs[0]),
                  static_cast<const T*>(c->fs[1])};
}

// Transpose of one stage evaluation at (phi_s, u_s) with stage pressure p_s:
// (l_dphi, l_du) -> (out_phi, out_u); parameter cotangents added to the
// accumulators at af(AF_GRAD).
template <typename T>
static tpf_status stage_vjp_t(tpf_ctx* c, const void* phi_s, const void* const u_s[2], const double* p_s,
                              const double* lk[3], double* out[3]) {
    const Phys P = phys_of(c);
    const Dims d = dims_of(c->n);
    const dim3 g = grid_of(c->n), b(BX, BY);
    const int nb = (int)nblocks_of(c->n);
    const void* u3[3] = {u_s[0], u_s[1], u_s[1]};
    // forward intermediates: normals, mu, CDI and mass fluxes, f*
    hipError_t e = launch_stage_fields(c, phi_s, u3);
    if (e == hipSuccess) e = launch_momentum(c, phi_s, u3, 0);
    // adjoint pressure: D(beta G q) = D(beta l_du), zero mean; warm start:
    // the adjoint pressure of the previous stage in the sweep
    if (e == hipSuccess)
        k_adj_rhs<T><<<g, b, 0, c->stream>>>(d, P, static_cast<const T*>(phi_s), lk[1], lk[2], c->b, c->partials);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = launch_finalize(c, nb, 1, FIN_MEAN);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->p, af(c, AF_Q), (size_t)c->N * 8, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint stage setup");
    int it = 0, outer = 0;
    double rr = 0.0;
    tpf_status st = poisson_solve(c, phi_s, &it, &rr, &outer);
    if (st != TPF_OK) return st;
    e = hipMemcpyAsync(af(c, AF_Q), c->p, (size_t)c->N * 8, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint pressure copy");
    const Fwd<T> F = fwd_of<T>(c, phi_s, u_s);
    AdjFields A{lk[0], lk[1], lk[2], p_s, c->p,
                af(c, AF_LX), af(c, AF_LX + 1), af(c, AF_LRHO), af(c, AF_LRHO + 1),
                af(c, AF_LR), af(c, AF_LR + 1), af(c, AF_LMU), af(c, AF_LDM), af(c, AF_LETA),
                af(c, AF_LG), af(c, AF_LG + 1), out[0], out[1], out[2]};
    double* grad = af(c, AF_GRAD);
    k_adj_proj<T><<<g, b, 0, c->stream>>>(d, P, F, A);
    k_adj_cell1<T><<<g, b, 0, c->stream>>>(d, P, F, A, c->partials);
    k_adj_grad<<<1, 256, 0, c->stream>>>(nb, nb, c->partials, grad);
    k_adj_face<T><<<g, b, 0, c->stream>>>(d, P, F, A, c->partials);
    k_adj_grad<<<1, 256, 0, c->stream>>>(nb, nb, c->partials, grad);
    k_adj_cell2<T><<<g, b, 0, c->stream>>>(d, P, F, A);
    k_adj_cell3<<<g, b, 0, c->stream>>>(d, P, A);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "adjoint stage kernels");
    return TPF_OK;
}

static tpf_status stage_vjp(tpf_ctx* c, const void* phi_s, const void* const u_s[2], const double* p_s,
                            const double* lk[3], double* out[3]) {
    return c->mixed ? stage_vjp_t<float>(c, phi_s, u_s, p_s, lk, out)
                    : stage_vjp_t<double>(c, phi_s, u_s, p_s, lk, out);
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
    hipError_t e = hipMemsetAsync(af(c, AF_GRAD), 0, 2 * sizeof(double), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(af(c, AF_Q), 0, (size_t)c->N * 8, c->stream);
    return e == hipSuccess ? TPF_OK : hip_fail(e, "gradient reset");
}

static tpf_status add_grad(tpf_ctx* c, double* grad_params) {
    double g[2] = {0.0, 0.0};
    hipError_t e = hipMemcpyAsync(g, af(c, AF_GRAD), sizeof(g), hipMemcpyDeviceToHost, c->stream);
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
                             double* gphi, double* gu0, double* gu1, double grad_params[2], int32_t on_device) {
    tpf_status st = adjoint_supported(c);
    if (st != TPF_OK) return st;
    if (!lphi || !lu0 || !lu1 || !gphi || !gu0 || !gu1) { set_error("NULL argument"); return TPF_EINVAL; }
    st = eval_current(c, 0);
    if (st != TPF_OK) return st;
    hipError_t e = hipMemcpyAsync(af(c, AF_PST), c->p, (size_t)c->N * 8, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(e, "stage pressure copy");
    const double* lin[3] = {lphi, lu0, lu1};
    for (int k = 0; k < 3 && st == TPF_OK; ++k) st = vec_in(c, af(c, AF_LK + k), lin[k], on_device);
    if (st == TPF_OK) st = zero_grad(c);
    if (st != TPF_OK) return st;
    const void* u[2] = {c->u[0][c->s_yn], c->u[1][c->s_yn]};
    const double* lk[3] = {af(c, AF_LK), af(c, AF_LK + 1), af(c, AF_LK + 2)};
    double* out[3] = {af(c, AF_LY), af(c, AF_LY + 1), af(c, AF_LY + 2)};
    st = stage_vjp(c, c->phi[c->s_yn], u, af(c, AF_PST), lk, out);
    if (st != TPF_OK) return st;
    double* gout[3] = {gphi, gu0, gu1};
    for (int k = 0; k < 3 && st == TPF_OK; ++k) st = vec_out(c, gout[k], out[k], on_device);
    if (st != TPF_OK) return st;
    c->p_valid = 0;
    c->hist2_valid = 0;
    return add_grad(c, grad_params);
}

tpf_status tpf_step_adjoint(tpf_ctx* c, void* tape, size_t tape_bytes, double dt, int32_t nsteps,
                            double* gphi, double* gu0, double* gu1, int32_t on_device, double grad_params[2]) {
    tpf_status st = adjoint_supported(c);
    if (st != TPF_OK) return st;
    if (!gphi || !gu0 || !gu1) { set_error("NULL cotangent"); return TPF_EINVAL; }
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
    double* gio[3] = {gphi, gu0, gu1};
    for (int k = 0; k < 3 && st == TPF_OK; ++k) st = vec_in(c, af(c, AF_LAM + k), gio[k], on_device);
    if (st == TPF_OK) st = zero_grad(c);
    if (st != TPF_OK) return st;
    const long N = c->N;
    const size_t fT = align256((size_t)N * c->tsz);
    const double wlam[4] = {dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0};
    const double wnext[4] = {dt / 2.0, dt / 2.0, dt, 0.0};
    double* lam[3] = {af(c, AF_LAM), af(c, AF_LAM + 1), af(c, AF_LAM + 2)};
    double* acc[3] = {af(c, AF_ACC), af(c, AF_ACC + 1), af(c, AF_ACC + 2)};
    double* lk[3] = {af(c, AF_LK), af(c, AF_LK + 1), af(c, AF_LK + 2)};
    double* ly[3] = {af(c, AF_LY), af(c, AF_LY + 1), af(c, AF_LY + 2)};
    const double* clk[3] = {lk[0], lk[1], lk[2]};
    for (int n = nsteps - 1; n >= 0; --n) {
        // y_{n+1} = y_n + sum_s wlam[s] k_s,  Y_{s+1} = y_n + wnext[s] k_s
        for (int k = 0; k < 3; ++k) k_axpby<<<vb(N), 256, 0, c->stream>>>(N, 1.0, lam[k], 0.0, nullptr, acc[k]);
        for (int s = 3; s >= 0; --s) {
            for (int k = 0; k < 3; ++k)
                k_axpby<<<vb(N), 256, 0, c->stream>>>(N, wlam[s], lam[k], wnext[s], s < 3 ? ly[k] : nullptr, lk[k]);
            const char* rec = T + ((size_t)n * 4 + s) * sb;
            const void* u[2] = {rec + fT, rec + 2 * fT};
            st = stage_vjp(c, rec, u, reinterpret_cast<const double*>(rec + 3 * fT), clk, ly);
            if (st != TPF_OK) return st;
            for (int k = 0; k < 3; ++k) k_axpby<<<vb(N), 256, 0, c->stream>>>(N, 1.0, acc[k], 1.0, ly[k], acc[k]);
        }
        for (int k = 0; k < 3; ++k) k_axpby<<<vb(N), 256, 0, c->stream>>>(N, 1.0, acc[k], 0.0, nullptr, lam[k]);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "adjoint sweep");
    for (int k = 0; k < 3 && st == TPF_OK; ++k) st = vec_out(c, gio[k], lam[k], on_device);
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
