/*
 * tpf_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Computes one time step of the incompressible two-phase solver assessed in
 * Mirjalili, Khanwale & Mani (arXiv 2205.05835): a second-order phase-field
 * equation (Table 1: CDI, SB, ISODI), the chemical potential (Eq. 2), a
 * surface tension force (energy-based Eq. 4, CSF, or localized CSF Eq. 11),
 * momentum advection and diffusion and a variable-density pressure
 * projection, discretised with second-order finite differences on a
 * staggered periodic grid and integrated with classical RK4 (Sec. 3).
 *
 * The paper defers the discrete operators to another publication; the
 * operators below are the plain central second-order ones on the MAC grid:
 *
 *   A_a q[c] = (q[c-e_a] + q[c]) / 2            cell -> face average
 *   G_a q[c] = (q[c] - q[c-e_a]) / h            cell -> face gradient
 *   D F[c]   = sum_a (F_a[c+e_a] - F_a[c]) / h  face -> cell divergence
 *   C_a q[c] = (q[c+e_a] - q[c-e_a]) / (2h)     central cell gradient
 *   L        = D o G
 *
 * An axis is periodic, or bounded by free-slip walls at both ends (the box
 * of Sec. 3.1 and the top and bottom of Sec. 3.2).  A free-slip wall is a
 * mirror plane of the solution: values outside the box are read from the
 * mirror image (fetch() below), which makes the normal velocity, the normal
 * derivative of the tangential velocity and of phi, and the normal pressure
 * gradient vanish on the wall.
 *
 * Everything is written for clarity, not speed: full temporaries, no fusion.
 * Loops are parallelised over grid rows with OpenMP; every reduction is
 * summed per row and then over rows in a fixed order, so results do not
 * depend on the thread count.  Nothing here is shared with the HIP library.
 */
#include "tpf_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* grid helpers                                                           */
/* ---------------------------------------------------------------------- */

static long ncell(const ora_params* P) { return (long)P->n[0] * P->n[1] * P->n[2]; }

static int wrapi(int i, int n) {
    while (i < 0) i += n;
    while (i >= n) i -= n;
    return i;
}

/* linear index of cell (i,j,k), periodic in every axis */
static long at(const ora_params* P, int i, int j, int k) {
    i = wrapi(i, P->n[0]);
    j = wrapi(j, P->n[1]);
    k = wrapi(k, P->n[2]);
    return ((long)k * P->n[1] + j) * P->n[0] + i;
}

/* Boundary rules.  A periodic axis wraps.  A walled axis a reads values
 * outside the box from the mirror image in the wall: a cell field is even
 * (cell -1-m holds cell m, cell n+m holds cell n-1-m); the a-component of a
 * cell vector (a normal) is odd; a face field normal to a is odd about the
 * wall faces 0 and n, which hold 0 (face -m holds minus face m); a face field
 * normal to another axis is even like a cell field. */
enum { K_CELL = 0, K_ODD = 1, K_FACE = 2 };
#define KIND_ODD(a) (K_ODD + 4 * (a))    /* cell vector component along a */
#define KIND_FACE(a) (K_FACE + 4 * (a))  /* face field normal to axis a   */

static int walled(const ora_params* P, int a) { return a < P->dim && ((P->walls >> a) & 1); }

/* value of field q (kind) at cell or face (i, j, k), at most two cells outside the box */
static double fetch(const ora_params* P, const double* q, int kind, int i, int j, int k) {
    int v[3] = {i, j, k};
    double sign = 1.0;
    const int base = kind & 3, ax = kind >> 2;
    for (int a = 0; a < 3; ++a) {
        const int n = P->n[a];
        if (!walled(P, a)) {
            v[a] = wrapi(v[a], n);
        } else if (base == K_FACE && ax == a) {
            if (v[a] == 0 || v[a] == n) return 0.0;
            if (v[a] < 0) { v[a] = -v[a]; sign = -sign; }
            else if (v[a] > n) { v[a] = 2 * n - v[a]; sign = -sign; }
        } else {
            const int odd = base == K_ODD && ax == a;
            if (v[a] < 0) { v[a] = -1 - v[a]; if (odd) sign = -sign; }
            else if (v[a] >= n) { v[a] = 2 * n - 1 - v[a]; if (odd) sign = -sign; }
        }
    }
    return sign * q[((long)v[2] * P->n[1] + v[1]) * P->n[0] + v[0]];
}

/* q (kind) at (i,j,k) + s e_a, and at (i,j,k) + s e_a + t e_b */
static double fsh(const ora_params* P, const double* q, int kind, int i, int j, int k, int a, int s) {
    int v[3] = {i, j, k};
    v[a] += s;
    return fetch(P, q, kind, v[0], v[1], v[2]);
}
static double fsh2(const ora_params* P, const double* q, int kind, int i, int j, int k, int a, int s,
                   int b, int t) {
    int v[3] = {i, j, k};
    v[a] += s;
    v[b] += t;
    return fetch(P, q, kind, v[0], v[1], v[2]);
}

#define FOR_CELLS(P)                                             \
    _Pragma("omp parallel for collapse(2) schedule(static)")    \
    for (int k = 0; k < (P)->n[2]; ++k)                          \
        for (int j = 0; j < (P)->n[1]; ++j)                      \
            for (int i = 0; i < (P)->n[0]; ++i)

static double* alloc0(const ora_params* P) {
    return (double*)calloc((size_t)ncell(P), sizeof(double));
}

/* Neumaier-compensated sum of a row-partial array, in order. */
static double ordered_sum(const double* part, long m) {
    double s = 0.0, comp = 0.0;
    for (long q = 0; q < m; ++q) {
        double t = s + part[q];
        if (fabs(s) >= fabs(part[q])) comp += (s - t) + part[q];
        else comp += (part[q] - t) + s;
        s = t;
    }
    return s + comp;
}

/* sum over all cells of x[c]*y[c] (y == NULL: sum of x); fixed order */
static double dot(const ora_params* P, const double* x, const double* y) {
    long rows = (long)P->n[1] * P->n[2];
    double* part = (double*)malloc(sizeof(double) * rows);
#pragma omp parallel for schedule(static)
    for (long r = 0; r < rows; ++r) {
        const double* xr = x + r * P->n[0];
        const double* yr = y ? y + r * P->n[0] : NULL;
        double s = 0.0, comp = 0.0;
        for (int i = 0; i < P->n[0]; ++i) {
            double v = yr ? xr[i] * yr[i] : xr[i];
            double t = s + v;
            if (fabs(s) >= fabs(v)) comp += (s - t) + v;
            else comp += (v - t) + s;
            s = t;
        }
        part[r] = s + comp;
    }
    double s = ordered_sum(part, rows);
    free(part);
    return s;
}

/* ---------------------------------------------------------------------- */
/* pointwise laws                                                         */
/* ---------------------------------------------------------------------- */

static double sigma_hat(const ora_params* P) { return 6.0 * P->sigma; } /* Eq. 2 footnote */

/* psi = [phi(1-phi)]^2 / 2 and its derivative (Eq. 2) */
static double psi(double f) { double w = f * (1.0 - f); return 0.5 * w * w; }
static double dpsi(double f) { return f * (1.0 - f) * (1.0 - 2.0 * f); }

static double clamped(const ora_params* P, double f) {
    if (!P->clamp) return f;
    return f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
}

/* linear mixture laws; phase 1 is phi = 1 */
static double rho_of(const ora_params* P, double f) {
    return P->rho2 + (P->rho1 - P->rho2) * clamped(P, f);
}
static double visc_of(const ora_params* P, double f) {
    return P->visc2 + (P->visc1 - P->visc2) * clamped(P, f);
}

/* face density A_a rho and its inverse beta_a on face (c, a) */
static double rho_face(const ora_params* P, const double* phi, int i, int j, int k, int a) {
    return 0.5 * (rho_of(P, fsh(P, phi, K_CELL, i, j, k, a, -1)) + rho_of(P, phi[at(P, i, j, k)]));
}
static double beta_face(const ora_params* P, const double* phi, int i, int j, int k, int a) {
    return 1.0 / rho_face(P, phi, i, j, k, a);
}

/* ---------------------------------------------------------------------- */
/* discrete operators                                                     */
/* ---------------------------------------------------------------------- */

/* A_a q (q of the given kind), G_a q and L q of a cell field, C_a q */
static double opA(const ora_params* P, const double* q, int kind, int i, int j, int k, int a) {
    return 0.5 * (fsh(P, q, kind, i, j, k, a, -1) + fetch(P, q, kind, i, j, k));
}
static double opG(const ora_params* P, const double* q, int i, int j, int k, int a) {
    return (fetch(P, q, K_CELL, i, j, k) - fsh(P, q, K_CELL, i, j, k, a, -1)) / P->h;
}
static double opC(const ora_params* P, const double* q, int kind, int i, int j, int k, int a) {
    return (fsh(P, q, kind, i, j, k, a, 1) - fsh(P, q, kind, i, j, k, a, -1)) / (2.0 * P->h);
}
/* D F of face fields F_a (normal to a) */
static double opD(const ora_params* P, double* const F[3], int i, int j, int k) {
    double s = 0.0;
    for (int a = 0; a < P->dim; ++a)
        s += (fsh(P, F[a], KIND_FACE(a), i, j, k, a, 1) - fetch(P, F[a], KIND_FACE(a), i, j, k)) / P->h;
    return s;
}
/* L = D o G written out */
static double opL(const ora_params* P, const double* q, int i, int j, int k) {
    double s = 0.0;
    const double qc = fetch(P, q, K_CELL, i, j, k);
    for (int a = 0; a < P->dim; ++a) {
        double gp = (fsh(P, q, K_CELL, i, j, k, a, 1) - qc) / P->h;
        double gm = (qc - fsh(P, q, K_CELL, i, j, k, a, -1)) / P->h;
        s += (gp - gm) / P->h;
    }
    return s;
}

void ora_divergence(const ora_params* P, const double* F0, const double* F1,
                    const double* F2, double* out) {
    double* const F[3] = {(double*)F0, (double*)F1, (double*)F2};
    FOR_CELLS(P) { out[at(P, i, j, k)] = opD(P, F, i, j, k); }
}

/* ---------------------------------------------------------------------- */
/* normals and curvature (Eq. 3, Table 1 caption)                         */
/* ---------------------------------------------------------------------- */

/* g_a = C_a phi;  n_a = g_a / sqrt(g.g + delta^2);  gmag = sqrt(g.g) */
void ora_normals(const ora_params* P, const double* phi, double* nx, double* ny,
                 double* nz, double* gmag) {
    double* n[3] = {nx, ny, nz};
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        double g[3] = {0.0, 0.0, 0.0}, gg = 0.0;
        for (int a = 0; a < P->dim; ++a) {
            g[a] = opC(P, phi, K_CELL, i, j, k, a);
            gg += g[a] * g[a];
        }
        double den = sqrt(gg + P->delta * P->delta);
        for (int a = 0; a < P->dim; ++a)
            if (n[a]) n[a][c] = g[a] / den;
        if (gmag) gmag[c] = sqrt(gg);
    }
}

/* kappa = - sum_a C_a n_a  (positive for a drop with phi = 1 inside) */
void ora_curvature(const ora_params* P, const double* phi, double* kappa) {
    double* n[3] = {alloc0(P), alloc0(P), alloc0(P)};
    ora_normals(P, phi, n[0], n[1], n[2], NULL);
    FOR_CELLS(P) {
        double s = 0.0;
        for (int a = 0; a < P->dim; ++a) s += opC(P, n[a], KIND_ODD(a), i, j, k, a);
        kappa[at(P, i, j, k)] = -s;
    }
    for (int a = 0; a < 3; ++a) free(n[a]);
}

/* ---------------------------------------------------------------------- */
/* chemical potential (Eq. 2)                                             */
/* ---------------------------------------------------------------------- */

void ora_chem_potential(const ora_params* P, const double* phi, double* mu) {
    double sh_ = sigma_hat(P);
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        mu[c] = (sh_ / P->eps) * dpsi(phi[c]) - sh_ * P->eps * opL(P, phi, i, j, k);
    }
}

/* ---------------------------------------------------------------------- */
/* phase-field regularisation g (Table 1) and phase-field RHS (Eq. 1)     */
/* ---------------------------------------------------------------------- */

/* CDI face flux r_a = gamma [ eps G_a phi - A_a(phi (1-phi) n_a) ] */
void ora_cdi_flux(const ora_params* P, const double* phi, double* r0, double* r1,
                  double* r2) {
    double* r[3] = {r0, r1, r2};
    double* n[3] = {alloc0(P), alloc0(P), alloc0(P)};
    double* w[3] = {alloc0(P), alloc0(P), alloc0(P)};
    ora_normals(P, phi, n[0], n[1], n[2], NULL);
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        for (int a = 0; a < P->dim; ++a) w[a][c] = phi[c] * (1.0 - phi[c]) * n[a][c];
    }
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        for (int a = 0; a < P->dim; ++a)
            r[a][c] = P->gamma * (P->eps * opG(P, phi, i, j, k, a) - opA(P, w[a], KIND_ODD(a), i, j, k, a));
    }
    for (int a = 0; a < 3; ++a) { free(n[a]); free(w[a]); }
}

void ora_regularization(const ora_params* P, const double* phi, double* gphi) {
    if (P->model == ORA_CDI) {
        double* r[3] = {alloc0(P), alloc0(P), alloc0(P)};
        ora_cdi_flux(P, phi, r[0], r[1], r[2]);
        ora_divergence(P, r[0], r[1], r[2], gphi);
        for (int a = 0; a < 3; ++a) free(r[a]);
        return;
    }
    double* kappa = alloc0(P);
    double* gmag = alloc0(P);
    ora_curvature(P, phi, kappa);
    ora_normals(P, phi, NULL, NULL, NULL, gmag);
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        double f = phi[c];
        double base = P->eps * opL(P, phi, i, j, k) - dpsi(f) / P->eps;
        double curv = (P->model == ORA_SB) ? P->eps * gmag[c] * kappa[c]   /* SB    */
                                           : f * (1.0 - f) * kappa[c];     /* ISODI */
        gphi[c] = P->gamma * (base + curv);
    }
    free(kappa);
    free(gmag);
}

/* dphi/dt = - D(u A phi) + g   (Eq. 1 with central face interpolation) */
void ora_phase_rhs(const ora_params* P, const double* phi, const double* u0,
                   const double* u1, const double* u2, double* dphi) {
    const double* u[3] = {u0, u1, u2};
    double* J[3] = {alloc0(P), alloc0(P), alloc0(P)};
    double* g = alloc0(P);
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        for (int a = 0; a < P->dim; ++a)
            J[a][c] = fetch(P, u[a], KIND_FACE(a), i, j, k) * opA(P, phi, K_CELL, i, j, k, a);
    }
    ora_regularization(P, phi, g);
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        dphi[c] = -opD(P, J, i, j, k) + g[c];
    }
    for (int a = 0; a < 3; ++a) free(J[a]);
    free(g);
}

/* ---------------------------------------------------------------------- */
/* surface tension force on faces                                         */
/* ---------------------------------------------------------------------- */

void ora_surface_force(const ora_params* P, const double* phi, double* F0,
                       double* F1, double* F2) {
    double* F[3] = {F0, F1, F2};
    double sh_ = sigma_hat(P);
    double* mu = alloc0(P);
    double* kappa = alloc0(P);
    double* w = alloc0(P);
    if (P->force == ORA_EB || P->force == ORA_EB_GAUGE) ora_chem_potential(P, phi, mu);
    if (P->force == ORA_CSF || P->force == ORA_LCSF) ora_curvature(P, phi, kappa);
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        w[c] = phi[c] * (1.0 - phi[c]);
    }
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        for (int a = 0; a < P->dim; ++a) {
            double gphi = opG(P, phi, i, j, k, a);
            double f;
            switch (P->force) {
            case ORA_EB:   /* F = mu grad phi (Eq. 4), + sign on the momentum RHS */
                f = opA(P, mu, K_CELL, i, j, k, a) * gphi;
                break;
            case ORA_CSF:  /* F = sigma kappa grad phi */
                f = P->sigma * opA(P, kappa, K_CELL, i, j, k, a) * gphi;
                break;
            case ORA_LCSF: /* F = sigma_hat kappa phi(1-phi) grad phi (Eq. 11) */
                f = sh_ * opA(P, kappa, K_CELL, i, j, k, a) * opA(P, w, K_CELL, i, j, k, a) * gphi;
                break;
            default:       /* EB minus the gradient G(mu phi): -A(phi) G(mu) */
                f = -opA(P, phi, K_CELL, i, j, k, a) * opG(P, mu, i, j, k, a);
                break;
            }
            F[a][c] = f;
        }
    }
    free(mu);
    free(kappa);
    free(w);
}

/* ---------------------------------------------------------------------- */
/* momentum: mass flux, advection, viscous stress                         */
/* ---------------------------------------------------------------------- */

/* m_a = rho_a u_a - (rho1 - rho2) r_a for CDI (mass flux consistent with the
 * phase-field flux); m_a = rho_a u_a for the non-conservative models */
void ora_mass_flux(const ora_params* P, const double* phi, const double* u0,
                   const double* u1, const double* u2, double* m0, double* m1,
                   double* m2) {
    const double* u[3] = {u0, u1, u2};
    double* m[3] = {m0, m1, m2};
    double* r[3] = {alloc0(P), alloc0(P), alloc0(P)};
    if (P->model == ORA_CDI) ora_cdi_flux(P, phi, r[0], r[1], r[2]);
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        for (int a = 0; a < P->dim; ++a)
            m[a][c] = rho_face(P, phi, i, j, k, a) * fetch(P, u[a], KIND_FACE(a), i, j, k) -
                      (P->rho1 - P->rho2) * r[a][c];
    }
    for (int a = 0; a < 3; ++a) free(r[a]);
}

/* N_a = [div(m (x) u)]_a - u_a A_a(D m), on the u_a control volume.
 * b == a: flux at cell q,  Phi_aa[q] = avg(m_a over q's two a-faces) * avg(u_a same)
 * b != a: flux at the edge between faces (c,a) and (c+e_b,a),
 *         Phi_ba[c] = avg(m_b[c+e_b], m_b[c-e_a+e_b]) * avg(u_a[c], u_a[c+e_b]) */
void ora_advection(const ora_params* P, const double* m0, const double* m1,
                   const double* m2, const double* u0, const double* u1,
                   const double* u2, double* N0, double* N1, double* N2) {
    const double* m[3] = {m0, m1, m2};
    const double* u[3] = {u0, u1, u2};
    double* N[3] = {N0, N1, N2};
    double* Dm = alloc0(P);
    ora_divergence(P, m0, m1, m2, Dm);
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        for (int a = 0; a < P->dim; ++a) {
            const int fa = KIND_FACE(a);
            double s = 0.0;
            for (int b = 0; b < P->dim; ++b) {
                double phi_hi, phi_lo;
                if (b == a) {
                    double mc = fetch(P, m[a], fa, i, j, k), uc = fetch(P, u[a], fa, i, j, k);
                    double mp = fsh(P, m[a], fa, i, j, k, a, 1), up = fsh(P, u[a], fa, i, j, k, a, 1);
                    double mm = fsh(P, m[a], fa, i, j, k, a, -1), um = fsh(P, u[a], fa, i, j, k, a, -1);
                    phi_hi = 0.5 * (mc + mp) * 0.5 * (uc + up);
                    phi_lo = 0.5 * (mm + mc) * 0.5 * (um + uc);
                } else {
                    const int fb = KIND_FACE(b);
                    /* edge flux at (c) and at (c - e_b) */
                    phi_hi = 0.5 * (fsh(P, m[b], fb, i, j, k, b, 1) + fsh2(P, m[b], fb, i, j, k, a, -1, b, 1)) *
                             0.5 * (fetch(P, u[a], fa, i, j, k) + fsh(P, u[a], fa, i, j, k, b, 1));
                    phi_lo = 0.5 * (fetch(P, m[b], fb, i, j, k) + fsh(P, m[b], fb, i, j, k, a, -1)) *
                             0.5 * (fsh(P, u[a], fa, i, j, k, b, -1) + fetch(P, u[a], fa, i, j, k));
                }
                s += (phi_hi - phi_lo) / P->h;
            }
            N[a][c] = s - fetch(P, u[a], fa, i, j, k) * opA(P, Dm, K_CELL, i, j, k, a);
        }
    }
    free(Dm);
}

void ora_viscosity_field(const ora_params* P, const double* phi, double* visc) {
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        visc[c] = visc_of(P, phi[c]);
    }
}

/* shear stress tau_ab on the edge shared by faces (c,a) and (c+e_b,a), c=(i,j,k):
 * edge viscosity = mean of the 4 cells around the edge */
static double edge_tau(const ora_params* P, const double* eta, const double* const u[3],
                       int a, int b, int i, int j, int k) {
    double eta_e = 0.25 * (fetch(P, eta, K_CELL, i, j, k) + fsh(P, eta, K_CELL, i, j, k, a, -1) +
                           fsh(P, eta, K_CELL, i, j, k, b, 1) + fsh2(P, eta, K_CELL, i, j, k, a, -1, b, 1));
    double dua_db = (fsh(P, u[a], KIND_FACE(a), i, j, k, b, 1) - fetch(P, u[a], KIND_FACE(a), i, j, k)) / P->h;
    double dub_da = (fsh(P, u[b], KIND_FACE(b), i, j, k, b, 1) - fsh2(P, u[b], KIND_FACE(b), i, j, k, a, -1, b, 1)) / P->h;
    return eta_e * (dua_db + dub_da);
}

/* V_a = [div(eta (grad u + grad u^T))]_a on the u_a control volume */
void ora_viscous(const ora_params* P, const double* eta, const double* u0,
                 const double* u1, const double* u2, double* V0, double* V1,
                 double* V2) {
    const double* const u[3] = {u0, u1, u2};
    double* V[3] = {V0, V1, V2};
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        for (int a = 0; a < P->dim; ++a) {
            const int fa = KIND_FACE(a);
            double s = 0.0;
            for (int b = 0; b < P->dim; ++b) {
                if (b == a) {
                    double uc = fetch(P, u[a], fa, i, j, k);
                    double t_hi = 2.0 * eta[c] * (fsh(P, u[a], fa, i, j, k, a, 1) - uc) / P->h;   /* at cell c     */
                    double t_lo = 2.0 * fsh(P, eta, K_CELL, i, j, k, a, -1) *
                                  (uc - fsh(P, u[a], fa, i, j, k, a, -1)) / P->h;               /* at cell c-e_a */
                    s += (t_hi - t_lo) / P->h;
                } else {
                    int v[3] = {i, j, k};
                    v[b] -= 1;
                    double t_hi = edge_tau(P, eta, u, a, b, i, j, k);
                    double t_lo = edge_tau(P, eta, u, a, b, v[0], v[1], v[2]);
                    s += (t_hi - t_lo) / P->h;
                }
            }
            V[a][c] = s;
        }
    }
}

/* f*_a = (-N_a + V_a + F_a) / rho_a   (no body force) */
void ora_fstar(const ora_params* P, const double* phi, const double* u0,
               const double* u1, const double* u2, double* f0, double* f1,
               double* f2) {
    const double* u[3] = {u0, u1, u2};
    double* f[3] = {f0, f1, f2};
    double *F[3], *m[3], *N[3], *V[3];
    for (int a = 0; a < 3; ++a) {
        F[a] = alloc0(P); m[a] = alloc0(P); N[a] = alloc0(P); V[a] = alloc0(P);
    }
    double* eta = alloc0(P);
    double* uz = alloc0(P);
    const double* uu[3] = {u[0], u[1], u[2] ? u[2] : uz};
    ora_surface_force(P, phi, F[0], F[1], F[2]);
    ora_mass_flux(P, phi, uu[0], uu[1], uu[2], m[0], m[1], m[2]);
    ora_advection(P, m[0], m[1], m[2], uu[0], uu[1], uu[2], N[0], N[1], N[2]);
    ora_viscosity_field(P, phi, eta);
    ora_viscous(P, eta, uu[0], uu[1], uu[2], V[0], V[1], V[2]);
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        for (int a = 0; a < P->dim; ++a)
            f[a][c] = (-N[a][c] + V[a][c] + F[a][c]) * beta_face(P, phi, i, j, k, a);
    }
    for (int a = 0; a < 3; ++a) { free(F[a]); free(m[a]); free(N[a]); free(V[a]); }
    free(eta);
    free(uz);
}

/* ---------------------------------------------------------------------- */
/* variable-density pressure Poisson equation                             */
/* ---------------------------------------------------------------------- */

/* beta_a on every face (reads through fetch() give 0 on wall faces: no
 * flux through a wall) */
static void face_betas(const ora_params* P, const double* phi, double* beta[3]) {
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        for (int a = 0; a < P->dim; ++a) beta[a][c] = beta_face(P, phi, i, j, k, a);
    }
}

/* y = D(beta G x) */
static void apply_with(const ora_params* P, double* const beta[3], const double* x, double* y) {
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        double s = 0.0;
        for (int a = 0; a < P->dim; ++a) {
            double flux_hi = fsh(P, beta[a], KIND_FACE(a), i, j, k, a, 1) *
                             (fsh(P, x, K_CELL, i, j, k, a, 1) - x[c]) / P->h;
            double flux_lo = fetch(P, beta[a], KIND_FACE(a), i, j, k) * opG(P, x, i, j, k, a);
            s += (flux_hi - flux_lo) / P->h;
        }
        y[c] = s;
    }
}

void ora_poisson_apply(const ora_params* P, const double* phi, const double* x, double* y) {
    double* beta[3] = {alloc0(P), alloc0(P), alloc0(P)};
    face_betas(P, phi, beta);
    apply_with(P, beta, x, y);
    for (int a = 0; a < 3; ++a) free(beta[a]);
}

/* Solve D(beta G x) = b - mean(b) with mean(x) = 0.  The pressure is the
 * exact solution of this singular-but-consistent system; any convergent
 * method gives it.  Here: conjugate gradients on the SPD form
 * -D(beta G) with a diagonal (Jacobi) preconditioner, from the warm start in
 * x, until ||r||_2 <= rtol ||rhs||_2.  Returns 0, or -1 if maxit is hit. */
int ora_poisson_solve(const ora_params* P, const double* phi, const double* b,
                      double* x, int* iters, double* relres) {
    long N = ncell(P);
    double* beta[3] = {alloc0(P), alloc0(P), alloc0(P)};
    double *f = alloc0(P), *r = alloc0(P), *z = alloc0(P), *p = alloc0(P),
           *q = alloc0(P), *dg = alloc0(P);
    face_betas(P, phi, beta);
    double h2 = P->h * P->h;
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        double s = 0.0;
        for (int a = 0; a < P->dim; ++a)
            s += fetch(P, beta[a], KIND_FACE(a), i, j, k) + fsh(P, beta[a], KIND_FACE(a), i, j, k, a, 1);
        dg[c] = s / h2;
    }
    double bmean = dot(P, b, NULL) / (double)N;
    for (long c = 0; c < N; ++c) f[c] = -(b[c] - bmean);      /* SPD form */
    double xmean = dot(P, x, NULL) / (double)N;
    for (long c = 0; c < N; ++c) x[c] -= xmean;
    double fnorm = sqrt(dot(P, f, f));
    int it = 0, rc = 0;
    if (fnorm == 0.0) {
        for (long c = 0; c < N; ++c) x[c] = 0.0;
    } else {
        apply_with(P, beta, x, q);
        for (long c = 0; c < N; ++c) r[c] = f[c] + q[c];      /* f - (-A x) */
        for (long c = 0; c < N; ++c) z[c] = r[c] / dg[c];
        memcpy(p, z, sizeof(double) * N);
        double rz = dot(P, r, z);
        double rnorm = sqrt(dot(P, r, r));
        while (rnorm > P->poisson_rtol * fnorm) {
            if (it >= P->poisson_maxit) { rc = -1; break; }
            apply_with(P, beta, p, q);
            for (long c = 0; c < N; ++c) q[c] = -q[c];
            double alpha = rz / dot(P, p, q);
            for (long c = 0; c < N; ++c) { x[c] += alpha * p[c]; r[c] -= alpha * q[c]; }
            rnorm = sqrt(dot(P, r, r));
            ++it;
            for (long c = 0; c < N; ++c) z[c] = r[c] / dg[c];
            double rz_new = dot(P, r, z);
            double bet = rz_new / rz;
            rz = rz_new;
            for (long c = 0; c < N; ++c) p[c] = z[c] + bet * p[c];
        }
        xmean = dot(P, x, NULL) / (double)N;
        for (long c = 0; c < N; ++c) x[c] -= xmean;
    }
    if (iters) *iters = it;
    if (relres) {
        if (fnorm == 0.0) {
            *relres = 0.0;
        } else {
            apply_with(P, beta, x, q);
            for (long c = 0; c < N; ++c) r[c] = f[c] + q[c];
            *relres = sqrt(dot(P, r, r)) / fnorm;
        }
    }
    for (int a = 0; a < 3; ++a) free(beta[a]);
    free(f); free(r); free(z); free(p); free(q); free(dg);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* stage derivative and classical RK4 with a projection at every stage    */
/* ---------------------------------------------------------------------- */

/* (dphi/dt, du/dt) at state (phi, u); pres: warm start in, pressure out.
 * du_a/dt = f*_a - beta_a G_a p  with  D(beta G p) = D f*. */
int ora_stage(const ora_params* P, const double* phi, const double* u0,
              const double* u1, const double* u2, double* dphi, double* du0,
              double* du1, double* du2, double* pres) {
    double* du[3] = {du0, du1, du2};
    double* fs[3] = {alloc0(P), alloc0(P), alloc0(P)};
    double* b = alloc0(P);
    double* uz = alloc0(P);
    ora_phase_rhs(P, phi, u0, u1, u2 ? u2 : uz, dphi);
    ora_fstar(P, phi, u0, u1, u2, fs[0], fs[1], fs[2]);
    ora_divergence(P, fs[0], fs[1], fs[2], b);
    int it;
    double rr;
    int rc = ora_poisson_solve(P, phi, b, pres, &it, &rr);
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        for (int a = 0; a < P->dim; ++a)
            du[a][c] = fs[a][c] - beta_face(P, phi, i, j, k, a) * opG(P, pres, i, j, k, a);
    }
    for (int a = 0; a < 3; ++a) free(fs[a]);
    free(b);
    free(uz);
    return rc;
}

/* nsteps classical RK4 steps of size dt, in place.  y_{n+1} = y_n +
 * dt/6 (k1 + 2 k2 + 2 k3 + k4) with k_s the projected stage derivatives.
 * pres is the Poisson warm start; on return it holds the last stage's p. */
int ora_step(const ora_params* P, double dt, int nsteps, double* phi, double* u0,
             double* u1, double* u2, double* pres) {
    long N = ncell(P);
    int d = P->dim;
    double* y[4] = {phi, u0, u1, u2};
    double* ys[4];
    double* kk[4][4];
    for (int v = 0; v < 4; ++v) {
        ys[v] = alloc0(P);
        for (int s = 0; s < 4; ++s) kk[s][v] = alloc0(P);
    }
    const double cstage[4] = {0.0, 0.5, 0.5, 1.0};
    int rc = 0;
    for (int n = 0; n < nsteps && rc == 0; ++n) {
        for (int s = 0; s < 4 && rc == 0; ++s) {
            for (int v = 0; v <= d; ++v)
                for (long c = 0; c < N; ++c)
                    ys[v][c] = (s == 0) ? y[v][c] : y[v][c] + cstage[s] * dt * kk[s - 1][v][c];
            rc = ora_stage(P, ys[0], ys[1], ys[2], d == 3 ? ys[3] : NULL, kk[s][0], kk[s][1],
                           kk[s][2], kk[s][3], pres);
        }
        if (rc != 0) break;
        for (int v = 0; v <= d; ++v)
            for (long c = 0; c < N; ++c)
                y[v][c] = y[v][c] + dt / 6.0 * (kk[0][v][c] + 2.0 * kk[1][v][c] +
                                                2.0 * kk[2][v][c] + kk[3][v][c]);
    }
    for (int v = 0; v < 4; ++v) {
        free(ys[v]);
        for (int s = 0; s < 4; ++s) free(kk[s][v]);
    }
    return rc;
}

/* ---------------------------------------------------------------------- */
/* initial droplet: equilibrium tanh profile in the signed distance       */
/* ---------------------------------------------------------------------- */

/* phi = [1 + tanh(s / (2 eps))] / 2 (Eq. 2 footnote).  For an ellipse or
 * ellipsoid with semi-axes a_i the signed distance is approximated to first
 * order by s = (1 - q) / |grad q|, q = sqrt(sum (x_i / a_i)^2), exact for a
 * circle or sphere; at the centre s = min a_i.  x_i is the minimum-image
 * offset of the cell centre from the droplet centre. */
void ora_init_droplet(const ora_params* P, const double center[3],
                      const double semi_axes[3], double* phi) {
    double Lx[3] = {P->n[0] * P->h, P->n[1] * P->h, P->n[2] * P->h};
    FOR_CELLS(P) {
        int v[3] = {i, j, k};
        double q2 = 0.0, g2 = 0.0, amin = semi_axes[0];
        for (int a = 0; a < P->dim; ++a) {
            double x = (v[a] + 0.5) * P->h - center[a];
            if (!walled(P, a)) x -= Lx[a] * floor(x / Lx[a] + 0.5);   /* minimum image */
            q2 += (x / semi_axes[a]) * (x / semi_axes[a]);
            g2 += x * x / (semi_axes[a] * semi_axes[a] * semi_axes[a] * semi_axes[a]);
            if (semi_axes[a] < amin) amin = semi_axes[a];
        }
        double q = sqrt(q2);
        double s = (q2 == 0.0) ? amin : (1.0 - q) * q / sqrt(g2);
        phi[at(P, i, j, k)] = 0.5 * (1.0 + tanh(s / (2.0 * P->eps)));
    }
}

/* ---------------------------------------------------------------------- */
/* diagnostics                                                            */
/* ---------------------------------------------------------------------- */

void ora_diagnostics(const ora_params* P, const double* phi, const double* u0,
                     const double* u1, const double* u2, const double* pres,
                     double* out) {
    const double* u[3] = {u0, u1, u2};
    long N = ncell(P);
    double hd = pow(P->h, P->dim);
    double sh_ = sigma_hat(P);
    double *speed = alloc0(P), *ke = alloc0(P), *se = alloc0(P), *dv = alloc0(P);
    double *pin = alloc0(P), *pout = alloc0(P), *min_ = alloc0(P), *mout = alloc0(P);
    FOR_CELLS(P) {
        long c = at(P, i, j, k);
        double s2 = 0.0, kin = 0.0, grad2 = 0.0, div = 0.0;
        for (int a = 0; a < P->dim; ++a) {
            double uc = fetch(P, u[a], KIND_FACE(a), i, j, k), up = fsh(P, u[a], KIND_FACE(a), i, j, k, a, 1);
            double ubar = 0.5 * (uc + up);    /* cell-averaged velocity */
            s2 += ubar * ubar;
            kin += 0.5 * rho_face(P, phi, i, j, k, a) * uc * uc;
            double g = opG(P, phi, i, j, k, a);
            grad2 += g * g;
            div += (up - uc) / P->h;
        }
        speed[c] = sqrt(s2);
        ke[c] = kin;
        /* free energy density (sigma_hat/eps) psi + (1/2) sigma_hat eps |grad phi|^2 */
        se[c] = (sh_ / P->eps) * psi(phi[c]) + 0.5 * sh_ * P->eps * grad2;
        dv[c] = fabs(div);
        if (pres) {
            if (phi[c] > 0.99) { pin[c] = pres[c]; min_[c] = 1.0; }
            if (phi[c] < 0.01) { pout[c] = pres[c]; mout[c] = 1.0; }
        }
    }
    double umax = 0.0, fmin = phi[0], fmax = phi[0], dmax = 0.0;
    for (long c = 0; c < N; ++c) {
        if (speed[c] > umax) umax = speed[c];
        if (phi[c] < fmin) fmin = phi[c];
        if (phi[c] > fmax) fmax = phi[c];
        if (dv[c] > dmax) dmax = dv[c];
    }
    out[ORA_D_MASS] = hd * dot(P, phi, NULL);
    out[ORA_D_PHIMIN] = fmin;
    out[ORA_D_PHIMAX] = fmax;
    out[ORA_D_UMAX] = umax;
    out[ORA_D_CAINF] = umax * P->visc1 / P->sigma;
    out[ORA_D_KE] = hd * dot(P, ke, NULL);
    out[ORA_D_SE] = hd * dot(P, se, NULL);
    if (pres) {
        double ni = dot(P, min_, NULL), no = dot(P, mout, NULL);
        out[ORA_D_DP] = (ni > 0 && no > 0) ? dot(P, pin, NULL) / ni - dot(P, pout, NULL) / no : NAN;
    } else {
        out[ORA_D_DP] = NAN;
    }
    out[ORA_D_DIVMAX] = dmax;
    free(speed); free(ke); free(se); free(dv); free(pin); free(pout); free(min_); free(mout);
}

int ora_threads(void) { return omp_get_max_threads(); }

/* set the OpenMP thread count of later calls; returns the previous count */
int ora_set_threads(int n) {
    const int prev = omp_get_max_threads();
    if (n > 0) omp_set_num_threads(n);
    return prev;
}
