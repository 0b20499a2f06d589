/*
 * Plain FP64 CPU oracle for one time step of the two-phase phase-field solver
 * of Mirjalili, Khanwale & Mani, "Assessment of an energy-based surface tension
 * model for simulation of two-phase flows using second-order phase field
 * methods" (arXiv 2205.05835).
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU
 * baseline leg of the benchmark call this library; the product (the HIP
 * library under paper_2205_05835_amd/) never links, includes or calls it, and
 * this file includes nothing from the product.
 *
 * Grid: uniform, cells indexed c = (k*ny + j)*nx + i (x fastest); each axis
 * periodic, or bounded by free-slip walls at both ends (ora_params.walls).
 * phi, p, mu, kappa live at cell centres; the velocity component u_a[c] lives
 * on the LOWER a-face of cell c, between c - e_a and c (staggered MAC grid,
 * Sec. 3 opening paragraph).  In 2D, n[2] = 1 and only axes 0,1 are used.
 */
#ifndef TPF_ORACLE_H
#define TPF_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_CDI = 0, ORA_SB = 1, ORA_ISODI = 2 };          /* Table 1 */
enum { ORA_EB = 0, ORA_CSF = 1, ORA_LCSF = 2,             /* Eq. 4, CSF, LCSF */
       ORA_EB_GAUGE = 3 };  /* -A(phi) G(mu): Eq. 4 minus a face gradient (Eq. 7) */

typedef struct {
    int dim;            /* 2 or 3 */
    int n[3];           /* cells per axis, n[2] = 1 in 2D */
    double h;           /* uniform spacing */
    int model;          /* ORA_CDI / ORA_SB / ORA_ISODI */
    int force;          /* ORA_EB / ORA_CSF / ORA_LCSF / ORA_EB_GAUGE */
    double sigma;       /* surface tension coefficient; sigma_hat = 6 sigma */
    double eps;         /* interface thickness epsilon */
    double gamma;       /* mobility / velocity scale of the regularisation */
    double rho1, rho2;  /* density of phase phi=1 and phi=0 */
    double visc1, visc2;/* dynamic viscosity of phase phi=1 and phi=0 */
    double delta;       /* normal regularisation: n = g / sqrt(g.g + delta^2) */
    int clamp;          /* clamp phi to [0,1] inside the property laws */
    double poisson_rtol;/* stop when ||r||_2 <= rtol ||rhs||_2 */
    int poisson_maxit;
    int walls;          /* bit a set: free-slip walls at both ends of axis a, else periodic */
} ora_params;

/* -- operators (each writes full arrays of n[0]*n[1]*n[2] doubles) -------- */
void ora_normals(const ora_params* P, const double* phi, double* nx, double* ny,
                 double* nz, double* gmag);
void ora_curvature(const ora_params* P, const double* phi, double* kappa);
void ora_chem_potential(const ora_params* P, const double* phi, double* mu);
void ora_regularization(const ora_params* P, const double* phi, double* gphi);
void ora_cdi_flux(const ora_params* P, const double* phi, double* r0, double* r1,
                  double* r2);
void ora_phase_rhs(const ora_params* P, const double* phi, const double* u0,
                   const double* u1, const double* u2, double* dphi);
void ora_surface_force(const ora_params* P, const double* phi, double* F0,
                       double* F1, double* F2);
void ora_mass_flux(const ora_params* P, const double* phi, const double* u0,
                   const double* u1, const double* u2, double* m0, double* m1,
                   double* m2);
void ora_advection(const ora_params* P, const double* m0, const double* m1,
                   const double* m2, const double* u0, const double* u1,
                   const double* u2, double* N0, double* N1, double* N2);
void ora_viscous(const ora_params* P, const double* visc, const double* u0,
                 const double* u1, const double* u2, double* V0, double* V1,
                 double* V2);
void ora_viscosity_field(const ora_params* P, const double* phi, double* visc);
void ora_fstar(const ora_params* P, const double* phi, const double* u0,
               const double* u1, const double* u2, double* f0, double* f1,
               double* f2);
void ora_divergence(const ora_params* P, const double* F0, const double* F1,
                    const double* F2, double* out);

/* -- pressure: D(beta G p) = b - mean(b), mean(p) = 0 ------------------- */
void ora_poisson_apply(const ora_params* P, const double* phi, const double* x,
                       double* y);
int ora_poisson_solve(const ora_params* P, const double* phi, const double* b,
                      double* x, int* iters, double* relres);

/* -- stage derivative and RK4 step -------------------------------------- */
int ora_stage(const ora_params* P, const double* phi, const double* u0,
              const double* u1, const double* u2, double* dphi, double* du0,
              double* du1, double* du2, double* pres);
int ora_step(const ora_params* P, double dt, int nsteps, double* phi, double* u0,
             double* u1, double* u2, double* pres);

/* -- initial state and diagnostics -------------------------------------- */
void ora_init_droplet(const ora_params* P, const double center[3],
                      const double semi_axes[3], double* phi);

enum { ORA_D_MASS = 0, ORA_D_PHIMIN, ORA_D_PHIMAX, ORA_D_UMAX, ORA_D_CAINF,
       ORA_D_KE, ORA_D_SE, ORA_D_DP, ORA_D_DIVMAX, ORA_D_COUNT };
void ora_diagnostics(const ora_params* P, const double* phi, const double* u0,
                     const double* u1, const double* u2, const double* pres,
                     double* out);

/* number of OpenMP threads the oracle's parallel loops use */
int ora_threads(void);
int ora_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
