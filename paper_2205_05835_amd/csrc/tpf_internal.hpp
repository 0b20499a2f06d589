// Host-side internals shared by the translation units of the library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/tpf.h"
#include "tpf_device.hpp"
#include "tpf_stage_ops.hpp"

namespace tpf {

// Mixed-precision pressure solves: each FP32 inner solve aims at this
// fraction of the residual reduction the FP64 outer tolerance still needs
// (the FP64 residual after the correction decides; a shortfall costs one more
// outer pass).  Measured on the 256^3 drop, 256^2 drops at density ratio
// 1000 and 2D/3D oscillating drops: as many outer passes at 0.9 as at 0.5,
// and 3.05 instead of 3.67 inner iterations per solve at 256^3.
constexpr double INNER_MARGIN = 0.9;


constexpr int MAX_LEVELS = 16;

// Device-resident scalars of the pressure solver.  Kernels read alpha/beta/
// mean from here, and every solver kernel returns at once when done != 0, so
// a batch of iterations can be queued without a host round trip.
struct SolverScalars {
    double mean;       // mean of the Poisson right-hand side b
    double ff;         // ||f||^2 of the system being solved
    double rr;         // ||r||^2 of the current residual
    double rz;         // <r, z>
    double pq;         // <p, A p>
    double alpha, beta;
    double tol2;       // stop when rr <= tol2 * ff
    double sum;        // generic sum (mean removal)
    double floor2;     // explicit residuals: squared rounding level of their FP64 evaluation
    int done;          // PCG finished (converged, or no work)
    int iters;         // PCG iterations performed
    int pad[2];
};

// The solver scalars as a kernel publishes them into pinned host memory:
// token is written last, after a system-scope fence, so a host that reads
// the token it asked for then reads a complete copy.
struct PubScalars {
    SolverScalars s;
    int token;
    int flag;      // the step's non-finite flag (k_publish_flag)
    int pad[2];
};


// Finalize operations on reduced partial sums (one single-block kernel).
enum FinOp {
    FIN_MEAN = 0,   // v0 = sum b           -> mean = v0 / N
    FIN_INIT = 1,   // v0 = ff, v1 = rr, v2 = |A||x| squared -> ff, rr, floor2,
                    //                  done = rr <= max(tol2 ff, floor2)
    FIN_RZ0 = 2,    // v0 = rz              -> rz (first), keeps done
    FIN_ALPHA = 3,  // v0 = pq              -> alpha = rz / pq
    FIN_BETA = 4,   // v0 = rr, v1 = rz_new, v2 = <A p, z_new> -> beta = -v2 / pq, rz, rr, done, iters++
    FIN_SUM = 5     // v0 = sum x           -> sum
};

struct Level {
    int n[3];
    long N;
    double h;
    void* beta[3];  // face coefficients 1/rho_a (solver precision)
    void* z;        // correction / PCG preconditioned residual at level 0
    void* zt;       // Jacobi ping-pong partner of z
    void* r;        // right-hand side (level 0: the PCG residual)
    void* dinv;     // coarse levels: 1 / diagonal, for the fused first two sweeps
};

// Kernel classes for the optional per-launch timing.  Each fine-level (level
// 0) solver class is one kernel symbol, so its timing can be compared with a
// profiler's per-kernel statistics.
enum ProfClass {
    PC_CELL = 0, PC_KAPPA, PC_FACE, PC_PHASE, PC_MOM, PC_DIV, PC_PROJ,
    PC_F_APPLY, PC_F_FIRST, PC_F_FIRST0, PC_F_SWEEP, PC_F_RESTRICT, PC_F_PROLONG, PC_F_SWEEPDOT,
    PC_COARSE_LEVELS, PC_RESID, PC_FINALIZE, PC_VECTOR,
    // backward-Euler ISODI phase-field step
    PC_IMP_NORMALS, PC_IMP_RESIDUAL, PC_IMP_DN, PC_IMP_APPLY, PC_IMP_VECTOR, PC_IMP_FINALIZE, PC_COUNT
};
constexpr int NPROF = PC_COUNT;

}  // namespace tpf

struct tpf_ctx {
    tpf_params P;
    int dim;
    int n[3];
    long N;
    double h;
    int mixed;           // 0: FP64, 1: FP32 state + FP64 pressure
    int march;           // 3D level 0 uses the z-marching kernels (TPF_MARCH=0 disables)
    int no_tail;         // TPF_TAIL=0: run every level with separate kernels
    size_t tsz;          // bytes per state value
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    int device;

    // state (precision T), four slots per variable; roles below
    void* phi[4];
    void* u[3][4];
    int s_yn, s_acc, s_y1, s_y2;

    // stage intermediates (T)
    void* nrm[3];
    void* mu;
    void* kappa;
    void* rflux[3];
    void* mflux[3];
    void* fs[3];
    void* force[3];      // only filled when tpf_eval_field asks for it

    // pressure (FP64)
    double* b;           // D f* (Poisson right-hand side)
    double* p;           // pressure = solver x (warm start)
    double* p_alt;       // the next stage's starting guess, written by the
                         // projection; the step then swaps it with p
    // PCG vectors at level 0 (solver precision S)
    void* pv;            // search direction
    void* pv2;           // search direction, ping-pong partner
    void* qv;            // A p
    void* ev;            // mixed: inner solution (correction)
    void* rhoh;          // fine-level half density rho(phi)/2 (solver precision)
    tpf::Level lv[tpf::MAX_LEVELS];
    int nlev;

    // reductions
    double* partials;
    long max_blocks;
    tpf::SolverScalars* scal;   // device
    int* flags;                 // device: [0] non-finite seen
    void* imp_scal;             // device: scalars of the implicit phase-field step (256 bytes)
    double* diag_part;          // per-block diagnostic partials
    double* diag_out;           // finalized diagnostics

    // bookkeeping
    double t;
    long step;
    double mass0;
    int p_valid;         // ctx->p holds the projection pressure of the current state
    // pressure history for the warm starts: p_hist1 = stage-1 pressure of
    // the current step (time t_n); p_hist2 = stage-2 pressure (t_n + dt/2,
    // of the previous step until stage 2 of this one); p_hist3 = stage-3
    // minus stage-2 pressure of the previous step
    double* p_hist1;
    double* p_hist2;
    double* p_hist3;
    int hist2_valid;
    // set by the step for one stage: the projection also writes the stage's
    // pressure into proj_hist (minus proj_hsub when that is set), and, when
    // proj_guess is set, proj_ga p + proj_gb proj_gsrc into p_alt (the array
    // beside p; the step swaps the two after the stage)
    double* proj_hist;
    const double* proj_hsub;
    int proj_guess;
    const double* proj_gsrc;
    double proj_ga, proj_gb;
    double last_relres;
    int last_outer, last_inner;
    long long stat_solves, stat_outer, stat_inner;   // pressure solves since the last reset
    int stat_recent[4];                              // PCG iterations of the last four solves

    // pairs of PCG iterations replayed from HIP graphs (TPF_PCG_GRAPH=1, a
    // measurement knob; off while profiling): captured on cap_stream, keyed
    // by the correction array and the direction buffer the pair starts from
    int pcg_graph;
    hipStream_t cap_stream;
    struct PcgGraph {
        const void* key[2];
        hipGraphExec_t exec;
    };
    PcgGraph pcg_graphs[4];
    int n_pcg_graphs;

    // profiling: HIP event pairs around the launches of the selected classes
    unsigned prof_mask;
    int ev_cap;
    hipEvent_t* ev_a;
    hipEvent_t* ev_b;
    int* ev_class;
    double* ev_bytes;
    int ev_count;
    int ev_open;         // a begin event is recorded and awaits its end
    double prof_ms[tpf::NPROF];
    long prof_launches[tpf::NPROF];
    double prof_bytes[tpf::NPROF];
    // launches issued per class (counted at issue, independent of the event
    // pool) and the part of them that found the solve already converged and
    // did no work: those count in the time, not in launches or bytes
    long prof_issued[tpf::NPROF];
    double prof_issued_bytes[tpf::NPROF];
    long prof_noop[tpf::NPROF];
    double prof_noop_bytes[tpf::NPROF];

    // adjoint scratch (contexts created with params.adjoint = 1):
    // adj_fields(dim) FP64 cell/face arrays of adj_stride elements each, then
    // the two parameter-gradient accumulators
    double* adj;
    long adj_stride;

    // PCG iterations of the previous solve of each kind (0: FP64 solve,
    // 1 + o: inner solve of outer iteration o); the host checks convergence
    // first after that many iterations
    int pred_iters[4][4];   // PCG iterations of the last solve of each kind (slot) and RK stage
    int rk_stage;           // RK stage of the solve under way (0 outside a step)
    int kz_override;     // planes per block of the z-marching kernels (0: automatic)
    int stage_kz;        // planes per block of the z-chunked stage kernels
    int stage_lds;       // 3D phase/momentum pass with its neighbourhoods staged in LDS
    int walls;           // bit a: free-slip walls at both ends of axis a
    int stage_lds_kz;    // planes per block of that pass
    int coarse_fused;    // 3D stored-coefficient levels: one fused launch down and one up
    tpf::PubScalars* pub;     // pinned host buffer for the solver scalars (null: copy and synchronise)
    tpf::PubScalars* pub_dev; // its device address
    int pub_token;       // last token asked for
    double mg_alpha;     // weight of the multigrid coarse-grid correction
    int coarse_sweeps_per_cell;   // coarsest-grid Jacobi sweeps per cell of its largest dimension (0: 2)
    // measurement mode with a fixed amount of solver work per pressure solve
    // (TPF_FIXED_PCG=outer,inner): exactly fixed_outer defect-correction passes
    // of exactly fixed_inner PCG iterations (FP64: one PCG of fixed_inner), no
    // convergence test; 0: off
    int fixed_outer, fixed_inner;
};

namespace tpf {

// validated copy of a parameter set with the defaults filled in
tpf_status resolve_params(const tpf_params* in, tpf_params* out);
Phys phys_of_params(const tpf_params& P);
void set_error(const std::string& msg);
tpf_status hip_fail(hipError_t e, const char* what);

// profiling hooks around launches
void prof_begin(tpf_ctx* c, int cls, double bytes);
void prof_end(tpf_ctx* c);

// stage kernels (tpf_stage.hip)
// normals: also store n (the step skips it where nothing reads it: the LDS
// pass with CDI and the energy-based force, which needs no kappa)
hipError_t launch_stage_fields(tpf_ctx* c, const void* phi_s, const void* const u_s[3], bool normals = true);
hipError_t launch_momentum(tpf_ctx* c, const void* phi_s, const void* const u_s[3], int want_force);
// phase update and momentum right-hand side fused (one pass over phi and u)
hipError_t launch_phase_momentum(tpf_ctx* c, const void* phi_s, const void* const u_s[3], const RKArgs& rk,
                                 void* out, int want_force);
hipError_t launch_divergence(tpf_ctx* c);
hipError_t launch_project_update(tpf_ctx* c, const void* phi_s, const RKArgs& rk, void* const out[3]);
hipError_t launch_init_droplet(tpf_ctx* c, const double center[3], const double axes[3]);
hipError_t launch_convert_in(tpf_ctx* c, const double* src, void* dst);
hipError_t launch_convert_out(tpf_ctx* c, const void* src, double* dst);
hipError_t launch_zero_state(tpf_ctx* c, void* dst);
hipError_t launch_diagnostics(tpf_ctx* c, const void* phi, const void* const u[3], const double* p);
// the same reduction on explicit arrays (fp32: phi and u are float) into the
// block partials `part` (ND_SUM + ND_MAX values per block of grid_of(n)) and
// the final sums `out` (ND_SUM + ND_MAX values)
hipError_t launch_diagnostics_arrays(hipStream_t st, int dim, const int n[3], int walls, int fp32, const Phys& P,
                                     const void* phi, const void* const u[3], const double* p, double* part,
                                     double* out);
int xcd_tiles_from_env();

// pressure solver (tpf_poisson.hip)
tpf_status poisson_solve(tpf_ctx* c, const void* phi, int* iters, double* relres, int* outer);
tpf_status gauge_pressure(tpf_ctx* c);    // subtract the mean of c->p
// advance nsteps RK4 steps; with a tape, record every stage's input state and
// its pressure (stage_bytes per stage, layout of the adjoint tape)
tpf_status advance(tpf_ctx* c, double dt, int nsteps, char* tape, size_t stage_bytes);
// one stage evaluation at the current state (pressure to c->p)
tpf_status eval_current(tpf_ctx* c, int want_force);
// FP64 fields of the adjoint scratch: 4 groups of (1 + dim) state
// cotangents, 4 groups of dim face cotangents and 7 cell fields
inline int adj_fields(int dim) { return 4 * (1 + dim) + 4 * dim + 7; }
size_t align256(size_t x);
hipError_t launch_finalize(tpf_ctx* c, int nblocks, int nv, int op);
hipError_t launch_rhs_mean(tpf_ctx* c);
// the step's non-finite flag as it stands after the work queued so far
// (through the pinned buffer when there is one)
hipError_t fetch_flag(tpf_ctx* c, int* flag);
// nbytes of device memory to the host after the work queued so far (through
// the pinned buffer when there is one and the bytes fit it)
hipError_t fetch_bytes(tpf_ctx* c, const void* dev, size_t nbytes, void* host);

// 1D grid over gx*gy*gz tiles, padded to a multiple of the XCD count
inline dim3 tile_grid(long gx, long gy, long gz) {
    const long nt = gx * gy * gz;
    return dim3((unsigned)((nt + NXCD - 1) / NXCD * NXCD), 1, 1);
}
inline dim3 grid_of(const int n[3]) {
    return tile_grid((n[0] + BX - 1) / BX, (n[1] + BY - 1) / BY, n[2]);
}
inline long nblocks_of(const int n[3]) { return (long)grid_of(n).x; }
// grid of the z-chunked stage kernels (kz planes per block)
inline dim3 zchunk_grid(const int n[3], int kz) {
    return tile_grid((n[0] + BX - 1) / BX, (n[1] + BY - 1) / BY, (n[2] + kz - 1) / kz);
}
extern int g_xcd_tiles;   // XCD slab tiling of the block grids (TPF_XCD_TILES=0 disables)
inline Dims dims_of(const int n[3], int walls = 0) { return Dims{n[0], n[1], n[2], g_xcd_tiles, walls}; }
Phys phys_of(const tpf_ctx* c);

}  // namespace tpf
