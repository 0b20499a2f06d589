// Host runtime behind the C ABI of include/tpf.h: parameter validation,
// workspace carving, the RK4 driver with a projection at every stage,
// state transfer, diagnostics and per-kernel timing.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "tpf_internal.hpp"

namespace tpf {

static thread_local std::string g_err;
int g_xcd_tiles = 0;

void set_error(const std::string& msg) { g_err = msg; }

tpf_status hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return TPF_EDEVICE;
}

Phys phys_of_params(const tpf_params& in) {
    Phys P;
    P.model = in.model;
    P.force = in.force;
    P.clamp = in.clamp_properties;
    P.h = in.length / in.n[0];
    P.inv_h = 1.0 / P.h;
    P.sigma = in.sigma;
    P.sigma_hat = 6.0 * in.sigma;
    P.eps = in.eps;
    P.gamma = in.gamma;
    P.rho1 = in.rho1;
    P.rho2 = in.rho2;
    P.visc1 = in.visc1;
    P.visc2 = in.visc2;
    P.delta2 = in.normal_delta * in.normal_delta;
    return P;
}

Phys phys_of(const tpf_ctx* c) { return phys_of_params(c->P); }

// ---------------------------------------------------------------- profiling
static const char* kProfNames[NPROF] = {
    "stage_cell", "stage_kappa", "stage_face", "stage_phase", "stage_phase_momentum", "stage_div",
    "stage_project", "fine_apply", "fine_update_sweep1", "fine_sweep1", "fine_sweep2",
    "fine_restrict", "fine_prolong", "fine_sweep4_dot", "mg_coarse_levels",
    "residual", "reduce_finalize", "vector", "imp_normals", "imp_residual", "imp_dn", "imp_apply",
    "imp_vector", "imp_finalize"};

static void prof_flush(tpf_ctx* c) {
    if (c->ev_count == 0) return;
    (void)hipStreamSynchronize(c->stream);
    for (int q = 0; q < c->ev_count; ++q) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, c->ev_a[q], c->ev_b[q]);
        c->prof_ms[c->ev_class[q]] += ms;
        c->prof_launches[c->ev_class[q]] += 1;
        c->prof_bytes[c->ev_class[q]] += c->ev_bytes[q];
    }
    c->ev_count = 0;
}

void prof_begin(tpf_ctx* c, int cls, double bytes) {
    c->ev_open = 0;
    if (!(c->prof_mask & (1u << cls))) return;
    c->prof_issued[cls] += 1;
    c->prof_issued_bytes[cls] += bytes;
    if (c->ev_count == c->ev_cap) prof_flush(c);
    const int q = c->ev_count;
    c->ev_class[q] = cls;
    c->ev_bytes[q] = bytes;
    (void)hipEventRecord(c->ev_a[q], c->stream);
    c->ev_open = 1;
}

void prof_end(tpf_ctx* c) {
    if (!c->ev_open) return;
    (void)hipEventRecord(c->ev_b[c->ev_count], c->stream);
    c->ev_count += 1;
    c->ev_open = 0;
}

static void prof_free(tpf_ctx* c) {
    for (int q = 0; q < c->ev_cap; ++q) {
        (void)hipEventDestroy(c->ev_a[q]);
        (void)hipEventDestroy(c->ev_b[q]);
    }
    delete[] c->ev_a;
    delete[] c->ev_b;
    delete[] c->ev_class;
    delete[] c->ev_bytes;
    c->ev_cap = 0;
}

static bool prof_alloc(tpf_ctx* c, int cap) {
    c->ev_a = new (std::nothrow) hipEvent_t[cap];
    c->ev_b = new (std::nothrow) hipEvent_t[cap];
    c->ev_class = new (std::nothrow) int[cap];
    c->ev_bytes = new (std::nothrow) double[cap];
    if (!c->ev_a || !c->ev_b || !c->ev_class || !c->ev_bytes) return false;
    // timing-only events: no system-scope fence (no cache writeback and
    // invalidation around each timed launch), so the timed kernels run as
    // they would without them
    for (int q = 0; q < cap; ++q) {
        if (hipEventCreateWithFlags(&c->ev_a[q], hipEventDisableSystemFence) != hipSuccess) return false;
        if (hipEventCreateWithFlags(&c->ev_b[q], hipEventDisableSystemFence) != hipSuccess) return false;
        c->ev_cap = q + 1;
    }
    return true;
}

// ---------------------------------------------------------------- workspace
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Carver {
    char* base;
    size_t off = 0;
    void* take(size_t bytes) {
        void* p = base ? base + off : nullptr;
        off = align256(off + bytes);
        return p;
    }
};

static int plan_levels(tpf_ctx* c) {
    int n[3] = {c->n[0], c->n[1], c->n[2]};
    int L = 1;
    const int maxl = c->P.mg_levels > 0 ? c->P.mg_levels : MAX_LEVELS;
    c->lv[0].n[0] = n[0];
    c->lv[0].n[1] = n[1];
    c->lv[0].n[2] = n[2];
    c->lv[0].h = c->h;
    while (L < maxl && L < MAX_LEVELS) {
        bool ok = true;
        for (int a = 0; a < c->dim; ++a)
            if (n[a] % 2 != 0 || n[a] < 8) ok = false;
        if (!ok) break;
        for (int a = 0; a < c->dim; ++a) n[a] /= 2;
        Level& Lv = c->lv[L];
        Lv.n[0] = n[0];
        Lv.n[1] = n[1];
        Lv.n[2] = c->dim == 3 ? n[2] : 1;
        Lv.h = c->lv[L - 1].h * 2.0;
        ++L;
    }
    for (int l = 0; l < L; ++l) c->lv[l].N = (long)c->lv[l].n[0] * c->lv[l].n[1] * c->lv[l].n[2];
    return L;
}

static size_t carve(tpf_ctx* c, char* base) {
    Carver cv{base};
    const size_t NT = (size_t)c->N * c->tsz;
    const size_t N8 = (size_t)c->N * 8;
    const size_t ssz = c->mixed ? 4 : 8;
    for (int s = 0; s < 4; ++s) {
        c->phi[s] = cv.take(NT);
        for (int a = 0; a < 3; ++a) c->u[a][s] = a < c->dim ? cv.take(NT) : nullptr;
    }
    for (int a = 0; a < 3; ++a) {
        const bool on = a < c->dim;
        c->nrm[a] = on ? cv.take(NT) : nullptr;
        c->rflux[a] = on ? cv.take(NT) : nullptr;
        c->mflux[a] = on ? cv.take(NT) : nullptr;
        c->fs[a] = on ? cv.take(NT) : nullptr;
        c->force[a] = on ? cv.take(NT) : nullptr;
    }
    c->mu = cv.take(NT);
    c->kappa = cv.take(NT);
    c->b = (double*)cv.take(N8);
    c->p = (double*)cv.take(N8);
    c->p_hist1 = (double*)cv.take(N8);
    c->p_hist2 = (double*)cv.take(N8);
    c->p_hist3 = (double*)cv.take(N8);
    c->p_alt = (double*)cv.take(N8);
    c->pv = cv.take((size_t)c->N * ssz);
    c->pv2 = cv.take((size_t)c->N * ssz);
    c->qv = cv.take((size_t)c->N * ssz);
    c->ev = c->mixed ? cv.take((size_t)c->N * ssz) : nullptr;
    c->rhoh = cv.take((size_t)c->N * ssz);
    for (int l = 0; l < c->nlev; ++l) {
        Level& L = c->lv[l];
        for (int a = 0; a < 3; ++a) L.beta[a] = a < c->dim ? cv.take((size_t)L.N * ssz) : nullptr;
        L.z = cv.take((size_t)L.N * ssz);
        L.zt = cv.take((size_t)L.N * ssz);
        L.r = cv.take((size_t)L.N * ssz);
        L.dinv = l > 0 ? cv.take((size_t)L.N * ssz) : nullptr;
    }
    c->max_blocks = std::max(nblocks_of(c->n), (long)((c->N + BLOCK - 1) / BLOCK));
    c->partials = (double*)cv.take((size_t)c->max_blocks * 3 * 8);
    c->diag_part = (double*)cv.take((size_t)nblocks_of(c->n) * 11 * 8);
    c->diag_out = (double*)cv.take(16 * 8);
    c->scal = (SolverScalars*)cv.take(sizeof(SolverScalars));
    c->flags = (int*)cv.take(64);
    c->imp_scal = cv.take(256);
    if (c->P.adjoint) {
        c->adj_stride = (long)(align256((size_t)c->N * 8) / 8);
        c->adj = (double*)cv.take((size_t)adj_fields(c->dim) * c->adj_stride * 8 + 256);
    } else {
        c->adj = nullptr;
        c->adj_stride = 0;
    }
    return cv.off;
}

tpf_status resolve_params(const tpf_params* in, tpf_params* P) {
    if (!in) { set_error("params is NULL"); return TPF_EINVAL; }
    *P = *in;
    if (P->dim != 2 && P->dim != 3) { set_error("dim must be 2 or 3"); return TPF_EINVAL; }
    if (P->dim == 2) P->n[2] = 1;
    for (int a = 0; a < P->dim; ++a)
        if (P->n[a] < 2) { set_error("each n[a] must be >= 2"); return TPF_EINVAL; }
    // kernels address fields with 32-bit byte offsets: FP64 fields must stay below 4 GiB
    const long long ncell = (long long)P->n[0] * P->n[1] * P->n[2];
    if (ncell > (1LL << 29)) {
        set_error("grid too large: at most 2^29 cells per case");
        return TPF_EINVAL;
    }
    if (P->length <= 0) P->length = 1.0;
    if (P->model < 0 || P->model > 2) { set_error("unknown model"); return TPF_EINVAL; }
    if (P->force < 0 || P->force > 2) { set_error("unknown force"); return TPF_EINVAL; }
    if (P->precision < 0 || P->precision > 1) { set_error("unknown precision"); return TPF_EINVAL; }
    if (!(P->eps > 0) || !(P->rho1 > 0) || !(P->rho2 > 0) || !(P->sigma >= 0) || !(P->gamma >= 0) ||
        !(P->visc1 >= 0) || !(P->visc2 >= 0)) {
        set_error("eps, rho1, rho2 must be > 0; sigma, gamma, visc1, visc2 >= 0");
        return TPF_EINVAL;
    }
    if (P->normal_delta <= 0) P->normal_delta = 1e-12;
    if (P->poisson_rtol <= 0) P->poisson_rtol = P->precision == TPF_FP64 ? 1e-13 : 1e-9;
    if (P->poisson_rtol_inner <= 0) P->poisson_rtol_inner = 1e-6;
    if (P->poisson_maxit <= 0) P->poisson_maxit = 400;
    if (P->mg_levels < 0) { set_error("mg_levels must be >= 0"); return TPF_EINVAL; }
    if (P->adjoint != 0 && P->adjoint != 1) { set_error("adjoint must be 0 or 1"); return TPF_EINVAL; }
    if (P->walls < 0 || P->walls >= (1 << P->dim)) {
        set_error("walls: one bit per axis of the grid (bit 0 = x)");
        return TPF_EINVAL;
    }
    return TPF_OK;
}

// Single-case contexts: the adjoint scratch is for periodic boxes only (the
// hand-written transpose has no wall rules).
static tpf_status single_case_params(const tpf_params* in, tpf_params* P) {
    tpf_status st = resolve_params(in, P);
    if (st != TPF_OK) return st;
    if (P->walls != 0 && P->adjoint) {
        set_error("the adjoint calls need a periodic box (params.walls = 0)");
        return TPF_EINVAL;
    }
    return TPF_OK;
}

int xcd_tiles_from_env() {
    const char* xt = std::getenv("TPF_XCD_TILES");
    return (xt && xt[0] == '0') ? 0 : 1;
}

static void init_geometry(tpf_ctx* c, const tpf_params* P) {
    c->P = *P;
    c->dim = P->dim;
    c->n[0] = P->n[0];
    c->n[1] = P->n[1];
    c->n[2] = P->dim == 3 ? P->n[2] : 1;
    c->N = (long)c->n[0] * c->n[1] * c->n[2];
    c->h = P->length / P->n[0];
    c->mixed = P->precision == TPF_FP32_MIXED;
    c->tsz = c->mixed ? 4 : 8;
    const char* m = std::getenv("TPF_MARCH");
    c->march = (m && m[0] == '0') ? 0 : 1;
    const char* tl = std::getenv("TPF_TAIL");
    c->no_tail = (tl && tl[0] == '0') ? 1 : 0;
    const char* mga = std::getenv("TPF_MG_ALPHA");
    c->mg_alpha = mga ? std::atof(mga) : 1.0;
    if (!(c->mg_alpha > 0.0 && c->mg_alpha < 2.0)) c->mg_alpha = 1.0;
    const char* cs = std::getenv("TPF_COARSE_SWEEPS");
    c->coarse_sweeps_per_cell = cs ? std::max(0, std::atoi(cs)) : 0;
    const char* kzs = std::getenv("TPF_KZ");
    c->kz_override = kzs ? std::atoi(kzs) : 0;
    const char* skz = std::getenv("TPF_STAGE_KZ");
    c->stage_kz = skz ? std::atoi(skz) : (c->dim == 3 ? 8 : 1);
    c->stage_kz = std::min(std::max(c->stage_kz, 1), 64);
    // fixed-iteration measurement mode "outer,inner" (0: off)
    const char* fx = std::getenv("TPF_FIXED_PCG");
    c->fixed_outer = c->fixed_inner = 0;
    if (fx && std::sscanf(fx, "%d,%d", &c->fixed_outer, &c->fixed_inner) != 2) c->fixed_outer = c->fixed_inner = 0;
    if (c->fixed_outer < 1 || c->fixed_inner < 1) c->fixed_outer = c->fixed_inner = 0;
    // LDS-staged phase/momentum pass: on by default for FP32 state (its FP64
    // form needs 104 KB of LDS and runs one block per CU); TPF_STAGE_LDS=0|1
    // overrides
    const char* sl = std::getenv("TPF_STAGE_LDS");
    c->stage_lds = sl ? (sl[0] == '1' ? 1 : 0) : (P->precision == TPF_FP32_MIXED ? 1 : 0);
    // free-slip walls: the global-memory stage kernels (their accessors apply
    // the wall rules; the LDS tiles are filled periodically)
    c->walls = P->walls;
    if (c->walls) c->stage_lds = 0;
    const char* pg = std::getenv("TPF_PCG_GRAPH");
    c->pcg_graph = (pg && pg[0] == '1') ? 1 : 0;
    const char* slk = std::getenv("TPF_STAGE_LDS_KZ");
    c->stage_lds_kz = slk ? std::atoi(slk) : 32;
    c->stage_lds_kz = std::min(std::max(c->stage_lds_kz, 1), 256);
    // fused coarse levels of the 3D V-cycle: on by default for FP32 solver
    // levels (the FP64 tiles need 88 KB of LDS, one block per CU);
    // TPF_COARSE_FUSED=0|1 overrides
    const char* cfz = std::getenv("TPF_COARSE_FUSED");
    c->coarse_fused = cfz ? (cfz[0] == '1' ? 1 : 0) : (P->precision == TPF_FP32_MIXED ? 1 : 0);
    g_xcd_tiles = xcd_tiles_from_env();
    c->nlev = plan_levels(c);
}

}  // namespace tpf

using namespace tpf;

// ================================================================== C ABI
extern "C" {

const char* tpf_last_error(void) { return g_err.c_str(); }
const char* tpf_version(void) { return "tpf 0.1 gfx950"; }
int32_t tpf_profile_classes(void) { return NPROF; }

tpf_status tpf_workspace_bytes(const tpf_params* params, size_t* bytes) {
    if (!bytes) { set_error("bytes is NULL"); return TPF_EINVAL; }
    tpf_params P;
    tpf_status st = single_case_params(params, &P);
    if (st != TPF_OK) return st;
    tpf_ctx tmp;
    std::memset(&tmp, 0, sizeof(tmp));
    init_geometry(&tmp, &P);
    *bytes = carve(&tmp, nullptr);
    return TPF_OK;
}

tpf_status tpf_create(const tpf_params* params, void* workspace, size_t ws_bytes, void* hip_stream,
                      tpf_ctx** out) {
    if (!out) { set_error("out is NULL"); return TPF_EINVAL; }
    *out = nullptr;
    tpf_params P;
    tpf_status st = single_case_params(params, &P);
    if (st != TPF_OK) return st;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255)) {
        set_error("workspace must be a non-NULL 256-byte aligned device pointer");
        return TPF_EINVAL;
    }
    tpf_ctx* c = new (std::nothrow) tpf_ctx;
    if (!c) { set_error("host allocation failed"); return TPF_ENOMEM; }
    std::memset(c, 0, sizeof(*c));
    init_geometry(c, &P);
    const size_t need = carve(c, nullptr);
    if (ws_bytes < need) {
        delete c;
        set_error("workspace too small: need " + std::to_string(need) + " bytes");
        return TPF_ENOMEM;
    }
    c->ws = static_cast<char*>(workspace);
    c->ws_bytes = ws_bytes;
    carve(c, c->ws);
    c->stream = static_cast<hipStream_t>(hip_stream);
    (void)hipGetDevice(&c->device);
    c->s_yn = 0;
    c->s_acc = 1;
    c->s_y1 = 2;
    c->s_y2 = 3;
    hipError_t e = hipMemsetAsync(c->ws, 0, need, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        tpf_status s = hip_fail(e, "workspace clear");
        delete c;
        return s;
    }
    // pinned, fine-grained host buffer for the solver scalars (the host then
    // polls it instead of copying and synchronising the stream);
    // TPF_HOST_POLL=0, or a failed allocation, keeps the copy
    c->pub = c->pub_dev = nullptr;
    c->pub_token = 0;
    const char* hp = std::getenv("TPF_HOST_POLL");
    if (!(hp && hp[0] == '0')) {
        void* hbuf = nullptr;
        if (hipHostMalloc(&hbuf, sizeof(PubScalars), hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess) {
            void* dbuf = nullptr;
            if (hipHostGetDevicePointer(&dbuf, hbuf, 0) == hipSuccess) {
                std::memset(hbuf, 0, sizeof(PubScalars));
                c->pub = static_cast<PubScalars*>(hbuf);
                c->pub_dev = static_cast<PubScalars*>(dbuf);
            } else {
                (void)hipHostFree(hbuf);
            }
        }
        (void)hipGetLastError();
    }
    *out = c;
    return TPF_OK;
}

tpf_status tpf_destroy(tpf_ctx* c) {
    if (!c) return TPF_OK;
    (void)hipStreamSynchronize(c->stream);
    prof_free(c);
    if (c->pub) (void)hipHostFree(c->pub);
    for (int g = 0; g < c->n_pcg_graphs; ++g) (void)hipGraphExecDestroy(c->pcg_graphs[g].exec);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return TPF_OK;
}

static tpf_status finish_set_state(tpf_ctx* c) {
    hipError_t e = hipMemsetAsync(c->p, 0, (size_t)c->N * 8, c->stream);
    if (e != hipSuccess) return hip_fail(e, "pressure reset");
    c->t = 0.0;
    c->step = 0;
    c->p_valid = 0;
    c->hist2_valid = 0;
    const void* u[3] = {c->u[0][c->s_yn], c->u[1][c->s_yn], c->dim == 3 ? c->u[2][c->s_yn] : c->u[1][c->s_yn]};
    e = launch_diagnostics(c, c->phi[c->s_yn], u, nullptr);
    if (e != hipSuccess) return hip_fail(e, "diagnostics");
    double out[11];
    e = hipMemcpyAsync(out, c->diag_out, sizeof(out), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "diagnostics readback");
    c->mass0 = out[0] * std::pow(c->h, c->dim);
    return TPF_OK;
}

tpf_status tpf_set_state(tpf_ctx* c, const double* phi, const double* u0, const double* u1,
                         const double* u2, int32_t on_device) {
    if (!c || !phi || !u0 || !u1 || (c->dim == 3 && !u2)) {
        set_error("tpf_set_state: NULL argument");
        return TPF_EINVAL;
    }
    const double* src[4] = {phi, u0, u1, u2};
    void* dst[4] = {c->phi[c->s_yn], c->u[0][c->s_yn], c->u[1][c->s_yn], c->u[2][c->s_yn]};
    for (int v = 0; v <= c->dim; ++v) {
        const double* s = src[v];
        hipError_t e;
        if (!on_device) {
            e = hipMemcpyAsync(c->b, s, (size_t)c->N * 8, hipMemcpyHostToDevice, c->stream);
            if (e != hipSuccess) return hip_fail(e, "host to device copy");
            s = c->b;
        }
        e = launch_convert_in(c, s, dst[v]);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(e, "state conversion");
    }
    return finish_set_state(c);
}

tpf_status tpf_field_offset(const tpf_ctx* c, int32_t field, size_t* byte_offset, int32_t* dtype) {
    if (!c || !byte_offset || !dtype) { set_error("tpf_field_offset: NULL argument"); return TPF_EINVAL; }
    const void* ptr = nullptr;
    int32_t ty = c->mixed ? TPF_DTYPE_F32 : TPF_DTYPE_F64;
    if (field == TPF_STATE_PHI) {
        ptr = c->phi[c->s_yn];
    } else if (field >= TPF_STATE_U0 && field <= TPF_STATE_U2) {
        const int a = field - TPF_STATE_U0;
        if (a >= c->dim) { set_error("velocity component beyond dim"); return TPF_EINVAL; }
        ptr = c->u[a][c->s_yn];
    } else if (field == TPF_STATE_P) {
        ptr = c->p;
        ty = TPF_DTYPE_F64;
    } else {
        set_error("unknown state field");
        return TPF_EINVAL;
    }
    *byte_offset = (size_t)(static_cast<const char*>(ptr) - c->ws);
    *dtype = ty;
    return TPF_OK;
}

tpf_status tpf_state_changed(tpf_ctx* c) {
    if (!c) { set_error("ctx is NULL"); return TPF_EINVAL; }
    return finish_set_state(c);
}

tpf_status tpf_init_droplet(tpf_ctx* c, const double center[3], const double semi_axes[3]) {
    if (!c || !center || !semi_axes) { set_error("tpf_init_droplet: NULL argument"); return TPF_EINVAL; }
    for (int a = 0; a < c->dim; ++a)
        if (!(semi_axes[a] > 0)) { set_error("semi axes must be > 0"); return TPF_EINVAL; }
    double cen[3] = {center[0], center[1], c->dim == 3 ? center[2] : 0.0};
    double ax[3] = {semi_axes[0], semi_axes[1], c->dim == 3 ? semi_axes[2] : 1.0};
    hipError_t e = launch_init_droplet(c, cen, ax);
    for (int a = 0; a < c->dim && e == hipSuccess; ++a) e = launch_zero_state(c, c->u[a][c->s_yn]);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "droplet initialisation");
    return finish_set_state(c);
}

// One stage evaluation at (phi_s, u_s): fields, phase RHS (+RK update),
// momentum RHS, pressure solve, projection (+RK update).
static tpf_status stage_eval(tpf_ctx* c, const void* phi_s, const void* const u_s[3], const RKArgs& rk,
                             void* phi_out, void* const u_out[3], int want_force, bool normals) {
    hipError_t e = launch_stage_fields(c, phi_s, u_s, normals);
    if (e == hipSuccess) e = launch_phase_momentum(c, phi_s, u_s, rk, phi_out, want_force);
    if (e == hipSuccess) e = launch_divergence(c);
    if (e != hipSuccess) return hip_fail(e, "stage kernels");
    int it = 0, outer = 0;
    double rr = 0;
    tpf_status st = poisson_solve(c, phi_s, &it, &rr, &outer);
    c->last_inner = it;
    c->last_outer = outer;
    c->last_relres = rr;
    c->stat_recent[c->stat_solves % 4] = it;
    c->stat_solves += 1;
    c->stat_outer += outer;
    c->stat_inner += it;
    if (st != TPF_OK) return st;
    e = launch_project_update(c, phi_s, rk, u_out);
    if (e != hipSuccess) return hip_fail(e, "projection");
    return TPF_OK;
}

static void state_ptrs(tpf_ctx* c, int slot, void** phi, void* u[3]) {
    *phi = c->phi[slot];
    for (int a = 0; a < 3; ++a) u[a] = c->u[a][slot] ? c->u[a][slot] : c->u[0][slot];
}

}  // extern "C"

namespace tpf {

static tpf_status copy_async(tpf_ctx* c, void* dst, const void* src, size_t bytes) {
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream);
    return e == hipSuccess ? TPF_OK : hip_fail(e, "device copy");
}

tpf_status advance(tpf_ctx* c, double dt, int nsteps, char* tape, size_t stage_bytes) {
    const double wacc[4] = {dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0};
    const double wnext[4] = {dt / 2.0, dt / 2.0, dt, 0.0};
    const size_t NT = (size_t)c->N * c->tsz;
    const size_t fT = align256(NT);
    for (int n = 0; n < nsteps; ++n) {
        hipError_t e = hipMemsetAsync(c->flags, 0, 64, c->stream);
        if (e != hipSuccess) return hip_fail(e, "flag reset");
        // stage inputs: yn, y1, y2, y1 ; stage outputs: y1, y2, y1, (acc)
        const int in_slot[4] = {c->s_yn, c->s_y1, c->s_y2, c->s_y1};
        const int out_slot[4] = {c->s_y1, c->s_y2, c->s_y1, c->s_acc};
        for (int s = 0; s < 4; ++s) {
            void *phi_s, *phi_o;
            void *u_s[3], *u_o[3];
            state_ptrs(c, in_slot[s], &phi_s, u_s);
            state_ptrs(c, out_slot[s], &phi_o, u_o);
            char* rec = tape ? tape + ((size_t)n * 4 + s) * stage_bytes : nullptr;
            if (rec) {
                tpf_status st = copy_async(c, rec, phi_s, NT);
                for (int a = 0; a < c->dim && st == TPF_OK; ++a)
                    st = copy_async(c, rec + (1 + a) * fT, u_s[a], NT);
                if (st != TPF_OK) return st;
            }
            RKArgs rk{s, 0, wacc[s], wnext[s]};
            const void* us[3] = {u_s[0], u_s[1], u_s[2]};
            c->rk_stage = s;
            // the projection of stages 1-3 keeps the history: p_hist1 = p(t),
            // p_hist2 = p(t + dt/2) of stage 2, p_hist3 = stage 3 minus stage 2
            double* const hist[4] = {c->p_hist1, c->p_hist2, c->p_hist3, nullptr};
            c->proj_hist = hist[s];
            c->proj_hsub = s == 2 ? c->p_hist2 : nullptr;
            // and writes the starting guess of the next stage's pressure solve
            // (stage 1, at time t, starts from the last pressure, stage 4 of
            // the previous step): stage 2 (t + dt/2) extrapolates linearly
            // from t - dt/2 and t, 2 p(t) - p_hist2 of the previous step;
            // stage 3 (t + dt/2 again) adds to the stage-2 pressure the
            // stage-3 minus stage-2 difference of the previous step, p_hist3;
            // stage 4 (t + dt) extrapolates from t and t + dt/2, 2 p - p_hist1
            const bool guess = (s < 2 && c->hist2_valid) || s == 2;
            c->proj_guess = guess ? 1 : 0;
            c->proj_gsrc = s == 0 ? c->p_hist2 : s == 1 ? c->p_hist3 : c->p_hist1;
            c->proj_ga = s == 1 ? 1.0 : 2.0;
            c->proj_gb = s == 1 ? 1.0 : -1.0;
            tpf_status st = stage_eval(c, phi_s, us, rk, phi_o, u_o, 0, false);
            c->rk_stage = 0;
            c->proj_hist = nullptr;
            c->proj_hsub = nullptr;
            c->proj_guess = 0;
            c->proj_gsrc = nullptr;
            if (st == TPF_OK && rec) st = copy_async(c, rec + (1 + c->dim) * fT, c->p, (size_t)c->N * 8);
            if (st != TPF_OK) {
                c->p_valid = 0;
                c->hist2_valid = 0;
                return st;
            }
            if (guess) std::swap(c->p, c->p_alt);
        }
        int flag = 0;
        e = fetch_flag(c, &flag);
        if (e != hipSuccess) return hip_fail(e, "step completion");
        if (flag) {
            c->p_valid = 0;
            c->hist2_valid = 0;
            set_error("non-finite value produced; state kept at the last completed step");
            return TPF_ENONFINITE;
        }
        c->hist2_valid = 1;
        const int t = c->s_yn;
        c->s_yn = c->s_acc;
        c->s_acc = t;
        c->t += dt;
        c->step += 1;
        c->p_valid = 0;
    }
    return TPF_OK;
}

}  // namespace tpf

extern "C" {

tpf_status tpf_step(tpf_ctx* c, double dt, int32_t nsteps) {
    if (!c) { set_error("ctx is NULL"); return TPF_EINVAL; }
    if (!(dt > 0) || nsteps < 0) { set_error("dt must be > 0 and nsteps >= 0"); return TPF_EINVAL; }
    return advance(c, dt, nsteps, nullptr, 0);
}

}  // extern "C"

// Evaluate one stage at the current state without updating it; the
// derivatives go to the y1 slot and the pressure to c->p.
tpf_status tpf::eval_current(tpf_ctx* c, int want_force) {
    void *phi_s, *phi_o;
    void *u_s[3], *u_o[3];
    state_ptrs(c, c->s_yn, &phi_s, u_s);
    state_ptrs(c, c->s_y1, &phi_o, u_o);
    RKArgs rk{0, 1, 0.0, 0.0};
    const void* us[3] = {u_s[0], u_s[1], u_s[2]};
    tpf_status st = stage_eval(c, phi_s, us, rk, phi_o, u_o, want_force, true);
    if (st == TPF_OK) st = gauge_pressure(c);
    if (st == TPF_OK) c->p_valid = 1;
    return st;
}

extern "C" {

static tpf_status copy_out(tpf_ctx* c, const void* src, int is_double, double* dst, int on_device) {
    hipError_t e;
    if (is_double) {
        e = hipMemcpyAsync(dst, src, (size_t)c->N * 8,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream);
    } else {
        double* tgt = on_device ? dst : c->b;
        e = launch_convert_out(c, src, tgt);
        if (e == hipSuccess && !on_device)
            e = hipMemcpyAsync(dst, c->b, (size_t)c->N * 8, hipMemcpyDeviceToHost, c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "copy out");
    return TPF_OK;
}

tpf_status tpf_get_state(tpf_ctx* c, double* phi, double* u0, double* u1, double* u2, double* p,
                         int32_t on_device) {
    if (!c) { set_error("ctx is NULL"); return TPF_EINVAL; }
    if (p && !c->p_valid) {
        tpf_status st = eval_current(c, 0);
        if (st != TPF_OK) return st;
    }
    double* dst[4] = {phi, u0, u1, c->dim == 3 ? u2 : nullptr};
    const void* src[4] = {c->phi[c->s_yn], c->u[0][c->s_yn], c->u[1][c->s_yn], c->u[2][c->s_yn]};
    for (int v = 0; v < 4; ++v) {
        if (!dst[v]) continue;
        tpf_status st = copy_out(c, src[v], 0, dst[v], on_device);
        if (st != TPF_OK) return st;
    }
    if (p) return copy_out(c, c->p, 1, p, on_device);
    return TPF_OK;
}

tpf_status tpf_diagnostics(tpf_ctx* c, tpf_diag* out) {
    if (!c || !out) { set_error("NULL argument"); return TPF_EINVAL; }
    if (!c->p_valid) {
        tpf_status st = eval_current(c, 0);
        if (st != TPF_OK) return st;
    }
    const void* u[3] = {c->u[0][c->s_yn], c->u[1][c->s_yn], c->dim == 3 ? c->u[2][c->s_yn] : c->u[1][c->s_yn]};
    hipError_t e = launch_diagnostics(c, c->phi[c->s_yn], u, c->p);
    double v[11];
    if (e == hipSuccess) e = hipMemcpyAsync(v, c->diag_out, sizeof(v), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "diagnostics");
    const double hd = std::pow(c->h, c->dim);
    out->t = c->t;
    out->step = c->step;
    out->mass = hd * v[0];
    out->mass0 = c->mass0;
    out->ke = hd * v[1];
    out->se = hd * v[2];
    out->dp = (v[4] > 0 && v[6] > 0) ? v[3] / v[4] - v[5] / v[6] : NAN;
    out->umax = v[7];
    out->ca_inf = c->P.sigma > 0 ? v[7] * c->P.visc1 / c->P.sigma : NAN;
    out->div_max = v[8];
    out->phi_min = -v[9];
    out->phi_max = v[10];
    out->poisson_relres = c->last_relres;
    out->poisson_outer = c->last_outer;
    out->poisson_inner = c->last_inner;
    return TPF_OK;
}

tpf_status tpf_eval_field(tpf_ctx* c, int32_t field, double* out, int32_t on_device) {
    if (!c || !out) { set_error("NULL argument"); return TPF_EINVAL; }
    if (field < 0 || field >= TPF_FIELD_COUNT) { set_error("unknown field"); return TPF_EINVAL; }
    auto comp = [&](int base) { return field - base; };
    int a = 0;
    if ((field >= TPF_FIELD_NORMAL0 && field <= TPF_FIELD_NORMAL2) ||
        (field >= TPF_FIELD_CDIFLUX0 && field <= TPF_FIELD_CDIFLUX2) ||
        (field >= TPF_FIELD_MASSFLUX0 && field <= TPF_FIELD_MASSFLUX2) ||
        (field >= TPF_FIELD_FORCE0 && field <= TPF_FIELD_FORCE2) ||
        (field >= TPF_FIELD_FSTAR0 && field <= TPF_FIELD_FSTAR2) ||
        (field >= TPF_FIELD_DU0 && field <= TPF_FIELD_DU2)) {
        if (field <= TPF_FIELD_NORMAL2) a = comp(TPF_FIELD_NORMAL0);
        else if (field <= TPF_FIELD_CDIFLUX2) a = comp(TPF_FIELD_CDIFLUX0);
        else if (field <= TPF_FIELD_MASSFLUX2) a = comp(TPF_FIELD_MASSFLUX0);
        else if (field <= TPF_FIELD_FORCE2) a = comp(TPF_FIELD_FORCE0);
        else if (field <= TPF_FIELD_FSTAR2) a = comp(TPF_FIELD_FSTAR0);
        else a = comp(TPF_FIELD_DU0);
        if (a >= c->dim) { set_error("component not present in this dimension"); return TPF_EINVAL; }
    }
    if (field == TPF_FIELD_KAPPA && c->P.model == TPF_CDI && c->P.force == TPF_EB) {
        set_error("kappa is not computed for CDI with the energy-based force");
        return TPF_EINVAL;
    }
    if (field == TPF_FIELD_MU && c->P.force != TPF_EB) {
        set_error("mu is only computed with the energy-based force");
        return TPF_EINVAL;
    }
    if (field >= TPF_FIELD_CDIFLUX0 && field <= TPF_FIELD_CDIFLUX2 && c->P.model != TPF_CDI) {
        set_error("CDI flux only exists for the CDI model");
        return TPF_EINVAL;
    }
    tpf_status st = eval_current(c, 1);
    if (st != TPF_OK) return st;
    const void* src = nullptr;
    int dbl = 0;
    switch (field) {
    case TPF_FIELD_NORMAL0: case TPF_FIELD_NORMAL1: case TPF_FIELD_NORMAL2: src = c->nrm[a]; break;
    case TPF_FIELD_MU: src = c->mu; break;
    case TPF_FIELD_KAPPA: src = c->kappa; break;
    case TPF_FIELD_CDIFLUX0: case TPF_FIELD_CDIFLUX1: case TPF_FIELD_CDIFLUX2: src = c->rflux[a]; break;
    case TPF_FIELD_MASSFLUX0: case TPF_FIELD_MASSFLUX1: case TPF_FIELD_MASSFLUX2: src = c->mflux[a]; break;
    case TPF_FIELD_DPHI: src = c->phi[c->s_y1]; break;
    case TPF_FIELD_FORCE0: case TPF_FIELD_FORCE1: case TPF_FIELD_FORCE2: src = c->force[a]; break;
    case TPF_FIELD_FSTAR0: case TPF_FIELD_FSTAR1: case TPF_FIELD_FSTAR2: src = c->fs[a]; break;
    case TPF_FIELD_DIVFSTAR: src = c->b; dbl = 1; break;
    case TPF_FIELD_PRESSURE: src = c->p; dbl = 1; break;
    default: src = c->u[a][c->s_y1]; break;
    }
    return copy_out(c, src, dbl, out, on_device);
}

tpf_status tpf_poisson_solve(tpf_ctx* c, const double* b, double* x, int32_t on_device, int32_t* iters,
                             double* relres) {
    if (!c || !b || !x) { set_error("NULL argument"); return TPF_EINVAL; }
    const hipMemcpyKind kin = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    hipError_t e = hipMemcpyAsync(c->b, b, (size_t)c->N * 8, kin, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->p, x, (size_t)c->N * 8, kin, c->stream);
    if (e != hipSuccess) return hip_fail(e, "copy in");
    e = launch_rhs_mean(c);
    if (e != hipSuccess) return hip_fail(e, "rhs mean");
    int it = 0, outer = 0;
    double rr = 0;
    tpf_status st = poisson_solve(c, c->phi[c->s_yn], &it, &rr, &outer);
    c->p_valid = 0;
    c->hist2_valid = 0;
    if (iters) *iters = it;
    if (relres) *relres = rr;
    if (st == TPF_OK) st = gauge_pressure(c);
    if (st != TPF_OK) return st;
    e = hipMemcpyAsync(x, c->p, (size_t)c->N * 8, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                       c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "copy out");
    return TPF_OK;
}

tpf_status tpf_solver_stats(tpf_ctx* c, int64_t out[7], int32_t reset) {
    if (!c) { set_error("ctx is NULL"); return TPF_EINVAL; }
    if (out) {
        out[0] = c->stat_solves;
        out[1] = c->stat_outer;
        out[2] = c->stat_inner;
        for (int k = 0; k < 4; ++k) {        // oldest first
            const long long q = c->stat_solves - 4 + k;
            out[3 + k] = q >= 0 ? c->stat_recent[q % 4] : -1;
        }
    }
    if (reset) c->stat_solves = c->stat_outer = c->stat_inner = 0;
    return TPF_OK;
}

tpf_status tpf_profile_enable(tpf_ctx* c, int32_t enable) {
    if (!c) { set_error("ctx is NULL"); return TPF_EINVAL; }
    prof_flush(c);
    if (enable && c->ev_cap == 0 && !prof_alloc(c, 8192)) {
        prof_free(c);
        set_error("hipEventCreate failed");
        return TPF_EDEVICE;
    }
    c->prof_mask = (unsigned)enable;
    if (enable) {
        for (int q = 0; q < NPROF; ++q) {
            c->prof_ms[q] = 0;
            c->prof_launches[q] = 0;
            c->prof_bytes[q] = 0;
            c->prof_issued[q] = 0;
            c->prof_issued_bytes[q] = 0;
            c->prof_noop[q] = 0;
            c->prof_noop_bytes[q] = 0;
        }
    }
    return TPF_OK;
}

tpf_status tpf_profile_read(tpf_ctx* c, int32_t cls, const char** name, double* total_ms,
                            int64_t* launches, double* bytes_per_launch) {
    if (!c || cls < 0 || cls >= NPROF) { set_error("bad profile class"); return TPF_EINVAL; }
    prof_flush(c);
    if (name) *name = kProfNames[cls];
    const long work = c->prof_launches[cls] - c->prof_noop[cls];
    if (total_ms) *total_ms = c->prof_ms[cls];
    if (launches) *launches = work;
    if (bytes_per_launch)
        *bytes_per_launch = work > 0 ? (c->prof_bytes[cls] - c->prof_noop_bytes[cls]) / work : 0.0;
    return TPF_OK;
}

}  // extern "C"

// ================================================================== no-allocation diagnostics
// tpf_diagnostics_noalloc keeps the block partials and the final sums of its
// reduction in this file-scope device array: no hipMalloc, no workspace.  The
// host side never uses the array's name as an address; it asks the runtime
// once per device for the array's device address (scratch_dev) and passes
// that to the kernels.
namespace tpf {
constexpr long kNoAllocBlocks = 65536;                       // 64 x 4-cell tiles
constexpr long kNoAllocValues = ND_SUM + ND_MAX;
constexpr size_t kNoAllocDoubles = (size_t)kNoAllocValues * kNoAllocBlocks + 32;
}  // namespace tpf

static __device__ __align__(256) double scratch[tpf::kNoAllocDoubles];

namespace tpf {
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_dev[kMaxDevices];

// device address of `scratch` on the current device, looked up once per device
static tpf_status scratch_dev(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index beyond the scratch table");
        return TPF_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
        g_scratch_dev[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_dev[dev];
    return TPF_OK;
}
}  // namespace tpf

extern "C" {

tpf_status tpf_diagnostics_noalloc(const tpf_params* params, const double* phi, const double* u0,
                                   const double* u1, const double* u2, const double* p, void* hip_stream,
                                   tpf_diag* out) {
    tpf_params P;
    tpf_status st = single_case_params(params, &P);
    if (st != TPF_OK) return st;
    if (!phi || !u0 || !u1 || (P.dim == 3 && !u2) || !out) {
        set_error("tpf_diagnostics_noalloc: NULL argument");
        return TPF_EINVAL;
    }
    const int n[3] = {P.n[0], P.n[1], P.dim == 3 ? P.n[2] : 1};
    const long nb = nblocks_of(n);
    if (nb > kNoAllocBlocks) {
        set_error("tpf_diagnostics_noalloc: grid needs " + std::to_string(nb) + " blocks of 64 x 4 cells, the "
                  "static scratch holds " + std::to_string(kNoAllocBlocks));
        return TPF_EINVAL;
    }
    double* sc = nullptr;
    st = scratch_dev(&sc);
    if (st != TPF_OK) return st;
    double* part = sc;
    double* fin = sc + kNoAllocValues * kNoAllocBlocks;
    g_xcd_tiles = xcd_tiles_from_env();
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const void* u[3] = {u0, u1, P.dim == 3 ? u2 : nullptr};
    // every partial the final sum reads is written by this call's first
    // kernel, so nothing in the scratch needs clearing
    hipError_t e = launch_diagnostics_arrays(stream, P.dim, n, P.walls, 0, phys_of_params(P), phi, u, p, part, fin);
    double v[kNoAllocValues];
    if (e == hipSuccess) e = hipMemcpyAsync(v, fin, sizeof(v), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "tpf_diagnostics_noalloc");
    const double hd = std::pow(P.length / P.n[0], P.dim);
    std::memset(out, 0, sizeof(*out));
    out->mass = hd * v[0];
    out->mass0 = NAN;
    out->ke = hd * v[1];
    out->se = hd * v[2];
    out->dp = (p && v[4] > 0 && v[6] > 0) ? v[3] / v[4] - v[5] / v[6] : NAN;
    out->umax = v[7];
    out->ca_inf = P.sigma > 0 ? v[7] * P.visc1 / P.sigma : NAN;
    out->div_max = v[8];
    out->phi_min = -v[9];
    out->phi_max = v[10];
    out->poisson_relres = NAN;
    return TPF_OK;
}

}  // extern "C"
