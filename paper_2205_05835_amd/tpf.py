"""ctypes binding of the C ABI in include/tpf.h (argument marshalling only).

Every computation runs in the HIP kernels of libtpf.so; this module only
converts Python arguments to the C types, raises TpfError on a non-zero
status and offers a small ``Solver`` convenience class that takes device
memory (the workspace) and the stream from PyTorch.  There is no CPU path:
if the library is missing, importing ``lib()`` raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtpf.so")

TPF_OK, TPF_EINVAL, TPF_ENOMEM, TPF_EDEVICE, TPF_ENOCONV, TPF_ENONFINITE, TPF_ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "TPF_OK", -1: "TPF_EINVAL", -2: "TPF_ENOMEM", -3: "TPF_EDEVICE", -4: "TPF_ENOCONV",
                -5: "TPF_ENONFINITE", -6: "TPF_ESTATE"}
TPF_CDI, TPF_SB, TPF_ISODI = 0, 1, 2
TPF_EB, TPF_CSF, TPF_LCSF = 0, 1, 2
TPF_FP64, TPF_FP32_MIXED = 0, 1
MODELS = {"CDI": TPF_CDI, "SB": TPF_SB, "ISODI": TPF_ISODI}
FORCES = {"EB": TPF_EB, "CSF": TPF_CSF, "LCSF": TPF_LCSF}
PRECISIONS = {"fp64": TPF_FP64, "fp32_mixed": TPF_FP32_MIXED}

FIELDS = ["NORMAL0", "NORMAL1", "NORMAL2", "MU", "KAPPA", "CDIFLUX0", "CDIFLUX1", "CDIFLUX2",
          "MASSFLUX0", "MASSFLUX1", "MASSFLUX2", "DPHI", "FORCE0", "FORCE1", "FORCE2",
          "FSTAR0", "FSTAR1", "FSTAR2", "DIVFSTAR", "PRESSURE", "DU0", "DU1", "DU2"]
FIELD = {name: q for q, name in enumerate(FIELDS)}

# every entry point the header declares (checked by the CPU test-suite)
EXPORTS = ["tpf_workspace_bytes", "tpf_create", "tpf_destroy", "tpf_set_state", "tpf_init_droplet",
           "tpf_step", "tpf_get_state", "tpf_diagnostics", "tpf_eval_field", "tpf_poisson_solve",
           "tpf_profile_enable", "tpf_profile_read", "tpf_profile_classes", "tpf_last_error",
           "tpf_version", "tpf_batch_workspace_bytes", "tpf_batch_create", "tpf_batch_destroy",
           "tpf_batch_set_state", "tpf_batch_init_droplet", "tpf_batch_get_state", "tpf_batch_step",
           "tpf_batch_status", "tpf_batch_clear_status", "tpf_batch_diagnostics", "tpf_batch_configs",
           "tpf_batch_config_info", "tpf_batch_set_config", "tpf_batch_tune", "tpf_checkpoint_bytes",
           "tpf_save_checkpoint", "tpf_load_checkpoint", "tpf_adjoint_tape_bytes", "tpf_stage_adjoint",
           "tpf_step_adjoint", "tpf_solver_stats", "tpf_implicit_phase_step", "tpf_field_offset",
           "tpf_state_changed", "tpf_diagnostics_noalloc", "tpf_batch_solver_stats"]

TPF_STATE_PHI, TPF_STATE_U0, TPF_STATE_U1, TPF_STATE_U2, TPF_STATE_P = 0, 1, 2, 3, 4
TPF_DTYPE_F64, TPF_DTYPE_F32 = 0, 1


class TpfError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class tpf_params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("length", ctypes.c_double),
                ("model", ctypes.c_int32), ("force", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("clamp_properties", ctypes.c_int32), ("sigma", ctypes.c_double),
                ("eps", ctypes.c_double), ("gamma", ctypes.c_double), ("rho1", ctypes.c_double),
                ("rho2", ctypes.c_double), ("visc1", ctypes.c_double), ("visc2", ctypes.c_double),
                ("normal_delta", ctypes.c_double), ("poisson_rtol", ctypes.c_double),
                ("poisson_rtol_inner", ctypes.c_double), ("poisson_maxit", ctypes.c_int32),
                ("mg_levels", ctypes.c_int32), ("adjoint", ctypes.c_int32), ("walls", ctypes.c_int32)]


class tpf_implicit_opts(ctypes.Structure):
    _fields_ = [("newton_tol", ctypes.c_double), ("krylov_rtol", ctypes.c_double),
                ("newton_maxit", ctypes.c_int32), ("krylov_maxit", ctypes.c_int32)]


class tpf_implicit_info(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int32), ("krylov_iters", ctypes.c_int32),
                ("residual", ctypes.c_double), ("newton_total", ctypes.c_int64),
                ("krylov_total", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class tpf_diag(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("step", ctypes.c_int64), ("mass", ctypes.c_double),
                ("mass0", ctypes.c_double), ("phi_min", ctypes.c_double), ("phi_max", ctypes.c_double),
                ("umax", ctypes.c_double), ("ca_inf", ctypes.c_double), ("ke", ctypes.c_double),
                ("se", ctypes.c_double), ("dp", ctypes.c_double), ("div_max", ctypes.c_double),
                ("poisson_relres", ctypes.c_double), ("poisson_outer", ctypes.c_int32),
                ("poisson_inner", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libtpf.so (built by paper_2205_05835_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
    try:
        import torch  # noqa: F401  -- share torch's HIP runtime instance
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, i32 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32
    P = ctypes.POINTER(tpf_params)
    sig = {
        "tpf_workspace_bytes": ([P, ctypes.POINTER(ctypes.c_size_t)], i32),
        "tpf_create": ([P, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)], i32),
        "tpf_destroy": ([vp], i32),
        "tpf_set_state": ([vp, vp, vp, vp, vp, i32], i32),
        "tpf_field_offset": ([vp, i32, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(i32)], i32),
        "tpf_state_changed": ([vp], i32),
        "tpf_diagnostics_noalloc": ([P, vp, vp, vp, vp, vp, vp, ctypes.POINTER(tpf_diag)], i32),
        "tpf_init_droplet": ([vp, dp, dp], i32),
        "tpf_step": ([vp, ctypes.c_double, i32], i32),
        "tpf_get_state": ([vp, vp, vp, vp, vp, vp, i32], i32),
        "tpf_diagnostics": ([vp, ctypes.POINTER(tpf_diag)], i32),
        "tpf_eval_field": ([vp, i32, vp, i32], i32),
        "tpf_poisson_solve": ([vp, vp, vp, i32, ctypes.POINTER(i32), dp], i32),
        "tpf_profile_enable": ([vp, i32], i32),
        "tpf_profile_read": ([vp, i32, ctypes.POINTER(ctypes.c_char_p), dp, ctypes.POINTER(ctypes.c_int64), dp], i32),
        "tpf_profile_classes": ([], i32),
        "tpf_last_error": ([], ctypes.c_char_p),
        "tpf_version": ([], ctypes.c_char_p),
        "tpf_batch_workspace_bytes": ([P, i32, ctypes.POINTER(ctypes.c_size_t)], i32),
        "tpf_batch_create": ([P, i32, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)], i32),
        "tpf_batch_destroy": ([vp], i32),
        "tpf_batch_set_state": ([vp, i32, vp, vp, vp, i32], i32),
        "tpf_batch_init_droplet": ([vp, i32, dp, dp], i32),
        "tpf_batch_get_state": ([vp, i32, vp, vp, vp, vp, i32], i32),
        "tpf_batch_step": ([vp, dp, i32], i32),
        "tpf_batch_status": ([vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_int64), dp], i32),
        "tpf_batch_clear_status": ([vp, i32], i32),
        "tpf_batch_diagnostics": ([vp, ctypes.POINTER(tpf_diag)], i32),
        "tpf_batch_configs": ([], i32),
        "tpf_batch_config_info": ([i32, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "tpf_batch_set_config": ([vp, i32], i32),
        "tpf_batch_tune": ([vp, dp, ctypes.c_char_p, ctypes.POINTER(i32)], i32),
        "tpf_batch_solver_stats": ([vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_int64), i32], i32),
        "tpf_checkpoint_bytes": ([vp, ctypes.POINTER(ctypes.c_size_t)], i32),
        "tpf_solver_stats": ([vp, ctypes.POINTER(ctypes.c_int64), i32], i32),
        "tpf_save_checkpoint": ([vp, vp], i32),
        "tpf_load_checkpoint": ([vp, vp], i32),
        "tpf_adjoint_tape_bytes": ([vp, i32, ctypes.POINTER(ctypes.c_size_t)], i32),
        "tpf_stage_adjoint": ([vp, vp, vp, vp, vp, vp, vp, vp, vp, dp, i32], i32),
        "tpf_step_adjoint": ([vp, vp, ctypes.c_size_t, ctypes.c_double, i32, vp, vp, vp, vp, i32, dp], i32),
        "tpf_implicit_phase_step": ([vp, ctypes.c_double, i32, ctypes.POINTER(tpf_implicit_opts),
                                     ctypes.POINTER(tpf_implicit_info)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(status: int, where: str) -> None:
    if status != TPF_OK:
        raise TpfError(status, where, lib().tpf_last_error().decode())


def make_params(n, length=1.0, model="CDI", force="EB", precision="fp64", clamp_properties=1,
                sigma=1.0, eps=None, gamma=1.0, rho1=1.0, rho2=1.0, visc1=0.1, visc2=0.1,
                normal_delta=1e-12, poisson_rtol=0.0, poisson_rtol_inner=0.0, poisson_maxit=0,
                mg_levels=0, adjoint=0, walls=0) -> tpf_params:
    n = tuple(int(x) for x in n)
    dim = len(n)
    h = length / n[0]
    p = tpf_params()
    p.dim = dim
    p.n = (ctypes.c_int32 * 3)(*(list(n) + [1] * (3 - dim)))
    p.length = length
    p.model = MODELS[model] if isinstance(model, str) else int(model)
    p.force = FORCES[force] if isinstance(force, str) else int(force)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.clamp_properties = clamp_properties
    p.sigma, p.eps, p.gamma = sigma, (eps if eps else h), gamma
    p.rho1, p.rho2, p.visc1, p.visc2 = rho1, rho2, visc1, visc2
    p.normal_delta = normal_delta
    p.poisson_rtol, p.poisson_rtol_inner = poisson_rtol, poisson_rtol_inner
    p.poisson_maxit, p.mg_levels = poisson_maxit, mg_levels
    p.adjoint = int(adjoint)
    p.walls = int(walls)
    return p


def workspace_bytes(params: tpf_params) -> int:
    out = ctypes.c_size_t(0)
    check(lib().tpf_workspace_bytes(ctypes.byref(params), ctypes.byref(out)), "tpf_workspace_bytes")
    return int(out.value)


def _host(a, N):
    a = np.ascontiguousarray(a, dtype=np.float64).ravel()
    if a.size != N:
        raise ValueError(f"array has {a.size} values, expected {N}")
    return a


class Solver:
    """One case on the current GPU: workspace and stream from PyTorch."""

    def __init__(self, params: tpf_params, stream=None, device=None):
        import torch
        self.torch = torch
        self.params = params
        self.dim = params.dim
        self.n = tuple(params.n[a] for a in range(self.dim))
        self.shape = tuple(reversed(self.n))
        self.N = int(np.prod(self.n))
        self.device = torch.device(device or "cuda")
        nbytes = workspace_bytes(params)
        # 256-byte alignment: torch's caching allocator returns 512-byte aligned blocks
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        check(lib().tpf_create(ctypes.byref(params), ctypes.c_void_p(self.workspace.data_ptr()),
                               nbytes, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)),
              "tpf_create")
        self.ctx = ctx

    def close(self):
        if self.ctx:
            check(lib().tpf_destroy(self.ctx), "tpf_destroy")
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- state
    def set_state(self, phi, u):
        """phi: array of N values; u: list of dim face arrays (host numpy or
        CUDA float64 tensors)."""
        torch = self.torch
        if isinstance(phi, torch.Tensor):
            arrs = [phi] + list(u)
            for t in arrs:
                if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                    raise ValueError("device arrays must be contiguous float64 CUDA tensors")
            ptrs = [ctypes.c_void_p(t.data_ptr()) for t in arrs] + [None] * (4 - len(arrs))
            check(lib().tpf_set_state(self.ctx, *ptrs[:4], 1), "tpf_set_state")
            return
        arrs = [_host(phi, self.N)] + [_host(x, self.N) for x in u]
        ptrs = [a.ctypes.data_as(ctypes.c_void_p) for a in arrs] + [None] * (4 - len(arrs))
        check(lib().tpf_set_state(self.ctx, *ptrs[:4], 0), "tpf_set_state")

    def field_offset(self, field: int):
        """(byte offset in the workspace, tpf_dtype) of a state field."""
        off = ctypes.c_size_t(0)
        ty = ctypes.c_int32(0)
        check(lib().tpf_field_offset(self.ctx, int(field), ctypes.byref(off), ctypes.byref(ty)),
              "tpf_field_offset")
        return int(off.value), ty.value

    def _view(self, field: int):
        torch = self.torch
        off, ty = self.field_offset(field)
        dt, esz = (torch.float32, 4) if ty == TPF_DTYPE_F32 else (torch.float64, 8)
        return self.workspace[off:off + self.N * esz].view(dt).view(self.shape)

    def state_views(self):
        """Zero-copy tensors over the current state inside the workspace:
        (phi, [u_a], p), in the state's own precision (p always float64).
        phi, u and p move to another array at every step: take new views
        after step()/step_adjoint().  After writing phi or u through them,
        call state_changed()."""
        phi = self._view(TPF_STATE_PHI)
        u = [self._view(TPF_STATE_U0 + a) for a in range(self.dim)]
        return phi, u, self._view(TPF_STATE_P)

    def state_changed(self):
        """Bookkeeping of tpf_set_state after an in-place write of the state."""
        check(lib().tpf_state_changed(self.ctx), "tpf_state_changed")

    def init_droplet(self, center, semi_axes):
        c = (ctypes.c_double * 3)(*(list(center) + [0.0] * (3 - len(center))))
        s = (ctypes.c_double * 3)(*(list(semi_axes) + [1.0] * (3 - len(semi_axes))))
        check(lib().tpf_init_droplet(self.ctx, c, s), "tpf_init_droplet")

    def step(self, dt: float, nsteps: int = 1):
        check(lib().tpf_step(self.ctx, float(dt), int(nsteps)), "tpf_step")

    def implicit_phase_step(self, dt: float, nsteps: int = 1, newton_tol: float = 0.0,
                            krylov_rtol: float = 0.0, newton_maxit: int = 0, krylov_maxit: int = 0) -> dict:
        """Backward-Euler ISODI phase-field steps (tpf_implicit_phase_step);
        returns the iteration counts."""
        o = tpf_implicit_opts(float(newton_tol), float(krylov_rtol), int(newton_maxit), int(krylov_maxit))
        info = tpf_implicit_info()
        check(lib().tpf_implicit_phase_step(self.ctx, float(dt), int(nsteps), ctypes.byref(o),
                                            ctypes.byref(info)), "tpf_implicit_phase_step")
        return info.as_dict()

    def get_state(self, with_pressure: bool = False):
        """Host numpy copies: (phi, [u_a], p or None), C-order grid shape."""
        phi = np.empty(self.shape)
        u = [np.empty(self.shape) for _ in range(self.dim)]
        p = np.empty(self.shape) if with_pressure else None
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a is not None else None
        uu = [ptr(x) for x in u] + [None] * (3 - self.dim)
        check(lib().tpf_get_state(self.ctx, ptr(phi), *uu, ptr(p), 0), "tpf_get_state")
        return phi, u, p

    def get_state_device(self):
        """(phi, [u_a]) as new CUDA float64 tensors of the grid shape."""
        torch = self.torch
        phi = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        u = [torch.empty(self.shape, dtype=torch.float64, device=self.device) for _ in range(self.dim)]
        ptrs = [ctypes.c_void_p(t.data_ptr()) for t in u] + [None] * (3 - self.dim)
        check(lib().tpf_get_state(self.ctx, ctypes.c_void_p(phi.data_ptr()), *ptrs, None, 1), "tpf_get_state")
        return phi, u

    def diagnostics(self) -> dict:
        d = tpf_diag()
        check(lib().tpf_diagnostics(self.ctx, ctypes.byref(d)), "tpf_diagnostics")
        return d.as_dict()

    def eval_field(self, name: str) -> np.ndarray:
        out = np.empty(self.shape)
        check(lib().tpf_eval_field(self.ctx, FIELD[name], out.ctypes.data_as(ctypes.c_void_p), 0),
              "tpf_eval_field")
        return out

    def poisson_solve(self, b, x0=None):
        bb = _host(b, self.N)
        x = _host(x0, self.N).copy() if x0 is not None else np.zeros(self.N)
        it = ctypes.c_int32(0)
        rr = ctypes.c_double(0)
        check(lib().tpf_poisson_solve(self.ctx, bb.ctypes.data_as(ctypes.c_void_p),
                                      x.ctypes.data_as(ctypes.c_void_p), 0, ctypes.byref(it),
                                      ctypes.byref(rr)), "tpf_poisson_solve")
        return x.reshape(self.shape), it.value, rr.value

    def solver_stats(self, reset: bool = False) -> dict:
        """Pressure solves, outer and PCG iterations since the last reset."""
        out = (ctypes.c_int64 * 7)()
        check(lib().tpf_solver_stats(self.ctx, out, int(reset)), "tpf_solver_stats")
        return {"solves": out[0], "outer": out[1], "inner": out[2], "recent": list(out[3:7])}

    # ---------------------------------------------------------------- checkpoints
    def checkpoint_bytes(self) -> int:
        out = ctypes.c_size_t(0)
        check(lib().tpf_checkpoint_bytes(self.ctx, ctypes.byref(out)), "tpf_checkpoint_bytes")
        return int(out.value)

    def save_checkpoint(self, buf=None):
        """Save the state into a device uint8 tensor (allocated if None)."""
        if buf is None:
            buf = self.torch.empty(self.checkpoint_bytes(), dtype=self.torch.uint8, device=self.device)
        check(lib().tpf_save_checkpoint(self.ctx, ctypes.c_void_p(buf.data_ptr())), "tpf_save_checkpoint")
        return buf

    def load_checkpoint(self, buf):
        check(lib().tpf_load_checkpoint(self.ctx, ctypes.c_void_p(buf.data_ptr())), "tpf_load_checkpoint")

    # ---------------------------------------------------------------- adjoint
    def tape_bytes(self, nsteps: int) -> int:
        out = ctypes.c_size_t(0)
        check(lib().tpf_adjoint_tape_bytes(self.ctx, int(nsteps), ctypes.byref(out)), "tpf_adjoint_tape_bytes")
        return int(out.value)

    def stage_adjoint(self, lphi, lu):
        """F'(y)^T (lphi, lu) of one stage evaluation at the current state:
        (gphi, [gu_a], [d/dsigma, d/deps]) as host arrays."""
        a = [_host(lphi, self.N)] + [_host(lu[k], self.N) for k in range(self.dim)]
        out = [np.empty(self.shape) for _ in range(1 + self.dim)]
        gp = (ctypes.c_double * 2)(0.0, 0.0)
        ptr = lambda x: x.ctypes.data_as(ctypes.c_void_p)
        ins = [ptr(x) for x in a] + [None] * (3 - self.dim)
        outs = [ptr(x) for x in out] + [None] * (3 - self.dim)
        check(lib().tpf_stage_adjoint(self.ctx, *ins, *outs, gp, 0), "tpf_stage_adjoint")
        return out[0], out[1:], [gp[0], gp[1]]

    def step_adjoint(self, dt: float, nsteps: int, gphi, gu, tape=None, grad_params=None):
        """Run nsteps from the current state recording a tape, then sweep
        back: returns (dL/dphi_0, [dL/du_0], grad_params + dL/d(sigma, eps)).
        gphi, gu: dL/dy at the end (host arrays or CUDA float64 tensors)."""
        torch = self.torch
        if tape is None:
            tape = torch.empty(max(self.tape_bytes(nsteps), 1), dtype=torch.uint8, device=self.device)
        gp = (ctypes.c_double * 2)(*(grad_params if grad_params is not None else (0.0, 0.0)))
        pad = [None] * (3 - self.dim)
        if isinstance(gphi, torch.Tensor):
            arrs = [gphi.contiguous().clone()] + [gu[k].contiguous().clone() for k in range(self.dim)]
            for t in arrs:
                if t.dtype != torch.float64 or not t.is_cuda:
                    raise ValueError("device cotangents must be float64 CUDA tensors")
            ptrs = [ctypes.c_void_p(t.data_ptr()) for t in arrs] + pad
            check(lib().tpf_step_adjoint(self.ctx, ctypes.c_void_p(tape.data_ptr()), tape.numel(), float(dt),
                                         int(nsteps), *ptrs, 1, gp), "tpf_step_adjoint")
            return arrs[0], arrs[1:], [gp[0], gp[1]]
        arrs = [_host(gphi, self.N).copy()] + [_host(gu[k], self.N).copy() for k in range(self.dim)]
        ptrs = [a.ctypes.data_as(ctypes.c_void_p) for a in arrs] + pad
        check(lib().tpf_step_adjoint(self.ctx, ctypes.c_void_p(tape.data_ptr()), tape.numel(), float(dt),
                                     int(nsteps), *ptrs, 0, gp), "tpf_step_adjoint")
        return (arrs[0].reshape(self.shape), [x.reshape(self.shape) for x in arrs[1:]], [gp[0], gp[1]])

    # ---------------------------------------------------------------- profiling
    def profile_enable(self, mask: int = -1):
        """Time the kernel classes in the bit mask (-1: all, 0: stop)."""
        check(lib().tpf_profile_enable(self.ctx, int(mask)), "tpf_profile_enable")

    def profile_classes(self) -> list:
        out = []
        for q in range(lib().tpf_profile_classes()):
            name = ctypes.c_char_p()
            check(lib().tpf_profile_read(self.ctx, q, ctypes.byref(name), None, None, None),
                  "tpf_profile_read")
            out.append(name.value.decode())
        return out

    def profile_read(self) -> dict:
        out = {}
        for q in range(lib().tpf_profile_classes()):
            name = ctypes.c_char_p()
            ms = ctypes.c_double()
            nl = ctypes.c_int64()
            bpl = ctypes.c_double()
            check(lib().tpf_profile_read(self.ctx, q, ctypes.byref(name), ctypes.byref(ms),
                                         ctypes.byref(nl), ctypes.byref(bpl)), "tpf_profile_read")
            out[name.value.decode()] = {"ms": ms.value, "launches": nl.value,
                                        "bytes_per_launch": bpl.value}
        return out


def solver_for_case(case, **overrides) -> Solver:
    """Solver for a workloads.Case (grid, properties, model, force, precision)."""
    kw = dict(length=case.length, model=case.model, force=case.force, precision=case.precision,
              sigma=case.sigma, eps=case.eps, gamma=case.gamma, rho1=case.rho1, rho2=case.rho2,
              visc1=case.visc1, visc2=case.visc2)
    kw.update(overrides)
    return Solver(make_params(case.n, **kw))


def params_for_case(case, **overrides) -> tpf_params:
    kw = dict(length=case.length, model=case.model, force=case.force, precision=case.precision,
              sigma=case.sigma, eps=case.eps, gamma=case.gamma, rho1=case.rho1, rho2=case.rho2,
              visc1=case.visc1, visc2=case.visc2)
    kw.update(overrides)
    return make_params(case.n, **kw)


def batch_workspace_bytes(params: list) -> int:
    arr = (tpf_params * len(params))(*params)
    out = ctypes.c_size_t(0)
    check(lib().tpf_batch_workspace_bytes(arr, len(params), ctypes.byref(out)), "tpf_batch_workspace_bytes")
    return int(out.value)


def batch_configs() -> list:
    """[(threads, lds_bytes)] of the batched launch configurations."""
    out = []
    for q in range(lib().tpf_batch_configs()):
        t, b = ctypes.c_int32(), ctypes.c_int32()
        check(lib().tpf_batch_config_info(q, ctypes.byref(t), ctypes.byref(b)), "tpf_batch_config_info")
        out.append((t.value, b.value))
    return out


class Batch:
    """Many independent 2D cases stepped together (one launch per step)."""

    def __init__(self, params: list, stream=None, device=None):
        import torch
        self.torch = torch
        self.params = list(params)
        self.ncases = len(self.params)
        self.shapes = [(p.n[1], p.n[0]) for p in self.params]
        self.device = torch.device(device or "cuda")
        arr = (tpf_params * self.ncases)(*self.params)
        nbytes = batch_workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        check(lib().tpf_batch_create(arr, self.ncases, ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
              "tpf_batch_create")
        self.h = h

    def close(self):
        if self.h:
            check(lib().tpf_batch_destroy(self.h), "tpf_batch_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dts(self, dt):
        d = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (self.ncases,)))
        return d, d.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def set_state(self, q: int, phi, u):
        N = int(np.prod(self.shapes[q]))
        a = [_host(phi, N), _host(u[0], N), _host(u[1], N)]
        ptrs = [x.ctypes.data_as(ctypes.c_void_p) for x in a]
        check(lib().tpf_batch_set_state(self.h, q, *ptrs, 0), "tpf_batch_set_state")

    def init_droplet(self, q: int, center, semi_axes):
        c = (ctypes.c_double * 2)(*center[:2])
        s = (ctypes.c_double * 2)(*semi_axes[:2])
        check(lib().tpf_batch_init_droplet(self.h, q, c, s), "tpf_batch_init_droplet")

    def get_state(self, q: int, with_pressure: bool = False):
        shape = self.shapes[q]
        phi = np.empty(shape)
        u = [np.empty(shape), np.empty(shape)]
        p = np.empty(shape) if with_pressure else None
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a is not None else None
        check(lib().tpf_batch_get_state(self.h, q, ptr(phi), ptr(u[0]), ptr(u[1]), ptr(p), 0),
              "tpf_batch_get_state")
        return phi, u, p

    def step(self, dt, nsteps: int = 1):
        d, dp = self._dts(dt)
        check(lib().tpf_batch_step(self.h, dp, int(nsteps)), "tpf_batch_step")

    def status(self):
        st = np.zeros(self.ncases, dtype=np.int32)
        steps = np.zeros(self.ncases, dtype=np.int64)
        t = np.zeros(self.ncases)
        check(lib().tpf_batch_status(self.h, st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     steps.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "tpf_batch_status")
        return st, steps, t

    def clear_status(self, q: int):
        check(lib().tpf_batch_clear_status(self.h, q), "tpf_batch_clear_status")

    def diagnostics(self) -> list:
        out = (tpf_diag * self.ncases)()
        check(lib().tpf_batch_diagnostics(self.h, out), "tpf_batch_diagnostics")
        return [out[q].as_dict() for q in range(self.ncases)]

    def set_config(self, config: int):
        check(lib().tpf_batch_set_config(self.h, int(config)), "tpf_batch_set_config")

    def solver_stats(self, reset: bool = False) -> dict:
        """Per-case pressure solves and their outer and PCG iterations since
        the last reset (numpy int64 arrays)."""
        out = [np.zeros(self.ncases, dtype=np.int64) for _ in range(3)]
        ptrs = [x.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) for x in out]
        check(lib().tpf_batch_solver_stats(self.h, *ptrs, int(reset)), "tpf_batch_solver_stats")
        return {"solves": out[0], "outer": out[1], "inner": out[2]}

    def tune(self, dt, cache_path=None) -> int:
        d, dp = self._dts(dt)
        ch = ctypes.c_int32(-1)
        path = cache_path.encode() if cache_path else None
        check(lib().tpf_batch_tune(self.h, dp, path, ctypes.byref(ch)), "tpf_batch_tune")
        return ch.value
