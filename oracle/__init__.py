"""Plain FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``tpf_oracle.c`` (plain C,
OpenMP over rows, fixed-order reductions) through ctypes and shares no code
with the HIP library in ``paper_2205_05835_amd/``.

Method: one time step of the two-phase solver of Mirjalili, Khanwale & Mani
(arXiv 2205.05835) -- phase-field models of Table 1, chemical potential of
Eq. 2, surface-tension forces (energy-based Eq. 4, CSF, localized CSF of
Eq. 11), central second-order staggered-grid operators and classical RK4
(Sec. 3), with a variable-density pressure projection at every stage.

Arrays are numpy float64, C order, shape ``(nz, ny, nx)`` in 3D and
``(ny, nx)`` in 2D; ``u`` is a list of ``dim`` face arrays where ``u[a][c]``
sits on the lower a-face of cell ``c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tpf_oracle.c")
_LIB = os.path.join(_HERE, "libtpf_oracle.so")

CDI, SB, ISODI = 0, 1, 2
EB, CSF, LCSF, EB_GAUGE = 0, 1, 2, 3
MODELS = {"CDI": CDI, "SB": SB, "ISODI": ISODI}
FORCES = {"EB": EB, "CSF": CSF, "LCSF": LCSF}

DIAG_NAMES = ("mass", "phi_min", "phi_max", "umax", "ca_inf", "ke", "se", "dp", "div_max")


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/libtpf_oracle.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _P(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.c_double),
                ("model", ctypes.c_int), ("force", ctypes.c_int),
                ("sigma", ctypes.c_double), ("eps", ctypes.c_double), ("gamma", ctypes.c_double),
                ("rho1", ctypes.c_double), ("rho2", ctypes.c_double),
                ("visc1", ctypes.c_double), ("visc2", ctypes.c_double),
                ("delta", ctypes.c_double), ("clamp", ctypes.c_int),
                ("poisson_rtol", ctypes.c_double), ("poisson_maxit", ctypes.c_int),
                ("walls", ctypes.c_int)]


@dataclass
class Params:
    """Physical and numerical parameters of one case (unit-free)."""
    n: tuple                 # cells per axis, (nx, ny) or (nx, ny, nz)
    length: float = 1.0      # box edge along x; h = length / nx
    model: int = CDI
    force: int = EB
    sigma: float = 1.0
    eps: float = 0.0         # 0 -> one cell width
    gamma: float = 1.0
    rho1: float = 1.0
    rho2: float = 1.0
    visc1: float = 0.1
    visc2: float = 0.1
    delta: float = 1e-12
    clamp: int = 1
    poisson_rtol: float = 1e-14
    poisson_maxit: int = 200000
    walls: int = 0           # bit a: free-slip walls at both ends of axis a (x = bit 0)

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def h(self) -> float:
        return self.length / self.n[0]

    @property
    def shape(self) -> tuple:
        return tuple(reversed(self.n))

    @property
    def epsilon(self) -> float:
        return self.eps if self.eps > 0 else self.h

    def c(self) -> _P:
        n3 = list(self.n) + [1] * (3 - len(self.n))
        return _P(self.dim, (ctypes.c_int * 3)(*n3), self.h, int(self.model), int(self.force),
                  self.sigma, self.epsilon, self.gamma, self.rho1, self.rho2, self.visc1,
                  self.visc2, self.delta, int(self.clamp), self.poisson_rtol, self.poisson_maxit,
                  int(self.walls))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_P)
        sig = {
            "ora_normals": [pp, dp, dp, dp, dp, dp],
            "ora_curvature": [pp, dp, dp],
            "ora_chem_potential": [pp, dp, dp],
            "ora_regularization": [pp, dp, dp],
            "ora_cdi_flux": [pp, dp, dp, dp, dp],
            "ora_phase_rhs": [pp, dp, dp, dp, dp, dp],
            "ora_surface_force": [pp, dp, dp, dp, dp],
            "ora_mass_flux": [pp, dp, dp, dp, dp, dp, dp, dp],
            "ora_advection": [pp, dp, dp, dp, dp, dp, dp, dp, dp, dp],
            "ora_viscous": [pp, dp, dp, dp, dp, dp, dp, dp],
            "ora_viscosity_field": [pp, dp, dp],
            "ora_fstar": [pp, dp, dp, dp, dp, dp, dp, dp],
            "ora_divergence": [pp, dp, dp, dp, dp],
            "ora_poisson_apply": [pp, dp, dp, dp],
            "ora_poisson_solve": [pp, dp, dp, dp, ctypes.POINTER(ctypes.c_int), dp],
            "ora_stage": [pp, dp, dp, dp, dp, dp, dp, dp, dp, dp],
            "ora_step": [pp, ctypes.c_double, ctypes.c_int, dp, dp, dp, dp, dp],
            "ora_init_droplet": [pp, dp, dp, dp],
            "ora_diagnostics": [pp, dp, dp, dp, dp, dp, dp],
        }
        L.ora_threads.argtypes = []
        L.ora_threads.restype = ctypes.c_int
        L.ora_set_threads.argtypes = [ctypes.c_int]
        L.ora_set_threads.restype = ctypes.c_int
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int if name in ("ora_poisson_solve", "ora_stage", "ora_step") else None
        _lib = L
    return _lib


def threads() -> int:
    """OpenMP threads the oracle uses (OMP_NUM_THREADS or all host cores)."""
    return int(lib().ora_threads())


def set_threads(n: int) -> int:
    """Use n OpenMP threads from now on; returns the previous count."""
    return int(lib().ora_set_threads(int(n)))


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _arr(P: Params, a=None):
    if a is None:
        return np.zeros(P.shape, dtype=np.float64)
    return np.ascontiguousarray(a, dtype=np.float64).reshape(P.shape)


def _vec(P: Params, u):
    """List of 3 face arrays (missing components zero)."""
    out = [_arr(P, u[a]) if (u is not None and a < len(u)) else _arr(P) for a in range(3)]
    return out


# ---------------------------------------------------------------- operators
def normals(P: Params, phi):
    n = [_arr(P) for _ in range(3)]
    gmag = _arr(P)
    lib().ora_normals(ctypes.byref(P.c()), _ptr(_arr(P, phi)), *map(_ptr, n), _ptr(gmag))
    return n[:P.dim], gmag


def curvature(P: Params, phi):
    k = _arr(P)
    lib().ora_curvature(ctypes.byref(P.c()), _ptr(_arr(P, phi)), _ptr(k))
    return k


def chem_potential(P: Params, phi):
    mu = _arr(P)
    lib().ora_chem_potential(ctypes.byref(P.c()), _ptr(_arr(P, phi)), _ptr(mu))
    return mu


def regularization(P: Params, phi):
    g = _arr(P)
    lib().ora_regularization(ctypes.byref(P.c()), _ptr(_arr(P, phi)), _ptr(g))
    return g


def cdi_flux(P: Params, phi):
    r = [_arr(P) for _ in range(3)]
    lib().ora_cdi_flux(ctypes.byref(P.c()), _ptr(_arr(P, phi)), *map(_ptr, r))
    return r[:P.dim]


def phase_rhs(P: Params, phi, u):
    uu = _vec(P, u)
    d = _arr(P)
    lib().ora_phase_rhs(ctypes.byref(P.c()), _ptr(_arr(P, phi)), *map(_ptr, uu), _ptr(d))
    return d


def surface_force(P: Params, phi):
    F = [_arr(P) for _ in range(3)]
    lib().ora_surface_force(ctypes.byref(P.c()), _ptr(_arr(P, phi)), *map(_ptr, F))
    return F[:P.dim]


def mass_flux(P: Params, phi, u):
    uu = _vec(P, u)
    m = [_arr(P) for _ in range(3)]
    lib().ora_mass_flux(ctypes.byref(P.c()), _ptr(_arr(P, phi)), *map(_ptr, uu), *map(_ptr, m))
    return m[:P.dim]


def advection(P: Params, m, u):
    mm, uu = _vec(P, m), _vec(P, u)
    N = [_arr(P) for _ in range(3)]
    lib().ora_advection(ctypes.byref(P.c()), *map(_ptr, mm), *map(_ptr, uu), *map(_ptr, N))
    return N[:P.dim]


def viscous(P: Params, eta, u):
    uu = _vec(P, u)
    V = [_arr(P) for _ in range(3)]
    lib().ora_viscous(ctypes.byref(P.c()), _ptr(_arr(P, eta)), *map(_ptr, uu), *map(_ptr, V))
    return V[:P.dim]


def viscosity_field(P: Params, phi):
    e = _arr(P)
    lib().ora_viscosity_field(ctypes.byref(P.c()), _ptr(_arr(P, phi)), _ptr(e))
    return e


def fstar(P: Params, phi, u):
    uu = _vec(P, u)
    f = [_arr(P) for _ in range(3)]
    lib().ora_fstar(ctypes.byref(P.c()), _ptr(_arr(P, phi)), *map(_ptr, uu), *map(_ptr, f))
    return f[:P.dim]


def divergence(P: Params, F):
    FF = _vec(P, F)
    out = _arr(P)
    lib().ora_divergence(ctypes.byref(P.c()), *map(_ptr, FF), _ptr(out))
    return out


def poisson_apply(P: Params, phi, x):
    y = _arr(P)
    lib().ora_poisson_apply(ctypes.byref(P.c()), _ptr(_arr(P, phi)), _ptr(_arr(P, x)), _ptr(y))
    return y


def poisson_solve(P: Params, phi, b, x0=None):
    """Return (x, iterations, relative residual); raises if not converged."""
    x = _arr(P, x0).copy() if x0 is not None else _arr(P)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    rc = lib().ora_poisson_solve(ctypes.byref(P.c()), _ptr(_arr(P, phi)), _ptr(_arr(P, b)),
                                 _ptr(x), ctypes.byref(it), ctypes.byref(rr))
    if rc != 0:
        raise RuntimeError(f"oracle Poisson solve did not converge (relres {rr.value:.3e})")
    return x, it.value, rr.value


def stage(P: Params, phi, u, pres=None):
    """Projected stage derivative: (dphi/dt, [du_a/dt], p)."""
    uu = _vec(P, u)
    d = _arr(P)
    du = [_arr(P) for _ in range(3)]
    p = _arr(P, pres).copy() if pres is not None else _arr(P)
    rc = lib().ora_stage(ctypes.byref(P.c()), _ptr(_arr(P, phi)), _ptr(uu[0]), _ptr(uu[1]),
                         _ptr(uu[2]) if P.dim == 3 else None, _ptr(d), *map(_ptr, du), _ptr(p))
    if rc != 0:
        raise RuntimeError("oracle Poisson solve did not converge")
    return d, du[:P.dim], p


def step(P: Params, dt: float, nsteps: int, phi, u, pres=None):
    """Advance nsteps RK4 steps; returns new (phi, u, p_warm) (inputs untouched)."""
    f = _arr(P, phi).copy()
    uu = [x.copy() for x in _vec(P, u)]
    p = _arr(P, pres).copy() if pres is not None else _arr(P)
    rc = lib().ora_step(ctypes.byref(P.c()), float(dt), int(nsteps), _ptr(f), _ptr(uu[0]),
                        _ptr(uu[1]), _ptr(uu[2]) if P.dim == 3 else None, _ptr(p))
    if rc != 0:
        raise RuntimeError("oracle Poisson solve did not converge")
    return f, uu[:P.dim], p


def pressure(P: Params, phi, u, pres=None):
    """Projection pressure of state (phi, u): the p of a stage evaluation there."""
    return stage(P, phi, u, pres)[2]


def init_droplet(P: Params, center, semi_axes):
    phi = _arr(P)
    c = (ctypes.c_double * 3)(*(list(center) + [0.0] * (3 - len(center))))
    s = (ctypes.c_double * 3)(*(list(semi_axes) + [1.0] * (3 - len(semi_axes))))
    lib().ora_init_droplet(ctypes.byref(P.c()), c, s, _ptr(phi))
    return phi


def diagnostics(P: Params, phi, u, pres=None) -> dict:
    uu = _vec(P, u)
    out = (ctypes.c_double * len(DIAG_NAMES))()
    lib().ora_diagnostics(ctypes.byref(P.c()), _ptr(_arr(P, phi)), *map(_ptr, uu),
                          _ptr(_arr(P, pres)) if pres is not None else None, out)
    return dict(zip(DIAG_NAMES, list(out)))
