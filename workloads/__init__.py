"""Seeded synthetic workloads shared by the oracle tests and the GPU tests.

This module holds configuration constants and random-number recipes only:
no arithmetic of the method itself.  Droplet profiles are produced by each
side's own initialiser; the random fields here are generic smooth periodic
fields (a few seeded Fourier modes) used to exercise operators away from
equilibrium.

The workloads are the paper's static-drop setting (Sec. 3.1: a tanh drop in a
unit box, properties set through the Laplace number) and the oscillating /
batched / adjoint variants that extend it.  Boxes are periodic everywhere.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

MODELS = ("CDI", "SB", "ISODI")
FORCES = ("EB", "CSF", "LCSF")


@dataclass
class Case:
    """One droplet case: grid, geometry, properties, discretisation, steps."""
    name: str
    n: tuple                       # cells per axis (nx, ny[, nz])
    center: tuple
    semi_axes: tuple
    rho1: float
    rho2: float
    visc1: float
    visc2: float
    sigma: float
    eps_over_h: float
    model: str = "CDI"
    force: str = "EB"
    precision: str = "fp64"       # "fp64" or "fp32_mixed"
    gamma: float = 1.0
    steps: int = 1
    length: float = 1.0

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def h(self) -> float:
        return self.length / self.n[0]

    @property
    def eps(self) -> float:
        return self.eps_over_h * self.h

    @property
    def cells(self) -> int:
        return int(np.prod(self.n))

    def dt(self, umax0: float = 0.0) -> float:
        return stable_dt(self.h, self.eps, self.gamma, umax0, self.rho1, self.rho2,
                         self.visc1, self.visc2, self.sigma)

    def to_dict(self) -> dict:
        return asdict(self)


def stable_dt(h, eps, gamma, umax0, rho1, rho2, visc1, visc2, sigma, cfl=0.1):
    """Time step of the explicit scheme: the smallest of the advective
    (cfl h / max(gamma, |u|)), regularisation-diffusion (cfl h^2/(gamma eps)),
    viscous (cfl h^2 / nu_max) and capillary (0.5 sqrt((rho1+rho2) h^3 /
    (4 pi sigma))) limits."""
    nu_max = max(visc1 / rho1, visc2 / rho2)
    lims = [cfl * h / max(gamma, umax0), cfl * h * h / (gamma * eps)]
    if nu_max > 0:
        lims.append(cfl * h * h / nu_max)
    if sigma > 0:
        lims.append(0.5 * math.sqrt((rho1 + rho2) * h ** 3 / (4.0 * math.pi * sigma)))
    return min(lims)


# ---------------------------------------------------------------- the five cases
def static_drop_64() -> Case:
    """64^2 static drop, uniform properties, La = sigma rho D / visc^2 = 12000
    with D = 0.5 and visc = 0.1 (rho = 240), CDI + energy-based force, FP64."""
    return Case("static_drop_64", (64, 64), (0.5, 0.5), (0.25, 0.25), 240.0, 240.0, 0.1, 0.1,
                1.0, 1.0, "CDI", "EB", "fp64", steps=200)


def static_drop_ratio(n: int, eps_over_h: float, model: str, force: str,
                      precision: str = "fp64") -> Case:
    """n^2 static drop, density ratio 1000 and viscosity ratio 100."""
    return Case(f"static_drop_{n}_{model}_{force}_{eps_over_h}", (n, n), (0.5, 0.5), (0.25, 0.25),
                240.0, 0.24, 0.1, 0.001, 1.0, eps_over_h, model, force, precision, steps=2000)


def oscillating_drop_3d(n: int = 256, precision: str = "fp32_mixed") -> Case:
    """n^3 oscillating ellipsoid (0.30, 0.25, 0.25), density and viscosity
    ratio 10, eps = 0.75 h, CDI + energy-based force."""
    return Case(f"oscillating_drop_{n}^3", (n, n, n), (0.5, 0.5, 0.5), (0.30, 0.25, 0.25),
                1.0, 0.1, 2e-3, 2e-4, 1.0, 0.75, "CDI", "EB", precision, steps=1000)


def oscillating_drop_2d(n: int = 256, precision: str = "fp32_mixed") -> Case:
    """n^2 oscillating ellipse (0.30, 0.22), density ratio 10 (adjoint case)."""
    return Case(f"oscillating_drop_{n}^2", (n, n), (0.5, 0.5), (0.30, 0.22),
                1.0, 0.1, 2e-3, 2e-4, 1.0, 1.0, "CDI", "EB", precision, steps=500)


def batched_cases(ncases: int = 512, seed: int = 0, precision: str = "fp32_mixed"):
    """Uneven batch of 2D drops.  numpy default_rng(seed); draw order: grid
    index in {64, 96, 128, 192}, R ~ U[0.15, 0.35], sigma ~ U[0.5, 2],
    eps/h ~ U[0.5, 1], log10(density ratio) ~ U[0, 3].  rho1 = 1,
    rho2 = 10^-x, visc1 = 0.01, visc2 = 0.01 rho2 (equal kinematic viscosity)."""
    rng = np.random.default_rng(seed)
    grids = np.array([64, 96, 128, 192])
    gi = rng.integers(0, 4, size=ncases)
    R = rng.uniform(0.15, 0.35, size=ncases)
    sig = rng.uniform(0.5, 2.0, size=ncases)
    eoh = rng.uniform(0.5, 1.0, size=ncases)
    lr = rng.uniform(0.0, 3.0, size=ncases)
    out = []
    for q in range(ncases):
        n = int(grids[gi[q]])
        rho2 = 10.0 ** (-lr[q])
        out.append(Case(f"batch_{q}", (n, n), (0.5, 0.5), (float(R[q]),) * 2, 1.0, rho2, 0.01,
                        0.01 * rho2, float(sig[q]), float(eoh[q]), "CDI", "EB", precision,
                        steps=500))
    return out


# ---------------------------------------------------------------- random fields
def smooth_field(shape, seed: int, modes: int = 3, amplitude: float = 1.0,
                 offset: float = 0.0) -> np.ndarray:
    """Seeded smooth periodic field: sum of random low Fourier modes on the
    cell-centre grid of the unit box.  shape is C order (nz, ny, nx) or (ny, nx)."""
    rng = np.random.default_rng(seed)
    dim = len(shape)
    coords = np.meshgrid(*[(np.arange(m) + 0.5) / m for m in shape], indexing="ij")
    out = np.full(shape, float(offset))
    for _ in range(modes):
        k = rng.integers(-3, 4, size=dim)
        ph = rng.uniform(0, 2 * math.pi)
        a = rng.normal()
        arg = sum(2 * math.pi * k[d] * coords[d] for d in range(dim)) + ph
        out += amplitude * a / modes * np.cos(arg)
    return np.ascontiguousarray(out)


def noise_field(shape, seed: int, amplitude: float = 1.0) -> np.ndarray:
    """Seeded white noise (uniform in [-amplitude, amplitude])."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(-amplitude, amplitude, size=shape))


def random_velocity(shape, seed: int, amplitude: float = 0.1, smooth: bool = True):
    """dim face-velocity arrays (not divergence free)."""
    dim = len(shape)
    if smooth:
        return [smooth_field(shape, seed + 101 * a, amplitude=amplitude) for a in range(dim)]
    return [noise_field(shape, seed + 101 * a, amplitude) for a in range(dim)]


def _fwd(q, axis_phys, dim):
    """q[c + e_a] - q[c] along physical axis a on a C-order array."""
    return np.roll(q, -1, axis=dim - 1 - axis_phys) - q


def divergence_free_velocity(shape, seed: int, amplitude: float = 0.1):
    """Seeded face velocity whose discrete MAC divergence is zero to round-off:
    the discrete curl of a smooth potential (a stream function on cell
    corners in 2D, a vector potential on cell edges in 3D)."""
    dim = len(shape)
    if dim == 2:
        psi = smooth_field(shape, seed, amplitude=amplitude / (2 * math.pi))
        h = 1.0 / shape[1]
        # psi[j, i] at corner (x_i, y_j); u_x[i,j] = (psi[i,j+1]-psi[i,j])/h ...
        return [np.ascontiguousarray(_fwd(psi, 1, 2) / h),
                np.ascontiguousarray(-_fwd(psi, 0, 2) / h)]
    h = 1.0 / shape[2]
    A = [smooth_field(shape, seed + 7 * a, amplitude=amplitude / (2 * math.pi)) for a in range(3)]
    ux = (_fwd(A[2], 1, 3) - _fwd(A[1], 2, 3)) / h
    uy = (_fwd(A[0], 2, 3) - _fwd(A[2], 0, 3)) / h
    uz = (_fwd(A[1], 0, 3) - _fwd(A[0], 1, 3)) / h
    return [np.ascontiguousarray(x) for x in (ux, uy, uz)]


# ---------------------------------------------------------------- implicit ISODI step
def implicit_drop(n=(256, 256), eps_over_h: float = 1.5) -> Case:
    """Drop for the backward-Euler phase-field step with the ISODI model:
    a circle (sphere) of radius 0.3 of the box centred in the unit box, eps =
    1.5 h, gamma = 1, FP64; the velocity is ``implicit_velocity`` (max |u_a| =
    0.5: half of gamma, the bound the paper keeps gamma above)."""
    dim = len(n)
    return Case(f"implicit_drop_{'x'.join(map(str, n))}", tuple(n), (0.5,) * dim, (0.3,) * dim,
                1.0, 1.0, 0.01, 0.01, 1.0, eps_over_h, "ISODI", "EB", "fp64", gamma=1.0)


def implicit_dt(case: Case, multiple: float) -> float:
    """multiple x h^2 / (2 dim gamma eps): the forward-Euler stability limit of
    the regularisation diffusion gamma eps L."""
    return multiple * case.h ** 2 / (2 * case.dim * case.gamma * case.eps)


def implicit_velocity(shape, seed: int, umax: float = 0.5):
    """``divergence_free_velocity`` scaled so that max_a max |u_a| = umax."""
    u = divergence_free_velocity(shape, seed, amplitude=1.0)
    m = max(float(np.abs(x).max()) for x in u)
    return [np.ascontiguousarray(x * (umax / m)) for x in u]
