"""Pins of the backward-Euler ISODI oracle (oracle/implicit.py).

Each test fixes the implicit step against something other than the oracle
itself: the exact root of the cubic a uniform state obeys, the exact
amplification factor of the linearised scheme on a Fourier mode, and the
second-order term that separates backward from forward Euler, built from the
pinned right-hand side of Eq. 1.  No GPU is needed.
"""
import math

import numpy as np
import pytest

import workloads


@pytest.fixture(scope="module")
def ora():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="module")
def imp():
    from oracle import implicit
    return implicit


def test_uniform_state_is_root_of_cubic(ora, imp):
    """A uniform phi under a uniform velocity has no transport, Laplacian or
    normal, so backward Euler reduces to phi1 - phi0 + (dt gamma / eps) psi'(phi1)
    = 0 with psi'(f) = f - 3 f^2 + 2 f^3: the root of a cubic next to phi0.
    (delta = 1e-3 keeps the normals linear over the oracle's finite-difference
    Jacobian steps; the root does not depend on it, since C phi = 0.)"""
    P = ora.Params(n=(6, 5), model=ora.ISODI, eps=0.05, gamma=1.3, delta=1e-3)
    for phi0, dt in [(0.3, 0.01), (0.8, 0.05), (0.52, 0.2), (-0.1, 0.02)]:
        a = dt * P.gamma / P.epsilon
        roots = np.roots([2 * a, -3 * a, 1 + a, -phi0])
        real = roots[np.abs(roots.imag) < 1e-12].real
        want = real[np.argmin(np.abs(real - phi0))]
        u = [np.full(P.shape, 0.7), np.full(P.shape, -0.4)]
        got, it, res = imp.isodi_backward_euler(P, dt, np.full(P.shape, phi0), u, tol=1e-14)
        assert np.max(np.abs(got - want)) < 1e-13, (phi0, dt)


@pytest.mark.parametrize("dim,n,k", [(2, (8, 6), (1, 2)), (2, (10, 10), (3, -1)), (3, (6, 4, 5), (1, 1, 2))])
def test_fourier_mode_amplification(ora, imp, dim, n, k):
    """Near phi = 0 and with a large normal regularisation delta (n ~ C phi /
    delta, so the curvature term phi (1 - phi) kappa is quadratic in the
    amplitude) the step is linear: -D(U A phi) + gamma (eps L phi - phi / eps).
    A mode exp(i k.x) is multiplied by 1 / (1 + dt [gamma (eps lam + 1/eps) +
    i sum_a U_a sin(k_a h) / h]) with lam = sum_a (4/h^2) sin^2(k_a h / 2), the
    eigenvalues of the central schemes."""
    P = ora.Params(n=n, model=ora.ISODI, eps=0.08, gamma=0.9, delta=1.0)
    h = P.h
    U = [0.6, -0.35, 0.2][:dim]
    kk = [2 * math.pi * k[a] / (n[a] * h) for a in range(dim)]
    coords = np.meshgrid(*[(np.arange(m) + 0.5) * h for m in P.shape], indexing="ij")
    x = coords[::-1]                         # physical axes
    theta = sum(kk[a] * x[a] for a in range(dim)) + 0.4
    amp = 1e-9
    phi0 = amp * np.cos(theta)
    dt = 0.004
    lam = sum(4.0 / h ** 2 * math.sin(kk[a] * h / 2) ** 2 for a in range(dim))
    m = 1.0 / (1.0 + dt * (P.gamma * (P.epsilon * lam + 1.0 / P.epsilon)
                           + 1j * sum(U[a] * math.sin(kk[a] * h) / h for a in range(dim))))
    want = amp * np.real(m * np.exp(1j * theta))
    u = [np.full(P.shape, U[a]) for a in range(dim)]
    got, it, res = imp.isodi_backward_euler(P, dt, phi0, u, tol=1e-24)
    assert np.max(np.abs(got - want)) < 1e-6 * amp


def test_second_order_term_is_backward_euler(ora, imp):
    """phi1 = phi0 + dt R(phi1) gives (phi1 - phi0 - dt R(phi0)) / dt^2 =
    R'(phi0) R(phi0) + O(dt): the term forward Euler lacks and that has the
    opposite sign for an explicit-in-time residual.  R is the pinned right-hand
    side of Eq. 1; R'(phi0) R(phi0) is its central directional difference."""
    case = workloads.implicit_drop((16, 14))
    P = ora.Params(n=case.n, model=ora.ISODI, eps=case.eps, gamma=case.gamma)
    phi0 = ora.init_droplet(P, case.center, (0.3 * 14 / 16,) * 2)
    u = workloads.implicit_velocity(P.shape, seed=3)
    R0 = ora.phase_rhs(P, phi0, u)
    s = 1e-4 / np.max(np.abs(R0))
    JR = (ora.phase_rhs(P, phi0 + s * R0, u) - ora.phase_rhs(P, phi0 - s * R0, u)) / (2 * s)
    errs = []
    for dt in [2e-5, 1e-5]:
        phi1, it, res = imp.isodi_backward_euler(P, dt, phi0, u, tol=1e-16)
        second = (phi1 - phi0 - dt * R0) / dt ** 2
        errs.append(np.max(np.abs(second - JR)) / np.max(np.abs(JR)))
    assert errs[0] < 0.05
    assert 0.4 < errs[1] / errs[0] < 0.6, errs


def test_residual_vanishes_and_rejects_other_models(ora, imp):
    """The returned state is a root of F(phi) = phi - phi0 - dt R(phi); the
    step is defined for ISODI only."""
    case = workloads.implicit_drop((12, 10))
    P = ora.Params(n=case.n, model=ora.ISODI, eps=case.eps, gamma=case.gamma)
    phi0 = ora.init_droplet(P, case.center, (0.25,) * 2)
    u = workloads.implicit_velocity(P.shape, seed=4)
    dt = workloads.implicit_dt(case, 10.0)
    phi1, it, res = imp.isodi_backward_euler(P, dt, phi0, u)
    F = phi1 - phi0 - dt * ora.phase_rhs(P, phi1, u)
    assert np.max(np.abs(F)) <= 1e-13 and it >= 2
    with pytest.raises(ValueError):
        imp.isodi_backward_euler(ora.Params(n=(8, 8), model=ora.SB), dt, phi0, u)
