"""Backward-Euler step of the phase-field equation with the ISODI model --
TEST INFRASTRUCTURE ONLY (same rules as the rest of ``oracle``: only
``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may use it; it shares no code with the HIP library).

Table 1 defines ISODI as the model of Sun and Beckermann with the gradient
magnitude in its curvature term replaced by the equilibrium value
phi (1 - phi) / eps, a change made so that fully implicit time steps can be
solved by Newton's method (the paragraph after Table 1).  The paper gives no
implicit scheme.  The reading used here: the simplest fully implicit step,
backward Euler for Eq. 1 with the face velocity u held fixed over the step,

    F(phi) = phi - phi_old - dt * rhs(phi; u) = 0,

where rhs is the right-hand side of Eq. 1 that ``phase_rhs`` evaluates
(central face interpolation of the advective flux, the ISODI regularisation
with the regularised normals of the Table 1 caption).

The oracle solves F = 0 by Newton's method.  The Jacobian dF/dphi is formed
column by column from central differences of ``phase_rhs`` and the Newton
system is solved densely: slow, for small grids only, and independent of how
the operator is built.  The Jacobian only steers the iteration; the answer is
the root of F, and the loop stops on max |F| alone.  The difference step is
small (1e-9) because the regularised normals change fast where |C phi| is
small, and a wide step smooths that change out of the Jacobian.
"""
from __future__ import annotations

import numpy as np

from . import ISODI, Params, phase_rhs


def be_residual(P: Params, dt: float, phi, phi_old, u):
    """F(phi) = phi - phi_old - dt rhs(phi; u) (backward Euler for Eq. 1)."""
    phi = np.asarray(phi, dtype=np.float64).reshape(P.shape)
    return phi - np.asarray(phi_old, dtype=np.float64).reshape(P.shape) - dt * phase_rhs(P, phi, u)


def isodi_backward_euler(P: Params, dt: float, phi_old, u, tol: float = 1e-13, maxit: int = 40,
                         fd_step: float = 1e-9):
    """One backward-Euler step of Eq. 1 with the ISODI regularisation.

    Returns (phi_new, newton_iterations, max |F| at phi_new).  Raises if max |F|
    does not fall to ``tol`` within ``maxit`` Newton iterations.
    """
    if P.model != ISODI:
        raise ValueError("the implicit step is defined for the ISODI model")
    phi_old = np.ascontiguousarray(phi_old, dtype=np.float64).reshape(P.shape)
    phi = phi_old.copy()
    N = phi.size
    res = np.inf
    for it in range(maxit + 1):
        F = be_residual(P, dt, phi, phi_old, u)
        res = float(np.max(np.abs(F)))
        if res <= tol:
            return phi, it, res
        if not np.isfinite(res) or it == maxit:
            break
        J = np.empty((N, N))
        x = phi.reshape(-1).copy()
        for j in range(N):
            xj = x[j]
            x[j] = xj + fd_step
            Fp = be_residual(P, dt, x, phi_old, u).reshape(-1)
            x[j] = xj - fd_step
            Fm = be_residual(P, dt, x, phi_old, u).reshape(-1)
            x[j] = xj
            J[:, j] = (Fp - Fm) / (2.0 * fd_step)
        phi = phi - np.linalg.solve(J, F.reshape(-1)).reshape(P.shape)
    raise RuntimeError(f"backward-Euler Newton did not converge: max|F| = {res:.3e}")
