"""The fused coarse multigrid levels of the 3D V-cycle (k_cdown, k_cup: one
launch down and one up per stored-coefficient level) against the six
separate kernels per level that they replace, and against the oracle.

The fused kernels do the same per-cell arithmetic in the same order, so
whole RK4 steps must give bitwise-equal states and equal iteration counts
with TPF_COARSE_FUSED=1 and =0.  The grids are chosen so that the fused
levels end in partial 8^3 tiles and so that their coarse grids are smaller
than a tile's coarse halo (periodic aliasing of the staged region).
"""
import os
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_05835_amd import tpf
    tpf.lib()
    return tpf


def drop_case(n, precision, ratio=1000.0):
    return workloads.Case(f"coarse3d_{n[0]}x{n[1]}x{n[2]}", n, (0.5, 0.5, 0.5), (0.3, 0.25, 0.22),
                          ratio, 1.0, 0.02, 0.004, 1.0, 1.0, "CDI", "EB", precision)


def solver(gpu, case, fused, **kw):
    os.environ["TPF_COARSE_FUSED"] = fused
    try:
        return gpu.solver_for_case(case, **kw)
    finally:
        del os.environ["TPF_COARSE_FUSED"]


@pytest.mark.parametrize("precision,n", [("fp32_mixed", (64, 64, 64)), ("fp32_mixed", (72, 24, 40)),
                                         ("fp64", (48, 40, 56)), ("fp32_mixed", (96, 48, 32))])
def test_coarse_fused_bitwise(gpu, precision, n):
    case = drop_case(n, precision)
    dt = 2e-4
    say(f"fused coarse levels {precision} {n}")
    out = []
    for fused in ("0", "1"):
        s = solver(gpu, case, fused)
        s.init_droplet(case.center, case.semi_axes)
        u = workloads.random_velocity(tuple(reversed(n)), 9, amplitude=0.05)
        phi, _, _ = s.get_state()
        s.set_state(phi, u)
        s.solver_stats(reset=True)
        s.step(dt, 3)
        st = s.solver_stats()
        out.append((s.get_state(), st))
        say(f"  TPF_COARSE_FUSED={fused}: {st}")
    (a_phi, a_u, a_p), sa = out[0]
    (b_phi, b_u, b_p), sb = out[1]
    assert sa["inner"] == sb["inner"] and sa["outer"] == sb["outer"]
    assert np.array_equal(a_phi, b_phi)
    for a in range(3):
        assert np.array_equal(a_u[a], b_u[a]), a
    assert np.array_equal(a_p, b_p)


@pytest.mark.parametrize("n", [(40, 32, 24), (48, 40, 56)])
def test_poisson_solve_fp64_fused(gpu, ora, n):
    """The FP64 solve with the fused levels forced on equals the oracle's
    converged solution at density ratio 1000 (random right-hand side)."""
    case = drop_case(n, "fp64")
    say(f"poisson fp64 fused {n}")
    P = ora.Params(n=case.n, length=case.length, rho1=case.rho1, rho2=case.rho2)
    phi = ora.init_droplet(P, case.center, case.semi_axes)
    s = solver(gpu, case, "1", poisson_rtol=1e-14, poisson_maxit=1000)
    s.set_state(phi, [np.zeros(P.shape)] * 3)
    b = workloads.noise_field(P.shape, 17)
    x_g, it, rr = s.poisson_solve(b)
    x_o, _, _ = ora.poisson_solve(P, phi, b)
    say(f"  iterations {it} relres {rr:.2e}")
    assert rr <= 1e-14
    assert np.abs(x_g - x_o).max() < 1e-11 * np.abs(x_o).max()
