"""GPU parity of the backward-Euler ISODI phase-field step
(tpf_implicit_phase_step) against the oracle's dense Newton solve.

Both sides solve F(phi) = phi - phi0 - dt R(phi) = 0 to max |F| <= 1e-12 from
the same inputs (the oracle's droplet and a seeded divergence-free
velocity).  Two roots of F that close differ by at most ||J^-1|| 1e-12, so the
states must agree to 1e-10.  At the full sizes the oracle cannot run Newton;
there its right-hand side of Eq. 1 checks the root the GPU returns.
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-10


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


def setup(ora, n, seed=11, eps_over_h=1.5):
    case = workloads.implicit_drop(n, eps_over_h)
    P = ora.Params(n=case.n, length=case.length, model=ora.ISODI, eps=case.eps, gamma=case.gamma)
    box = [case.h * m for m in case.n]
    R = 0.3 * min(box)
    phi0 = ora.init_droplet(P, [0.5 * b for b in box], [R] * case.dim)
    u = workloads.implicit_velocity(P.shape, seed=seed)
    return case, P, phi0, u


def gpu_step(gpu, case, phi0, u, dt, nsteps=1, **opts):
    s = gpu.solver_for_case(case)
    s.set_state(phi0, u)
    info = s.implicit_phase_step(dt, nsteps, **opts)
    phi, uu, _ = s.get_state()
    return s, phi, uu, info


@pytest.mark.parametrize("n,mult", [((72, 24), 10.0), ((12, 10), 10.0), ((18, 12, 11), 10.0), ((20, 18), 1.0), ((7, 6, 5), 6.0)])
def test_implicit_step_matches_oracle(gpu, ora, n, mult):
    from oracle import implicit
    case, P, phi0, u = setup(ora, n)
    dt = workloads.implicit_dt(case, mult)
    say(f"implicit parity {n} dt={dt:.3e} ({mult} x explicit diffusion limit)")
    ref, it, res = implicit.isodi_backward_euler(P, dt, phi0, u, tol=1e-12)
    s, phi, uu, info = gpu_step(gpu, case, phi0, u, dt)
    say(f"  oracle {it} Newton, GPU {info}")
    assert info["residual"] <= 1e-12 and info["newton_iters"] >= 1
    assert np.abs(phi - ref).max() < TOL
    for a in range(case.dim):
        assert np.array_equal(uu[a], u[a])       # u held fixed
    # the GPU root is a root of the oracle's F
    F = phi - phi0 - dt * ora.phase_rhs(P, phi, u)
    assert np.abs(F).max() < 1e-11


def test_implicit_three_steps_match_oracle(gpu, ora):
    from oracle import implicit
    case, P, phi0, u = setup(ora, (40, 36), seed=12)
    dt = workloads.implicit_dt(case, 8.0)
    say(f"implicit three steps {case.n} dt={dt:.3e}")
    ref = phi0
    for _ in range(3):
        ref, _, _ = implicit.isodi_backward_euler(P, dt, ref, u, tol=1e-12)
    for rtol in (0.0, 1e-6):          # adaptive forcing, fixed forcing
        s, phi, _, info = gpu_step(gpu, case, phi0, u, dt, nsteps=3, krylov_rtol=rtol)
        say(f"  krylov_rtol {rtol}: {info}")
        assert info["newton_total"] >= 3
        assert np.abs(phi - ref).max() < 3 * TOL


@pytest.mark.fullsize
@pytest.mark.parametrize("n", [(256, 256), (128, 128, 128), (256, 256, 256)])
def test_implicit_step_fullsize_residual(gpu, ora, n):
    """At 256^2, 128^3 and the 256^3 of the benchmark the oracle's F at the
    GPU's root must vanish."""
    case, P, phi0, u = setup(ora, n, seed=13)
    dt = workloads.implicit_dt(case, 10.0)
    say(f"implicit full size {n} dt={dt:.3e}")
    s, phi, _, info = gpu_step(gpu, case, phi0, u, dt)
    say(f"  GPU {info}")
    assert info["residual"] <= 1e-12
    F = phi - phi0 - dt * ora.phase_rhs(P, phi, u)
    assert np.abs(F).max() < 1e-11
    assert np.abs(phi - phi0).max() > 1e-3          # the step moved the interface


@pytest.mark.parametrize("n", [(3, 2), (2, 2, 2)])
def test_implicit_uniform_state_smallest_grids(gpu, n):
    """On the smallest grids a uniform phi under a uniform velocity solves
    phi1 - phi0 + (dt gamma / eps) psi'(phi1) = 0: the root of a cubic."""
    case = workloads.implicit_drop(n)
    dt = 0.3 * case.eps / case.gamma
    a = dt * case.gamma / case.eps
    shape = tuple(reversed(n))
    say(f"implicit uniform state {n}")
    for phi0 in (0.3, 0.8):
        roots = np.roots([2 * a, -3 * a, 1 + a, -phi0])
        real = roots[np.abs(roots.imag) < 1e-12].real
        want = real[np.argmin(np.abs(real - phi0))]
        u = [np.full(shape, 0.4 - 0.3 * q) for q in range(len(n))]
        s, phi, _, info = gpu_step(gpu, case, np.full(shape, phi0), u, dt)
        assert np.abs(phi - want).max() < 1e-13


def test_implicit_edge_cases(gpu, ora):
    case, P, phi0, u = setup(ora, (24, 20), seed=14)
    say("implicit edge cases: dt = 0, nsteps = 0")
    s, phi, _, info = gpu_step(gpu, case, phi0, u, 0.0)
    assert np.array_equal(phi, phi0) and info["newton_iters"] == 0 and info["krylov_iters"] == 0
    s, phi, _, info = gpu_step(gpu, case, phi0, u, 1e-3, nsteps=0)
    assert np.array_equal(phi, phi0) and info["newton_total"] == 0
    say("implicit edge cases: Newton cap -> ENOCONV with phi rolled back")
    s = gpu.solver_for_case(case)
    s.set_state(phi0, u)
    with pytest.raises(gpu.TpfError) as e:
        s.implicit_phase_step(workloads.implicit_dt(case, 10.0), 1, newton_maxit=1)
    assert e.value.status == gpu.TPF_ENOCONV
    phi, _, _ = s.get_state()
    assert np.array_equal(phi, phi0)
    say("implicit edge cases: invalid arguments")
    with pytest.raises(gpu.TpfError) as e:
        s.implicit_phase_step(-1e-3)
    assert e.value.status == gpu.TPF_EINVAL
    with pytest.raises(gpu.TpfError) as e:
        s.implicit_phase_step(1e-3, krylov_rtol=1.5)
    assert e.value.status == gpu.TPF_EINVAL
    for kw in (dict(model="SB"), dict(precision="fp32_mixed")):
        t = gpu.solver_for_case(case, **kw)
        with pytest.raises(gpu.TpfError) as e:
            t.implicit_phase_step(1e-3)
        assert e.value.status == gpu.TPF_EINVAL


def test_implicit_then_rk4_step(gpu, ora):
    """The implicit step uses the RK4 stage scratch: a following RK4 step of the
    same context must equal one started from the implicit step's output."""
    case, P, phi0, u = setup(ora, (32, 28), seed=15)
    dt = workloads.implicit_dt(case, 5.0)
    say(f"implicit then RK4 {case.n}")
    s, phi1, u1, _ = gpu_step(gpu, case, phi0, u, dt)
    s.step(1e-4, 1)
    a_phi, a_u, _ = s.get_state()
    t = gpu.solver_for_case(case)
    t.set_state(phi1, u1)
    t.step(1e-4, 1)
    b_phi, b_u, _ = t.get_state()
    assert np.array_equal(a_phi, b_phi)
    for a in range(case.dim):
        assert np.array_equal(a_u[a], b_u[a])
