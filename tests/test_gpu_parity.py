"""GPU (MI355X) parity of the HIP path against the FP64 oracle, through the C ABI.

Every case prints its name before touching the GPU.  FP64 results must
match the oracle to 1e-12 relative (fields scaled by their max magnitude;
velocities by U_ref = max(|u|, dt |beta G p|) because the static-drop
velocity is a small residue of cancelling force and pressure gradient).
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


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


def oparams(ora, case, **kw):
    base = dict(n=case.n, length=case.length, model=ora.MODELS[case.model],
                force=ora.FORCES[case.force], sigma=case.sigma, eps=case.eps, gamma=case.gamma,
                rho1=case.rho1, rho2=case.rho2, visc1=case.visc1, visc2=case.visc2)
    base.update(kw)
    return ora.Params(**base)


def rel(a, b):
    s = np.abs(b).max()
    return np.abs(a - b).max() / (s if s > 0 else 1.0)


def small_case(dim, model="CDI", force="EB", n=None, ratio=10.0, precision="fp64"):
    if dim == 2:
        n = n or (48, 40)
        return workloads.Case(f"small2d_{model}_{force}", n, (0.5, 0.5), (0.3, 0.22), ratio, 1.0,
                              0.02, 0.004, 1.0, 1.0, model, force, precision)
    n = n or (24, 16, 20)
    return workloads.Case(f"small3d_{model}_{force}", n, (0.5, 0.5, 0.5), (0.3, 0.25, 0.22),
                          ratio, 1.0, 0.02, 0.004, 1.0, 1.0, model, force, precision)


def test_init_droplet_matches_oracle(gpu, ora):
    for case in (small_case(2), small_case(3), workloads.oscillating_drop_3d(64, "fp64")):
        say(f"init_droplet {case.name} {case.n}")
        s = gpu.solver_for_case(case)
        s.init_droplet(case.center, case.semi_axes)
        phi, u, _ = s.get_state()
        ref = ora.init_droplet(oparams(ora, case), case.center, case.semi_axes)
        assert np.abs(phi - ref).max() < 1e-14        # tanh of two libms: a few ulp
        assert all(np.abs(x).max() == 0 for x in u)


FIELD_CHECKS = [
    ("NORMAL0", lambda ora, P, phi, u: ora.normals(P, phi)[0][0]),
    ("NORMAL1", lambda ora, P, phi, u: ora.normals(P, phi)[0][1]),
    ("MU", lambda ora, P, phi, u: ora.chem_potential(P, phi)),
    ("KAPPA", lambda ora, P, phi, u: ora.curvature(P, phi)),
    ("CDIFLUX0", lambda ora, P, phi, u: ora.cdi_flux(P, phi)[0]),
    ("CDIFLUX1", lambda ora, P, phi, u: ora.cdi_flux(P, phi)[1]),
    ("MASSFLUX0", lambda ora, P, phi, u: ora.mass_flux(P, phi, u)[0]),
    ("MASSFLUX1", lambda ora, P, phi, u: ora.mass_flux(P, phi, u)[1]),
    ("DPHI", lambda ora, P, phi, u: ora.phase_rhs(P, phi, u)),
    ("FORCE0", lambda ora, P, phi, u: ora.surface_force(P, phi)[0]),
    ("FORCE1", lambda ora, P, phi, u: ora.surface_force(P, phi)[1]),
    ("FSTAR0", lambda ora, P, phi, u: ora.fstar(P, phi, u)[0]),
    ("FSTAR1", lambda ora, P, phi, u: ora.fstar(P, phi, u)[1]),
    ("DIVFSTAR", lambda ora, P, phi, u: ora.divergence(P, ora.fstar(P, phi, u))),
]


def applicable(name, case):
    if name == "MU":
        return case.force == "EB"
    if name == "KAPPA":
        return not (case.model == "CDI" and case.force == "EB")
    if name.startswith("CDIFLUX"):
        return case.model == "CDI"
    return True


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("model,force", [("CDI", "EB"), ("CDI", "CSF"), ("SB", "LCSF"),
                                         ("ISODI", "EB"), ("SB", "CSF"), ("ISODI", "LCSF")])
def test_stage_fields_fp64(gpu, ora, dim, model, force):
    """a1-a5: normals, curvature, mu, CDI flux, mass flux, dphi/dt, surface
    force, f* and D f* at a droplet state with a random velocity field."""
    case = small_case(dim, model, force, ratio=1000.0)
    say(f"stage_fields {case.name} {case.n}")
    P = oparams(ora, case)
    phi = ora.init_droplet(P, case.center, case.semi_axes)
    u = workloads.random_velocity(P.shape, 3, amplitude=0.05)
    s = gpu.solver_for_case(case, poisson_rtol=1e-14)
    s.set_state(phi, u)
    checks = list(FIELD_CHECKS)
    if dim == 3:
        checks += [("NORMAL2", lambda ora, P, phi, u: ora.normals(P, phi)[0][2]),
                   ("MASSFLUX2", lambda ora, P, phi, u: ora.mass_flux(P, phi, u)[2]),
                   ("FSTAR2", lambda ora, P, phi, u: ora.fstar(P, phi, u)[2])]
    for name, fn in checks:
        if not applicable(name, case):
            continue
        g = s.eval_field(name)
        r = fn(ora, P, phi, u)
        e = rel(g, r)
        assert e < TOL64, (name, e)


@pytest.mark.parametrize("model,force", [("CDI", "EB"), ("CDI", "CSF"), ("SB", "EB"), ("ISODI", "LCSF")])
@pytest.mark.parametrize("n", [(24, 16, 20), (70, 12, 40)])
def test_stage_fields_fp64_lds_pass(gpu, ora, model, force, n):
    """The 3D LDS passes (the FP32 default; forced here on FP64 contexts,
    TPF_STAGE_LDS=1): normals, mu or kappa, CDI and mass fluxes from the
    fused cell/face pass, dphi/dt and f* from the phase/momentum pass, to the
    FP64 bound: one z chunk with a ragged x tile, and two x tiles with two z
    chunks (32 + 8 planes)."""
    import os
    case = small_case(3, model, force, n=n, ratio=1000.0)
    say(f"stage_fields LDS pass {case.name} {case.n}")
    P = oparams(ora, case)
    phi = ora.init_droplet(P, case.center, case.semi_axes)
    u = workloads.random_velocity(P.shape, 4, amplitude=0.05)
    os.environ["TPF_STAGE_LDS"] = "1"
    try:
        s = gpu.solver_for_case(case, poisson_rtol=1e-14)
    finally:
        del os.environ["TPF_STAGE_LDS"]
    s.set_state(phi, u)
    checks = [("DPHI", lambda: ora.phase_rhs(P, phi, u))]
    checks += [(f"FSTAR{a}", (lambda a=a: ora.fstar(P, phi, u)[a])) for a in range(3)]
    checks += [(f"NORMAL{a}", (lambda a=a: ora.normals(P, phi)[0][a])) for a in range(3)]
    checks += [(f"MASSFLUX{a}", (lambda a=a: ora.mass_flux(P, phi, u)[a])) for a in range(3)]
    if model == "CDI":
        checks += [(f"CDIFLUX{a}", (lambda a=a: ora.cdi_flux(P, phi)[a])) for a in range(3)]
    if force == "EB":
        checks += [("MU", lambda: ora.chem_potential(P, phi))]
    else:
        checks += [("KAPPA", lambda: ora.curvature(P, phi))]
    for name, fn in checks:
        e = rel(s.eval_field(name), fn())
        assert e < TOL64, (name, e)


@pytest.mark.parametrize("dim", [2, 3])
def test_pressure_and_projection_fp64(gpu, ora, dim):
    """a6-a7: projection pressure (zero mean) and projected du/dt."""
    case = small_case(dim, "CDI", "EB", ratio=1000.0)
    say(f"pressure {case.name} {case.n}")
    P = oparams(ora, case)
    phi = ora.init_droplet(P, case.center, case.semi_axes)
    u = workloads.random_velocity(P.shape, 5, amplitude=0.05)
    s = gpu.solver_for_case(case, poisson_rtol=1e-14)
    s.set_state(phi, u)
    d_o, du_o, p_o = ora.stage(P, phi, u)
    p_g = s.eval_field("PRESSURE")
    edu = [rel(s.eval_field(f"DU{a}"), du_o[a]) for a in range(dim)]
    say(f"  p rel {rel(p_g, p_o):.2e}  du rel {max(edu):.2e}")
    # density ratio 1000 (measured: p 3e-15, du/dt 1.3e-13)
    assert rel(p_g, p_o) < 1e-12
    assert abs(p_g.mean()) < 1e-12 * np.abs(p_o).max()
    for a in range(dim):
        assert edu[a] < 1e-12, a
    assert rel(s.eval_field("DPHI"), d_o) < TOL64


@pytest.mark.parametrize("dim,n", [(2, (64, 64)), (2, (40, 24)), (3, (16, 16, 16)), (3, (24, 20, 12))])
def test_poisson_solve_fp64(gpu, ora, dim, n):
    """a6: multigrid-PCG solution equals the oracle's converged solution of
    D(beta G x) = b - mean(b) at density ratio 1000 (random b)."""
    case = small_case(dim, n=n, ratio=1000.0)
    say(f"poisson {case.name} {n}")
    P = oparams(ora, case)
    phi = ora.init_droplet(P, case.center, case.semi_axes)
    s = gpu.solver_for_case(case, poisson_rtol=1e-14, poisson_maxit=1000)
    s.set_state(phi, [np.zeros(P.shape)] * dim)
    b = workloads.noise_field(P.shape, 17)
    x_g, it, rr = s.poisson_solve(b)
    x_o, _, _ = ora.poisson_solve(P, phi, b)
    say(f"  iterations {it} relres {rr:.2e}  x rel {rel(x_g, x_o):.2e}")
    assert rr <= 1e-14
    assert rel(x_g, x_o) < 1e-12
    res = ora.poisson_apply(P, phi, x_g) - (b - b.mean())
    assert np.abs(res).max() < 1e-12 * np.abs(b).max()


def test_static_drop_64_fp64_200_steps(gpu, ora):
    """The 64^2 static drop (CDI + energy-based force, FP64, 200 steps)."""
    case = workloads.static_drop_64()
    say(f"step parity {case.name} {case.n} x {case.steps}")
    P = oparams(ora, case)
    phi0 = ora.init_droplet(P, case.center, case.semi_axes)
    zero = [np.zeros(P.shape)] * 2
    dt = case.dt()
    s = gpu.solver_for_case(case, poisson_rtol=1e-14)
    s.set_state(phi0, zero)
    s.step(dt, case.steps)
    phi_g, u_g, p_g = s.get_state(with_pressure=True)
    phi_o, u_o, pw = ora.step(P, dt, case.steps, phi0, zero)
    p_o = ora.pressure(P, phi_o, u_o, pw)
    d_o, du_o, _ = ora.stage(P, phi_o, u_o, pw)
    uref = max(max(np.abs(x).max() for x in u_o), dt * max(np.abs(x).max() for x in du_o))
    ephi = np.abs(phi_g - phi_o).max()
    eu = max(np.abs(u_g[a] - u_o[a]).max() for a in range(2)) / uref
    ep = rel(p_g, p_o)
    say(f"  |dphi| {ephi:.2e}  |du|/Uref {eu:.2e}  |dp|/|p| {ep:.2e}")
    assert ephi < TOL64 and eu < TOL64 and ep < TOL64
    dg = s.diagnostics()
    do = ora.diagnostics(P, phi_o, u_o, p_o)
    assert abs(dg["mass"] - dg["mass0"]) / dg["mass0"] < 1e-13      # CDI conserves mass
    for k in ("mass", "se", "dp"):
        assert abs(dg[k] - do[k]) <= 1e-12 * abs(do[k]), k
    assert abs(dg["ke"] - do["ke"]) <= 1e-9 * do["ke"] + 1e-30
    assert abs(dg["ca_inf"] - do["ca_inf"]) <= 1e-9 * do["ca_inf"] + 1e-30


@pytest.mark.parametrize("model,force", [("CDI", "CSF"), ("SB", "EB"), ("ISODI", "LCSF"),
                                         ("SB", "CSF"), ("CDI", "LCSF"), ("ISODI", "EB")])
def test_ratio1000_steps_fp64(gpu, ora, model, force):
    """Static drop at density ratio 1000, viscosity ratio 100 (48^2, 10 steps)."""
    case = workloads.static_drop_ratio(48, 0.75, model, force)
    say(f"step parity {case.name}")
    P = oparams(ora, case)
    phi0 = ora.init_droplet(P, case.center, case.semi_axes)
    zero = [np.zeros(P.shape)] * 2
    dt = case.dt()
    steps = 10
    s = gpu.solver_for_case(case, poisson_rtol=1e-14, poisson_maxit=2000)
    s.set_state(phi0, zero)
    s.step(dt, steps)
    phi_g, u_g, _ = s.get_state()
    phi_o, u_o, pw = ora.step(P, dt, steps, phi0, zero)
    _, du_o, _ = ora.stage(P, phi_o, u_o, pw)
    uref = max(max(np.abs(x).max() for x in u_o), dt * max(np.abs(x).max() for x in du_o))
    ephi = np.abs(phi_g - phi_o).max()
    eu = max(np.abs(u_g[a] - u_o[a]).max() for a in range(2)) / uref
    say(f"  |dphi| {ephi:.2e}  |du|/Uref {eu:.2e}")
    # density ratio 1000: the projection's condition number (~5e5 here) turns
    # the 1e-14 solver residual into ~3e-12 in u (measured bound)
    assert ephi < TOL64 and eu < 1e-11


def test_oscillating_drop_3d_fp64(gpu, ora):
    """3D ellipsoid, density ratio 10 (32^3, 4 steps, CDI + EB)."""
    case = workloads.oscillating_drop_3d(32, "fp64")
    say(f"step parity {case.name}")
    P = oparams(ora, case)
    phi0 = ora.init_droplet(P, case.center, case.semi_axes)
    zero = [np.zeros(P.shape)] * 3
    dt = case.dt()
    s = gpu.solver_for_case(case, poisson_rtol=1e-14)
    s.set_state(phi0, zero)
    s.step(dt, 4)
    phi_g, u_g, _ = s.get_state()
    phi_o, u_o, pw = ora.step(P, dt, 4, phi0, zero)
    _, du_o, _ = ora.stage(P, phi_o, u_o, pw)
    uref = max(max(np.abs(x).max() for x in u_o), dt * max(np.abs(x).max() for x in du_o))
    ephi = np.abs(phi_g - phi_o).max()
    eu = max(np.abs(u_g[a] - u_o[a]).max() for a in range(3)) / uref
    say(f"  |dphi| {ephi:.2e}  |du|/Uref {eu:.2e}")
    assert ephi < TOL64 and eu < TOL64


def test_mixed_precision_error_statement(gpu, ora):
    """a9: FP32 state/stencils with FP64 pressure against the FP64 oracle
    (64^2 ellipse, ratio 10, 20 steps); the stated bounds."""
    case = workloads.Case("mixed64", (64, 64), (0.5, 0.5), (0.3, 0.22), 1.0, 0.1, 2e-3, 2e-4, 1.0,
                          1.0, "CDI", "EB", "fp32_mixed")
    say(f"mixed precision {case.name}")
    P = oparams(ora, case)
    phi0 = ora.init_droplet(P, case.center, case.semi_axes)
    zero = [np.zeros(P.shape)] * 2
    dt = case.dt()
    s = gpu.solver_for_case(case)
    s.set_state(phi0, zero)
    s.step(dt, 20)
    phi_g, u_g, p_g = s.get_state(with_pressure=True)
    phi0_32 = phi0.astype(np.float32).astype(np.float64)
    phi_o, u_o, pw = ora.step(P, dt, 20, phi0_32, zero)
    p_o = ora.pressure(P, phi_o, u_o, pw)
    umax = max(np.abs(x).max() for x in u_o)
    ephi = np.abs(phi_g - phi_o).max()
    eu = max(np.abs(u_g[a] - u_o[a]).max() for a in range(2)) / umax
    ep = rel(p_g, p_o)
    dg = s.diagnostics()
    do = ora.diagnostics(P, phi_o, u_o, p_o)
    edp = abs(dg["dp"] - do["dp"]) / abs(do["dp"])
    say(f"  |dphi| {ephi:.2e} |du|/|u| {eu:.2e} |dp|/|p| {ep:.2e} dp err {edp:.2e}")
    assert ephi < 1e-5 and eu < 1e-2 and ep < 1e-4 and edp < 1e-4


def test_nonconvergence_rolls_back(gpu, ora):
    """poisson_maxit = 1 cannot converge: TPF_ENOCONV and the state is kept."""
    case = small_case(2)
    say("failure: non-convergence")
    P = oparams(ora, case)
    phi0 = ora.init_droplet(P, case.center, case.semi_axes)
    s = gpu.solver_for_case(case, poisson_maxit=1, poisson_rtol=1e-14)
    s.set_state(phi0, [np.zeros(P.shape)] * 2)
    with pytest.raises(gpu.TpfError) as e:
        s.step(1e-4, 1)
    assert e.value.status == gpu.TPF_ENOCONV
    phi, u, _ = s.get_state()
    assert np.array_equal(phi, phi0) and all(np.abs(x).max() == 0 for x in u)


def test_nonfinite_rolls_back(gpu, ora):
    """A NaN in the state gives TPF_ENONFINITE (host-forced), state kept."""
    case = small_case(2)
    say("failure: non-finite")
    P = oparams(ora, case)
    phi0 = ora.init_droplet(P, case.center, case.semi_axes)
    phi0[3, 5] = np.nan
    s = gpu.solver_for_case(case, poisson_maxit=50)
    s.set_state(phi0, [np.zeros(P.shape)] * 2)
    with pytest.raises(gpu.TpfError) as e:
        s.step(1e-4, 1)
    assert e.value.status in (gpu.TPF_ENONFINITE, gpu.TPF_ENOCONV)
    phi, _, _ = s.get_state()
    assert np.isnan(phi[3, 5])


def test_determinism_bitwise(gpu, ora):
    """Two runs of the same steps give bit-identical states."""
    case = small_case(3, ratio=10.0)
    say("determinism")
    outs = []
    for _ in range(2):
        s = gpu.solver_for_case(case)
        s.init_droplet(case.center, case.semi_axes)
        s.step(case.dt(), 3)
        outs.append(s.get_state(with_pressure=True))
    assert np.array_equal(outs[0][0], outs[1][0])
    for a in range(3):
        assert np.array_equal(outs[0][1][a], outs[1][1][a])
    assert np.array_equal(outs[0][2], outs[1][2])
