"""GPU tests of free-slip walls in the batched form, through the C ABI.

A walled axis is closed by free-slip walls at both ends (the box of Sec. 3.1,
the top and bottom of Sec. 3.2).  Every walled case is compared with the
FP64 oracle run on that case alone with the same walls; the oracle's wall
rules are pinned on the CPU against the mirror-doubled periodic box.  At
sizes beyond the oracle, the walled GPU case is compared with the periodic
GPU case of twice the size that holds its mirror image.
"""
import dataclasses
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


def oparams(ora, case, walls):
    return ora.Params(n=case.n, length=case.length, model=ora.MODELS[case.model],
                      force=ora.FORCES[case.force], sigma=case.sigma, eps=case.eps, gamma=case.gamma,
                      rho1=case.rho1, rho2=case.rho2, visc1=case.visc1, visc2=case.visc2, walls=walls)


def shut_walls(u, walls):
    """Copies of the 2D face velocities with 0 on the wall faces."""
    u = [x.copy() for x in u]
    if walls & 1:
        u[0][:, 0] = 0.0
    if walls & 2:
        u[1][0, :] = 0.0
    return u


def wall_cases():
    """The nine model x force pairs, each with walls on x, y or both, drops
    that reach into the wall region (the interface layer touches the wall),
    box edges 1, 2 pi and 2, non-square grids, density ratios 1 to 1000; plus
    one periodic case sharing the launch."""
    C = workloads.Case
    L = 2.0 * np.pi
    return [
        (C("w_cdi_eb", (32, 24), (0.3, 0.3), (0.25, 0.2), 1.0, 0.1, 2e-3, 2e-4, 1.0, 1.0, "CDI", "EB", "fp64"), 3),
        (C("w_cdi_csf", (24, 24), (0.5, 0.32), (0.3, 0.25), 240.0, 0.24, 0.1, 0.001, 1.0, 0.75, "CDI", "CSF",
           "fp64"), 2),
        (C("w_cdi_lcsf", (32, 32), (0.3 * L, 0.5 * L), (0.25 * L, 0.2 * L), 1.0, 1.0, 0.01, 0.01, 1.0, 1.0,
           "CDI", "LCSF", "fp64", length=L), 1),
        (C("w_sb_eb", (40, 20), (0.6, 0.35), (0.5, 0.3), 2.0, 1.0, 0.02, 0.01, 0.8, 0.9, "SB", "EB", "fp64",
           length=2.0), 3),
        (C("w_sb_csf", (20, 28), (0.5, 0.7), (0.3, 0.25), 10.0, 1.0, 0.02, 0.004, 1.5, 1.0, "SB", "CSF", "fp64"), 2),
        (C("w_sb_lcsf", (28, 28), (0.32, 0.5), (0.3, 0.22), 1.0, 0.01, 0.01, 1e-4, 1.0, 0.8, "SB", "LCSF", "fp64"),
         1),
        (C("w_isodi_eb", (24, 32), (0.5, 0.6), (0.3, 0.3), 1.0, 0.001, 0.01, 1e-5, 1.0, 0.75, "ISODI", "EB",
           "fp64"), 3),
        (C("w_isodi_csf", (32, 32), (0.5 * L, 0.35 * L), (0.3 * L, 0.22 * L), 3.0, 1.0, 0.03, 0.01, 2.0, 1.0,
           "ISODI", "CSF", "fp64", length=L), 2),
        (C("w_isodi_lcsf", (36, 20), (0.4, 0.3), (0.3, 0.2), 1.0, 0.5, 0.02, 0.01, 0.7, 1.0, "ISODI", "LCSF",
           "fp64"), 3),
        (C("w_periodic", (24, 24), (0.5, 0.5), (0.3, 0.25), 10.0, 1.0, 0.02, 0.004, 1.5, 1.0, "SB", "CSF", "fp64"),
         0),
    ]


def initial_states(ora, cases, seed0):
    init, dts = [], []
    for q, (c, w) in enumerate(cases):
        P = oparams(ora, c, w)
        phi0 = ora.init_droplet(P, c.center, c.semi_axes)
        u0 = shut_walls(workloads.random_velocity(P.shape, seed0 + q, 0.01 * c.length), w)
        init.append((phi0, u0))
        dts.append(c.dt(umax0=max(np.abs(x).max() for x in u0)))
    return init, np.array(dts)


def errors(ora, P, dt, steps, init, got):
    phi_o, u_o, p_o = ora.step(P, dt, steps, *init)
    _, du_o, _ = ora.stage(P, phi_o, u_o, p_o)
    phi_g, u_g, p_g = got
    uref = max(max(np.abs(x).max() for x in u_o), dt * max(np.abs(x).max() for x in du_o))
    ephi = np.abs(phi_g - phi_o).max()
    eu = max(np.abs(u_g[a] - u_o[a]).max() for a in range(2)) / uref
    ep = np.abs(p_g - p_o).max() / np.abs(p_o).max()
    return ephi, eu, ep


def test_batch_walls_init_droplet(gpu, ora):
    """Across a walled axis the drop has no periodic image."""
    cases = wall_cases()
    say(f"walled init_droplet, {len(cases)} cases")
    b = gpu.Batch([gpu.params_for_case(c, walls=w) for c, w in cases])
    for q, (c, w) in enumerate(cases):
        b.init_droplet(q, c.center, c.semi_axes)
    for q, (c, w) in enumerate(cases):
        phi, _, _ = b.get_state(q)
        ref = ora.init_droplet(oparams(ora, c, w), c.center, c.semi_axes)
        assert np.abs(phi - ref).max() < 1e-14, c.name


def test_batch_walls_all_pairs_match_oracle(gpu, ora):
    """All nine pairs with walls (and a periodic case in the same launch),
    FP64, 4 steps from a seeded velocity that is 0 on the wall faces: every
    case against the oracle to the periodic cases' bounds."""
    cases = wall_cases()
    steps = 4
    say(f"walled FP64 parity, {len(cases)} cases x {steps} steps")
    b = gpu.Batch([gpu.params_for_case(c, walls=w, poisson_rtol=1e-14, poisson_maxit=4000) for c, w in cases])
    init, dts = initial_states(ora, cases, 40)
    for q in range(len(cases)):
        b.set_state(q, *init[q])
    b.step(dts, steps)
    st, nst, _ = b.status()
    assert (st == 0).all() and (nst == steps).all()
    for q, (c, w) in enumerate(cases):
        got = b.get_state(q, with_pressure=True)
        ephi, eu, ep = errors(ora, oparams(ora, c, w), dts[q], steps, init[q], got)
        say(f"  {c.name} walls {w}: |dphi| {ephi:.2e} |du|/Uref {eu:.2e} |dp|/|p| {ep:.2e}")
        assert ephi < 1e-12 and eu < 1e-11 and ep < 1e-12, c.name
        for a in range(2):
            if (w >> a) & 1:
                face = got[1][a][:, 0] if a == 0 else got[1][a][0, :]
                assert np.all(face == 0.0), (c.name, a)


def test_batch_walls_mixed_error_statement(gpu, ora):
    """FP32-mixed walled cases against the FP64 oracle from the FP32-rounded
    initial state: the mixed-precision bounds of the periodic cases."""
    cases = [(dataclasses.replace(c, precision="fp32_mixed"), w) for c, w in wall_cases()[:6]]
    steps = 5
    say(f"walled FP32-mixed error statement, {len(cases)} cases x {steps} steps")
    b = gpu.Batch([gpu.params_for_case(c, walls=w) for c, w in cases])
    init, dts = initial_states(ora, cases, 60)
    init = [(phi.astype(np.float32).astype(np.float64), [x.astype(np.float32).astype(np.float64) for x in u])
            for phi, u in init]
    for q in range(len(cases)):
        b.set_state(q, *init[q])
    b.step(dts, steps)
    st, _, _ = b.status()
    assert (st == 0).all()
    for q, (c, w) in enumerate(cases):
        ephi, eu, _ = errors(ora, oparams(ora, c, w), dts[q], steps, init[q], b.get_state(q, with_pressure=True))
        say(f"  {c.name} walls {w}: |dphi| {ephi:.2e} |du|/Uref {eu:.2e}")
        assert ephi < 1e-5 and eu < 1e-2, c.name


def test_batch_walls_diagnostics_match_oracle(gpu, ora):
    """Diagnostics of a walled state (wall faces count as 0) against the
    oracle's diagnostics of the same state."""
    cases = wall_cases()[:5]
    say("walled diagnostics")
    b = gpu.Batch([gpu.params_for_case(c, walls=w, poisson_rtol=1e-14) for c, w in cases])
    init, dts = initial_states(ora, cases, 80)
    for q in range(len(cases)):
        b.set_state(q, *init[q])
    b.step(dts, 2)
    dg = b.diagnostics()
    for q, (c, w) in enumerate(cases):
        phi, u, p = b.get_state(q, with_pressure=True)
        do = ora.diagnostics(oparams(ora, c, w), phi, u, p)
        for k in ("mass", "se", "ke", "umax", "phi_min", "phi_max", "div_max", "dp"):
            tol = 1e-12 * max(abs(do[k]), 1e-300) + (1e-15 if k == "div_max" else 0.0)
            assert abs(dg[q][k] - do[k]) <= tol, (c.name, k, dg[q][k], do[k])


def test_batch_wall_faces_are_read_as_zero(gpu, ora):
    """Whatever the velocity array holds on the wall faces is read as 0 and
    left as it was: a run from junk there equals, bit for bit, the run from
    zeros everywhere else."""
    cases = [wall_cases()[0], wall_cases()[4]]
    say("wall faces read as 0")
    params = [gpu.params_for_case(c, walls=w) for c, w in cases]
    init, dts = initial_states(ora, cases, 90)
    runs = []
    for junk in (0.0, 0.37):
        b = gpu.Batch(params)
        for q, (c, w) in enumerate(cases):
            phi0, u0 = init[q]
            u = [x.copy() for x in u0]
            if w & 1:
                u[0][:, 0] = junk
            if w & 2:
                u[1][0, :] = junk
            b.set_state(q, phi0, u)
        b.step(dts, 3)
        runs.append([b.get_state(q, with_pressure=True) for q in range(len(cases))])
        b.close()
    for q, (c, w) in enumerate(cases):
        (f0, u0, p0), (f1, u1, p1) = runs[0][q], runs[1][q]
        assert np.array_equal(f0, f1) and np.array_equal(p0, p1), c.name
        for a in range(2):
            if (w >> a) & 1:
                sl = (slice(None), 0) if a == 0 else (0, slice(None))
                assert np.all(u1[a][sl] == 0.37) and np.all(u0[a][sl] == 0.0)
                u1[a][sl] = 0.0
            assert np.array_equal(u0[a], u1[a]), (c.name, a)


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_batch_walls_equal_doubled_periodic_box(gpu, precision):
    """At a size beyond the oracle: a 96 x 64 box walled on both axes evolves
    like the lower-left quarter of the 192 x 128 periodic box that holds its
    mirror image (both on the GPU, in one batch), 10 steps, every pair."""
    C = workloads.Case
    n = (96, 64)
    cases = []
    for model in ("CDI", "SB", "ISODI"):
        for force in ("EB", "CSF", "LCSF"):
            cases.append(C(f"{model}_{force}", n, (0.62, 0.45), (0.3, 0.24), 10.0, 1.0, 0.02, 0.004, 1.0, 1.0,
                           model, force, precision, length=1.5))
    say(f"walled vs doubled periodic, {precision}, {len(cases)} pairs at {n}")
    rtol = 1e-13 if precision == "fp64" else 1e-8
    params = []
    for c in cases:
        params.append(gpu.params_for_case(c, walls=3, poisson_rtol=rtol, poisson_maxit=2000))
        d = dataclasses.replace(c, n=(2 * n[0], 2 * n[1]), length=2 * c.length)
        params.append(gpu.params_for_case(d, walls=0, poisson_rtol=rtol, poisson_maxit=2000))
    b = gpu.Batch(params)
    dts = []
    for q, c in enumerate(cases):
        b.init_droplet(2 * q, c.center, c.semi_axes)
        phi, _, _ = b.get_state(2 * q)
        big = np.concatenate([phi, phi[:, ::-1]], axis=1)
        big = np.concatenate([big, big[::-1, :]], axis=0)
        b.set_state(2 * q + 1, big, [np.zeros_like(big)] * 2)
        dts += [c.dt()] * 2
    dts = np.array(dts)
    b.step(dts, 10)
    st, _, _ = b.status()
    assert (st == 0).all()
    for q, c in enumerate(cases):
        fw, uw, _ = b.get_state(2 * q)
        fd, ud, _ = b.get_state(2 * q + 1)
        us = max(np.abs(x).max() for x in ud)
        ephi = np.abs(fw - fd[: n[1], : n[0]]).max()
        eu = max(np.abs(uw[a] - ud[a][: n[1], : n[0]]).max() for a in range(2)) / us
        # the doubled box keeps the mirror symmetry (odd normal velocity about the wall faces)
        ux_mirror = -np.roll(ud[0][:, ::-1], 1, axis=1)
        esym = np.abs(ud[0] - ux_mirror).max() / us
        say(f"  {c.name}: |dphi| {ephi:.2e} |du|/|u| {eu:.2e} mirror {esym:.2e}")
        bound = (1e-12, 1e-11) if precision == "fp64" else (1e-6, 2e-4)
        assert ephi < bound[0] and eu < bound[1] and esym < bound[1], c.name


# ------------------------------------------------------------ single-case contexts


def shut_walls3(u, walls):
    """Copies of the 3D face velocities with 0 on the wall faces."""
    u = [x.copy() for x in u]
    for a in range(3):
        if (walls >> a) & 1:
            idx = [slice(None)] * 3
            idx[2 - a] = 0
            u[a][tuple(idx)] = 0.0
    return u


def single_cases():
    """Walled single cases: 2D (FP64, the plain solver kernels) and 3D (the
    z-marching fine level, stored-coefficient and fused coarse levels, the LDS
    tail), every model, walls on one to three axes."""
    C = workloads.Case
    return [
        (C("s2_cdi_eb", (48, 40), (0.3, 0.35), (0.25, 0.2), 10.0, 1.0, 0.02, 0.004, 1.0, 1.0, "CDI", "EB", "fp64"), 3),
        (C("s2_sb_lcsf", (40, 48), (0.55, 0.3), (0.3, 0.25), 1.0, 0.01, 0.01, 1e-4, 1.0, 0.8, "SB", "LCSF", "fp64"), 2),
        (C("s3_isodi_csf", (24, 20, 16), (0.35, 0.45, 0.3), (0.3, 0.25, 0.22), 10.0, 1.0, 0.02, 0.004, 1.2, 1.0,
           "ISODI", "CSF", "fp64"), 5),
        (C("s3_cdi_eb", (16, 16, 16), (0.4, 0.5, 0.35), (0.3, 0.25, 0.25), 10.0, 1.0, 0.02, 0.002, 1.0, 0.75,
           "CDI", "EB", "fp64"), 7),
    ]


@pytest.mark.parametrize("k", range(4))
def test_single_case_walls_match_oracle(gpu, ora, k):
    """A single-case context with walls against the walled oracle, FP64,
    3 steps from a seeded velocity that is 0 on the wall faces."""
    c, w = single_cases()[k]
    steps = 3
    say(f"single-case walled parity {c.name} walls {w}")
    P = oparams(ora, c, w)
    phi0 = ora.init_droplet(P, c.center, c.semi_axes)
    u0 = workloads.random_velocity(P.shape, 70 + k, 0.01)
    u0 = shut_walls(u0, w) if c.dim == 2 else shut_walls3(u0, w)
    dt = c.dt(umax0=max(np.abs(x).max() for x in u0))
    s = gpu.solver_for_case(c, walls=w, poisson_rtol=1e-14, poisson_maxit=2000)
    s.init_droplet(c.center, c.semi_axes)
    phi_i, _, _ = s.get_state()
    assert np.abs(phi_i - phi0).max() < 1e-14
    s.set_state(phi0, u0)
    s.step(dt, steps)
    # a single-case context reports the projection pressure of its current
    # state (a stage evaluation there), not the last stage's
    got = s.get_state(with_pressure=True)
    phi_o, u_o, p_last = ora.step(P, dt, steps, phi0, u0)
    _, du_o, p_o = ora.stage(P, phi_o, u_o, p_last)
    uref = max(max(np.abs(x).max() for x in u_o), dt * max(np.abs(x).max() for x in du_o))
    ephi = np.abs(got[0] - phi_o).max()
    eu = max(np.abs(got[1][a] - u_o[a]).max() for a in range(c.dim)) / uref
    ep = np.abs(got[2] - p_o).max() / np.abs(p_o).max()
    say(f"  |dphi| {ephi:.2e} |du|/Uref {eu:.2e} |dp|/|p| {ep:.2e}")
    assert ephi < 1e-12 and eu < 1e-11 and ep < 1e-12
    d = s.diagnostics()
    do = ora.diagnostics(P, got[0], got[1], got[2])
    for key in ("mass", "se", "ke", "umax", "div_max"):
        assert abs(d[key] - do[key]) <= 1e-12 * max(abs(do[key]), 1e-300) + (1e-15 if key == "div_max" else 0.0), key


def test_single_case_walls_mixed_error_statement(gpu, ora):
    """FP32-mixed 3D walled case (24 x 20 x 16, walls on x and z) against the
    FP64 oracle from the FP32-rounded state: the mixed-precision bounds."""
    c, w = single_cases()[2]
    c = dataclasses.replace(c, precision="fp32_mixed")
    say(f"single-case walled FP32-mixed {c.name}")
    P = oparams(ora, c, w)
    phi0 = ora.init_droplet(P, c.center, c.semi_axes).astype(np.float32).astype(np.float64)
    u0 = [x.astype(np.float32).astype(np.float64) for x in shut_walls3(workloads.random_velocity(P.shape, 77, 0.01), w)]
    dt = c.dt(umax0=max(np.abs(x).max() for x in u0))
    s = gpu.solver_for_case(c, walls=w)
    s.set_state(phi0, u0)
    s.step(dt, 4)
    phi_g, u_g, _ = s.get_state()
    phi_o, u_o, _ = ora.step(P, dt, 4, phi0, u0)
    us = max(np.abs(x).max() for x in u_o)
    ephi = np.abs(phi_g - phi_o).max()
    eu = max(np.abs(u_g[a] - u_o[a]).max() for a in range(3)) / us
    say(f"  |dphi| {ephi:.2e} |du|/|u| {eu:.2e}")
    assert ephi < 1e-5 and eu < 1e-4


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_single_case_walls_equal_doubled_periodic_box(gpu, precision):
    """Beyond the oracle: a 64^3 box walled on all axes evolves like one octant
    of the 128^3 periodic box holding its mirror images (both single-case
    contexts on the GPU), 5 steps: the z-marching kernels, the coarse levels
    and the tail with wall faces."""
    C = workloads.Case
    n = 64
    c = C("box", (n, n, n), (0.4, 0.45, 0.55), (0.3, 0.25, 0.22), 10.0, 1.0, 0.02, 0.002, 1.0, 0.75, "CDI", "EB",
          precision)
    d = dataclasses.replace(c, n=(2 * n,) * 3, length=2.0)
    say(f"single-case walled 64^3 vs doubled periodic 128^3, {precision}")
    rtol = 1e-13 if precision == "fp64" else 1e-9
    sw = gpu.solver_for_case(c, walls=7, poisson_rtol=rtol)
    sw.init_droplet(c.center, c.semi_axes)
    phi, _, _ = sw.get_state()
    big = phi
    for ax in range(3):
        big = np.concatenate([big, np.flip(big, ax)], ax)
    sp = gpu.solver_for_case(d, poisson_rtol=rtol)
    sp.set_state(big, [np.zeros_like(big)] * 3)
    dt = c.dt()
    sw.step(dt, 5)
    sp.step(dt, 5)
    fw, uw, _ = sw.get_state()
    fp, up, _ = sp.get_state()
    us = max(np.abs(x).max() for x in up)
    ephi = np.abs(fw - fp[:n, :n, :n]).max()
    eu = max(np.abs(uw[a] - up[a][:n, :n, :n]).max() for a in range(3)) / us
    say(f"  |dphi| {ephi:.2e} |du|/|u| {eu:.2e}")
    bound = (1e-12, 1e-11) if precision == "fp64" else (2e-6, 3e-4)
    assert ephi < bound[0] and eu < bound[1]


def test_single_case_walls_match_batch(gpu):
    """The same walled 2D case in a single-case context and in a batch
    (different kernels and solvers), FP64, 4 steps."""
    c, w = single_cases()[0]
    say("single-case vs batch, walled")
    s = gpu.solver_for_case(c, walls=w, poisson_rtol=1e-14)
    s.init_droplet(c.center, c.semi_axes)
    b = gpu.Batch([gpu.params_for_case(c, walls=w, poisson_rtol=1e-14)])
    b.init_droplet(0, c.center, c.semi_axes)
    dt = c.dt()
    s.step(dt, 4)
    b.step(np.array([dt]), 4)
    fs, us_, _ = s.get_state()
    fb, ub, _ = b.get_state(0)
    um = max(np.abs(x).max() for x in us_)
    ephi = np.abs(fs - fb).max()
    eu = max(np.abs(us_[a] - ub[a]).max() for a in range(2)) / um
    say(f"  |dphi| {ephi:.2e} |du|/|u| {eu:.2e}")
    assert ephi < 1e-12 and eu < 1e-10
