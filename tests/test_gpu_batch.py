"""GPU tests of the batched persistent form (tpf_batch_*), through the C ABI.

Every case of a batch is compared with the FP64 oracle run on that case
alone; cases of different size, model, force, density ratio and time step
share one launch per step.
"""
import os
import sys
import tempfile

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


def oparams(ora, case, **kw):
    base = dict(n=case.n, length=case.length, model=ora.MODELS[case.model],
                force=ora.FORCES[case.force], sigma=case.sigma, eps=case.eps, gamma=case.gamma,
                rho1=case.rho1, rho2=case.rho2, visc1=case.visc1, visc2=case.visc2)
    base.update(kw)
    return ora.Params(**base)


def mixed_cases(precision):
    C = workloads.Case
    return [
        C("b32_cdi_eb", (32, 32), (0.5, 0.5), (0.25, 0.25), 1.0, 0.1, 2e-3, 2e-4, 1.0, 1.0,
          "CDI", "EB", precision),
        C("b48_sb_csf", (48, 48), (0.5, 0.5), (0.3, 0.22), 240.0, 0.24, 0.1, 0.001, 1.0, 0.75,
          "SB", "CSF", precision),
        C("b40x24_isodi_lcsf", (40, 24), (0.5, 0.3), (0.2, 0.15), 1.0, 0.5, 0.02, 0.01, 0.7, 1.0,
          "ISODI", "LCSF", precision),
        C("b16_cdi_lcsf", (16, 16), (0.45, 0.5), (0.3, 0.25), 1.0, 0.01, 0.01, 1e-4, 1.3, 0.9,
          "CDI", "LCSF", precision),
        C("b36_cdi_eb", (36, 36), (0.5, 0.55), (0.28, 0.2), 10.0, 1.0, 0.05, 0.005, 2.0, 0.6,
          "CDI", "EB", precision),
        C("b64_sb_eb", (64, 64), (0.5, 0.5), (0.25, 0.25), 1.0, 0.1, 2e-3, 2e-4, 1.0, 1.0,
          "SB", "EB", precision),
    ]


def run_oracle(ora, case, dt, steps, phi0):
    P = oparams(ora, case)
    zero = [np.zeros(P.shape)] * 2
    phi, u, pw = ora.step(P, dt, steps, phi0, zero)
    _, du, _ = ora.stage(P, phi, u, pw)
    return P, phi, u, pw, du


def uref_of(u, du, dt):
    return max(max(np.abs(x).max() for x in u), dt * max(np.abs(x).max() for x in du))


def test_batch_init_droplet(gpu, ora):
    cases = mixed_cases("fp64")
    say(f"batch init_droplet, {len(cases)} cases")
    b = gpu.Batch([gpu.params_for_case(c) for c in cases])
    for q, c in enumerate(cases):
        b.init_droplet(q, c.center, c.semi_axes)
    for q, c in enumerate(cases):
        phi, u, _ = b.get_state(q)
        ref = ora.init_droplet(oparams(ora, c), c.center, c.semi_axes)
        assert np.abs(phi - ref).max() < 1e-14, c.name
        assert all(np.abs(x).max() == 0 for x in u)


def test_batch_fp64_matches_oracle(gpu, ora):
    """Six cases of different grids, models, forces, ratios and dt: FP64,
    3 steps, every case against the oracle to the single-case bounds."""
    cases = mixed_cases("fp64")
    steps = 3
    say(f"batch FP64 parity, {len(cases)} cases x {steps} steps")
    params = [gpu.params_for_case(c, poisson_rtol=1e-14, poisson_maxit=2000) for c in cases]
    b = gpu.Batch(params)
    dts = np.array([c.dt() for c in cases])
    phi0s = []
    for q, c in enumerate(cases):
        phi0 = ora.init_droplet(oparams(ora, c), c.center, c.semi_axes)
        phi0s.append(phi0)
        b.set_state(q, phi0, [np.zeros_like(phi0)] * 2)
    b.step(dts, steps)
    st, nst, t = b.status()
    assert (st == 0).all() and (nst == steps).all()
    assert np.allclose(t, dts * steps, rtol=1e-15)
    for q, c in enumerate(cases):
        P, phi_o, u_o, p_o, du_o = run_oracle(ora, c, dts[q], steps, phi0s[q])
        phi_g, u_g, p_g = b.get_state(q, with_pressure=True)
        uref = uref_of(u_o, du_o, dts[q])
        ephi = np.abs(phi_g - phi_o).max()
        eu = max(np.abs(u_g[a] - u_o[a]).max() for a in range(2)) / uref
        ep = np.abs(p_g - p_o).max() / np.abs(p_o).max()
        say(f"  {c.name}: |dphi| {ephi:.2e} |du|/Uref {eu:.2e} |dp|/|p| {ep:.2e}")
        assert ephi < 1e-12 and eu < 1e-11 and ep < 1e-12, c.name


def all_pair_cases():
    """The nine model x force pairs of Table 1 / Eqs. 4, 11 and CSF, one case
    each, on grids and boxes of several shapes: box edges 1, 2 pi (the
    standing wave's box) and 2, non-square grids, density ratios 1 to 1000."""
    C = workloads.Case
    L = 2.0 * np.pi
    return [
        C("p_cdi_eb", (32, 24), (0.5, 0.3), (0.25, 0.2), 1.0, 0.1, 2e-3, 2e-4, 1.0, 1.0, "CDI", "EB", "fp64"),
        C("p_cdi_csf", (24, 24), (0.5, 0.5), (0.3, 0.25), 240.0, 0.24, 0.1, 0.001, 1.0, 0.75, "CDI", "CSF", "fp64"),
        C("p_cdi_lcsf", (32, 32), (0.5 * L, 0.5 * L), (0.25 * L, 0.2 * L), 1.0, 1.0, 0.01, 0.01, 1.0, 1.0,
          "CDI", "LCSF", "fp64", length=L),
        C("p_sb_eb", (40, 20), (1.0, 0.5), (0.5, 0.3), 2.0, 1.0, 0.02, 0.01, 0.8, 0.9, "SB", "EB", "fp64",
          length=2.0),
        C("p_sb_csf", (20, 28), (0.5, 0.7), (0.3, 0.25), 10.0, 1.0, 0.02, 0.004, 1.5, 1.0, "SB", "CSF", "fp64"),
        C("p_sb_lcsf", (28, 28), (0.5, 0.5), (0.3, 0.22), 1.0, 0.01, 0.01, 1e-4, 1.0, 0.8, "SB", "LCSF", "fp64"),
        C("p_isodi_eb", (24, 32), (0.5, 0.6), (0.3, 0.3), 1.0, 0.001, 0.01, 1e-5, 1.0, 0.75, "ISODI", "EB",
          "fp64"),
        C("p_isodi_csf", (32, 32), (0.5 * L, 0.5 * L), (0.3 * L, 0.22 * L), 3.0, 1.0, 0.03, 0.01, 2.0, 1.0,
          "ISODI", "CSF", "fp64", length=L),
        C("p_isodi_lcsf", (36, 20), (0.4, 0.3), (0.3, 0.2), 1.0, 0.5, 0.02, 0.01, 0.7, 1.0, "ISODI", "LCSF",
          "fp64"),
    ]


def test_batch_fp64_all_pairs_matches_oracle(gpu, ora):
    """All nine model/force pairs in one FP64 batch, with a seeded
    divergence-free initial velocity (advection and viscous terms active),
    4 steps, each case against the oracle."""
    cases = all_pair_cases()
    steps = 4
    say(f"batch FP64 parity, all pairs, {len(cases)} cases x {steps} steps")
    params = [gpu.params_for_case(c, poisson_rtol=1e-14, poisson_maxit=4000) for c in cases]
    b = gpu.Batch(params)
    init, dts = [], []
    for q, c in enumerate(cases):
        P = oparams(ora, c)
        phi0 = ora.init_droplet(P, c.center, c.semi_axes)
        u0 = workloads.divergence_free_velocity(P.shape, 20 + q, amplitude=0.01 * c.length)
        init.append((phi0, u0))
        dts.append(c.dt(umax0=max(np.abs(x).max() for x in u0)))
        b.set_state(q, phi0, u0)
    dts = np.array(dts)
    b.step(dts, steps)
    st, nst, _ = b.status()
    assert (st == 0).all() and (nst == steps).all()
    for q, c in enumerate(cases):
        P = oparams(ora, c)
        phi_o, u_o, p_o = ora.step(P, dts[q], steps, *init[q])     # p: the last stage's pressure
        _, du_o, _ = ora.stage(P, phi_o, u_o, p_o)
        phi_g, u_g, p_g = b.get_state(q, with_pressure=True)
        uref = uref_of(u_o, du_o, dts[q])
        ephi = np.abs(phi_g - phi_o).max()
        eu = max(np.abs(u_g[a] - u_o[a]).max() for a in range(2)) / uref
        ep = np.abs(p_g - p_o).max() / np.abs(p_o).max()
        say(f"  {c.name}: |dphi| {ephi:.2e} |du|/Uref {eu:.2e} |dp|/|p| {ep:.2e}")
        assert ephi < 1e-12 and eu < 1e-11 and ep < 1e-12, c.name


def test_batch_mixed_error_statement(gpu, ora):
    """FP32-mixed batch against the FP64 oracle (started from the FP32-rounded
    phi0): the mixed-precision bounds of the single-case path."""
    cases = mixed_cases("fp32_mixed")
    steps = 5
    say(f"batch FP32-mixed error statement, {len(cases)} cases x {steps} steps")
    b = gpu.Batch([gpu.params_for_case(c) for c in cases])
    dts = np.array([c.dt() for c in cases])
    phi0s = []
    for q, c in enumerate(cases):
        phi0 = ora.init_droplet(oparams(ora, c), c.center, c.semi_axes)
        phi0s.append(phi0.astype(np.float32).astype(np.float64))
        b.set_state(q, phi0s[-1], [np.zeros_like(phi0)] * 2)
    b.step(dts, steps)
    for q, c in enumerate(cases):
        P, phi_o, u_o, p_o, du_o = run_oracle(ora, c, dts[q], steps, phi0s[q])
        phi_g, u_g, p_g = b.get_state(q, with_pressure=True)
        uref = uref_of(u_o, du_o, dts[q])
        ephi = np.abs(phi_g - phi_o).max()
        eu = max(np.abs(u_g[a] - u_o[a]).max() for a in range(2)) / uref
        say(f"  {c.name}: |dphi| {ephi:.2e} |du|/Uref {eu:.2e}")
        assert ephi < 1e-5 and eu < 1e-2, c.name


def test_batch_mixed_matches_single_case_path(gpu, ora):
    """The batched and the single-case FP32-mixed paths compute the same step
    (they differ in reduction order and preconditioner launch layout only)."""
    cases = mixed_cases("fp32_mixed")[:3]
    say("batch vs single-case FP32-mixed")
    b = gpu.Batch([gpu.params_for_case(c) for c in cases])
    dts = np.array([c.dt() for c in cases])
    for q, c in enumerate(cases):
        b.init_droplet(q, c.center, c.semi_axes)
    b.step(dts, 4)
    for q, c in enumerate(cases):
        s = gpu.solver_for_case(c)
        s.init_droplet(c.center, c.semi_axes)
        s.step(dts[q], 4)
        phi_s, u_s, _ = s.get_state()
        phi_b, u_b, _ = b.get_state(q)
        umax = max(np.abs(x).max() for x in u_s) + 1e-300
        ephi = np.abs(phi_b - phi_s).max()
        eu = max(np.abs(u_b[a] - u_s[a]).max() for a in range(2)) / umax
        say(f"  {c.name}: |dphi| {ephi:.2e} |du|/|u| {eu:.2e}")
        # measured: phi to 1.5e-8, u to 7e-7 of max|u| after 4 steps
        assert ephi < 1e-6 and eu < 1e-5, c.name


def test_batch_failure_is_isolated(gpu, ora):
    """A case whose pressure solve cannot converge stops at its last completed
    state; the others advance untouched."""
    cases = mixed_cases("fp64")[:3]
    say("batch failure isolation")
    params = [gpu.params_for_case(c, poisson_rtol=1e-14) for c in cases]
    params[1].poisson_maxit = 1
    b = gpu.Batch(params)
    dts = np.array([c.dt() for c in cases])
    phi0s = []
    for q, c in enumerate(cases):
        phi0s.append(ora.init_droplet(oparams(ora, c), c.center, c.semi_axes))
        b.set_state(q, phi0s[-1], [np.zeros_like(phi0s[-1])] * 2)
    with pytest.raises(gpu.TpfError) as e:
        b.step(dts, 2)
    assert e.value.status == gpu.TPF_ENOCONV
    st, nst, _ = b.status()
    assert list(st) == [0, gpu.TPF_ENOCONV, 0]
    assert list(nst) == [2, 0, 2]
    phi1, u1, _ = b.get_state(1)
    assert np.array_equal(phi1, phi0s[1]) and all(np.abs(x).max() == 0 for x in u1)
    for q in (0, 2):
        _, phi_o, u_o, _, du_o = run_oracle(ora, cases[q], dts[q], 2, phi0s[q])
        phi_g, u_g, _ = b.get_state(q)
        assert np.abs(phi_g - phi_o).max() < 1e-12


def test_batch_graph_replay_is_bitwise(gpu):
    """10 steps in one call (a captured graph of 8 launches, then 2 launches)
    equal 10 calls of one step, bit for bit."""
    cases = mixed_cases("fp32_mixed")[:4]
    say("batch graph replay")
    dts = np.array([c.dt() for c in cases])
    outs = []
    for mode in ("graph", "single"):
        b = gpu.Batch([gpu.params_for_case(c) for c in cases])
        for q, c in enumerate(cases):
            b.init_droplet(q, c.center, c.semi_axes)
        if mode == "graph":
            b.step(dts, 10)
        else:
            for _ in range(10):
                b.step(dts, 1)
        outs.append([b.get_state(q) for q in range(len(cases))])
        b.close()
    for q in range(len(cases)):
        assert np.array_equal(outs[0][q][0], outs[1][q][0])
        for a in range(2):
            assert np.array_equal(outs[0][q][1][a], outs[1][q][1][a])


def test_batch_launch_configs_agree(gpu, ora):
    """Every launch configuration computes the same FP64 step (reduction
    order aside)."""
    cases = mixed_cases("fp64")[:4]
    say("batch launch configurations")
    dts = np.array([c.dt() for c in cases])
    ref = None
    for cfg, (threads, lds) in enumerate(gpu.batch_configs()):
        b = gpu.Batch([gpu.params_for_case(c, poisson_rtol=1e-14) for c in cases])
        b.set_config(cfg)
        for q, c in enumerate(cases):
            b.init_droplet(q, c.center, c.semi_axes)
        b.step(dts, 2)
        got = [b.get_state(q) for q in range(len(cases))]
        b.close()
        say(f"  config {cfg}: {threads} threads, {lds} B LDS")
        if ref is None:
            ref = got
            continue
        for q in range(len(cases)):
            assert np.abs(got[q][0] - ref[q][0]).max() < 1e-13
            umax = max(np.abs(x).max() for x in ref[q][1]) + 1e-300
            assert max(np.abs(got[q][1][a] - ref[q][1][a]).max() for a in range(2)) < 1e-9 * umax


def test_batch_tuner_cache(gpu):
    cases = mixed_cases("fp32_mixed")
    say("batch tuner")
    dts = np.array([c.dt() for c in cases])
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.txt")
        b = gpu.Batch([gpu.params_for_case(c) for c in cases])
        for q, c in enumerate(cases):
            b.init_droplet(q, c.center, c.semi_axes)
        chosen = b.tune(dts, path)
        assert 0 <= chosen < len(gpu.batch_configs())
        st, nst, _ = b.status()
        assert (nst == 0).all()                     # tuning does not advance the state
        lines = open(path).read().split("\n")
        assert len([x for x in lines if x.strip()]) == 1
        b2 = gpu.Batch([gpu.params_for_case(c) for c in cases])
        assert b2.tune(dts, path) == chosen         # read back, not re-timed
        assert len([x for x in open(path).read().split("\n") if x.strip()]) == 1
        b.step(dts, 2)
        assert (b.status()[0] == 0).all()


def test_batch_tuning_leaves_the_run_unchanged(gpu):
    """Tuning between steps times stage evaluations only: with the same launch
    configuration afterwards, a tuned batch steps bit for bit like an untuned
    one (state, pressure warm start, status and step count untouched)."""
    cases = mixed_cases("fp32_mixed")
    say("batch tuning is invisible")
    dts = np.array([c.dt() for c in cases])
    runs = []
    for tune in (False, True):
        b = gpu.Batch([gpu.params_for_case(c) for c in cases])
        b.set_config(2)
        for q, c in enumerate(cases):
            b.init_droplet(q, c.center, c.semi_axes)
        b.step(dts, 2)
        if tune:
            b.tune(dts, None)
            b.set_config(2)
        b.step(dts, 3)
        st, nst, t = b.status()
        assert (st == 0).all() and (nst == 5).all()
        runs.append([b.get_state(q, with_pressure=True) for q in range(len(cases))])
        b.close()
    for q in range(len(cases)):
        for k in (0, 2):
            assert np.array_equal(runs[0][q][k], runs[1][q][k]), (q, k)
        for a in range(2):
            assert np.array_equal(runs[0][q][1][a], runs[1][q][1][a]), (q, a)


def test_batch_solver_stats(gpu):
    """Per-case pressure-solve counters: four solves per step, PCG
    iterations counted, zero after a reset."""
    cases = mixed_cases("fp32_mixed")
    say("batch solver counters")
    dts = np.array([c.dt() for c in cases])
    b = gpu.Batch([gpu.params_for_case(c) for c in cases])
    for q, c in enumerate(cases):
        b.init_droplet(q, c.center, c.semi_axes)
    b.solver_stats(reset=True)
    b.step(dts, 3)
    s = b.solver_stats(reset=True)
    assert (s["solves"] == 12).all()
    assert (s["inner"] >= s["outer"]).all() and (s["inner"] > 0).all()
    z = b.solver_stats()
    assert (z["solves"] == 0).all() and (z["inner"] == 0).all()


def test_batch_diagnostics_match_single_case(gpu):
    cases = mixed_cases("fp64")[:3]
    say("batch diagnostics")
    dts = np.array([c.dt() for c in cases])
    b = gpu.Batch([gpu.params_for_case(c, poisson_rtol=1e-14) for c in cases])
    for q, c in enumerate(cases):
        b.init_droplet(q, c.center, c.semi_axes)
    b.step(dts, 3)
    dg = b.diagnostics()
    for q, c in enumerate(cases):
        s = gpu.solver_for_case(c, poisson_rtol=1e-14)
        s.init_droplet(c.center, c.semi_axes)
        s.step(dts[q], 3)
        ds = s.diagnostics()
        for k in ("mass", "mass0", "se", "phi_min", "phi_max"):
            assert abs(dg[q][k] - ds[k]) <= 1e-12 * max(abs(ds[k]), 1e-300), (c.name, k)
        for k in ("ke", "umax", "dp"):
            assert abs(dg[q][k] - ds[k]) <= 1e-8 * max(abs(ds[k]), 1e-300), (c.name, k)
        assert dg[q]["step"] == 3


@pytest.mark.fullsize
def test_batch_workload_sample_against_oracle(gpu, ora):
    """The 512-drop batched workload (FP32-mixed, its launch configuration
    picked by the tuner): a seeded sample of 16 of its cases
    (default_rng(3)), 2 steps, against the FP64 oracle on each case from the
    same FP32-rounded initial phi: phi to 1e-5, u to 1e-2 of its max (the
    single-case mixed-precision bounds)."""
    cases = workloads.batched_cases(512)
    pick = sorted(int(q) for q in np.random.default_rng(3).choice(len(cases), 16, replace=False))
    say(f"batch workload: 512 cases, oracle sample {pick}")
    b = gpu.Batch([gpu.params_for_case(c) for c in cases])
    for q, c in enumerate(cases):
        b.init_droplet(q, c.center, c.semi_axes)
    dts = np.array([c.dt() for c in cases])
    b.tune(dts)
    phi0 = {q: b.get_state(q)[0] for q in pick}      # FP32-rounded initial phi
    b.step(dts, 2)
    worst_phi = worst_u = 0.0
    for q in pick:
        c = cases[q]
        P = oparams(ora, c)
        phi_o, u_o, _ = ora.step(P, dts[q], 2, phi0[q], [np.zeros(P.shape)] * 2)
        phi_g, u_g, _ = b.get_state(q)
        umax = max(np.abs(x).max() for x in u_o)
        ephi = np.abs(phi_g - phi_o).max()
        eu = max(np.abs(u_g[a] - u_o[a]).max() for a in range(2)) / umax
        worst_phi, worst_u = max(worst_phi, ephi), max(worst_u, eu)
        say(f"  case {q} {c.n}: |dphi| {ephi:.2e} |du|/|u| {eu:.2e}")
        assert ephi < 1e-5 and eu < 1e-2, q
    say(f"  worst: |dphi| {worst_phi:.2e} |du|/|u| {worst_u:.2e}")
