"""The standing-wave study: the exact small-amplitude solution against its
limits and symmetries, the initial state, and short batched runs on the GPU
(against the walled oracle step for step, and against the exact solution)."""
import json
import math

import numpy as np
import pytest

from paper_2205_05835_amd import standing_wave as sw


def test_exact_solution_limits():
    t = np.linspace(0.0, 20.0, 41)
    a = sw.prosperetti(t, 1.0, sw.NU, 1.0, 1.0, sw.SIGMA)
    assert a[0] == pytest.approx(1.0, abs=1e-12)                 # a(0) = a0
    h = 1e-6                                                      # released from rest
    d = (sw.prosperetti([h], 1.0, sw.NU, 1.0, 1.0, sw.SIGMA)[0] - 1.0) / h
    assert abs(d) < 1e-5
    w0 = math.sqrt(sw.SIGMA / 2.0)                                # sigma k^3 / (rho1 + rho2)
    # inviscid limit: a -> cos(w0 t); the interfacial boundary layers correct
    # it by O(sqrt(nu)), so the deviation falls 10x per 100x in nu
    dev = [np.abs(sw.prosperetti(t, 1.0, nu, 1.0, 1.0, sw.SIGMA) - np.cos(w0 * t)).max() for nu in (1e-8, 1e-12)]
    assert dev[1] < 1e-4 and 80 < dev[0] / dev[1] < 120
    # the wave decays: energy is dissipated by viscosity
    assert np.abs(a[-10:]).max() < 0.3
    # the two fluids enter through beta and rho1 + rho2 only
    b1 = sw.prosperetti(t, 1.0, 0.05, 1.0, 3.0, 2.0)
    b2 = sw.prosperetti(t, 1.0, 0.05, 3.0, 1.0, 2.0)
    assert np.abs(b1 - b2).max() < 1e-12


def test_initial_state():
    n = 32
    phi = sw.initial_phi(n, sw.eps_of("fixed", n))
    assert phi.shape == (n, n)
    # 1 at the bottom wall, 0 at the top one
    assert phi[0].min() > 1 - 1e-6 and phi[-1].max() < 1e-6
    # the trough sits at x = dx/2: the first column has the largest amplitude
    amps = [sw.Y0 - (np.nonzero(phi[:n, i] >= 0.5)[0][-1] + 0.5) * (sw.L / n) for i in range(n)]
    assert int(np.argmax(amps)) in (0, n - 1)
    assert sw.amplitude(phi, n) == pytest.approx(sw.A0, rel=1e-3)
    assert sw.eps_of("fixed", 64) / (sw.L / 64) == pytest.approx(2.0)


@pytest.mark.gpu
def test_short_standing_wave_on_gpu(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    out = tmp_path / "w.json"
    print("standing wave, N = 16 and 32, 100 steps", flush=True)
    sw.main(["--n", "16", "32", "--t-end", "0.3", "--sample-steps", "50", "--out", str(out)])
    d = json.loads(out.read_text())
    assert len(d["cases"]) == 36 and len(d["t"]) == 3
    for c in d["cases"]:
        a = c["amplitude"]
        # the trough rises towards y0 (surface tension pulls the interface flat)
        assert a[0] > a[1] > a[2] > 0.0
        assert abs(a[2] - d["exact"][2]) < 0.2 * sw.A0
        # released from rest; the surface energy changes also as the initial
        # tanh profile relaxes to the model's discrete profile, so only the
        # kinetic energy is checked here
        assert c["ke"][0] == 0.0 and c["ke"][2] > 0.0


@pytest.mark.gpu
def test_standing_wave_matches_walled_oracle(ora):
    """Three of the study's cases (N = 16, fixed eps, one pair per model), 100
    steps of dt = 0.003 in the batched form with the bottom and top walls,
    against the oracle with the same walls: phi to 1e-12, u to 1e-10 of its
    maximum, the amplitude to 1e-12 of A0."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_05835_amd import tpf
    n, steps = 16, 100
    pairs = {("CDI", "EB"), ("SB", "CSF"), ("ISODI", "LCSF")}
    cases = [c for c in sw.build_cases([n], 0.1, "fp64") if c["panel"] == "fixed" and (c["model"], c["force"]) in pairs]
    print(f"standing wave vs oracle, N = {n}, {steps} steps, {len(cases)} cases", flush=True)
    b = tpf.Batch([c["params"] for c in cases])
    zero = np.zeros((n, n))
    phi0 = [sw.initial_phi(n, c["eps"]) for c in cases]
    for q in range(len(cases)):
        b.set_state(q, phi0[q], [zero, zero])
    b.step(sw.DT, steps)
    st, _, _ = b.status()
    assert (st == 0).all()
    for q, c in enumerate(cases):
        P = ora.Params(n=(n, n), length=sw.L, model=ora.MODELS[c["model"]], force=ora.FORCES[c["force"]],
                       sigma=sw.SIGMA, eps=c["eps"], gamma=0.1, rho1=sw.RHO, rho2=sw.RHO, visc1=sw.NU * sw.RHO,
                       visc2=sw.NU * sw.RHO, walls=2, poisson_rtol=1e-13)
        phi_o, u_o, _ = ora.step(P, sw.DT, steps, phi0[q], [zero, zero])
        phi_g, u_g, _ = b.get_state(q)
        us = max(np.abs(x).max() for x in u_o)
        ephi = np.abs(phi_g - phi_o).max()
        eu = max(np.abs(u_g[a] - u_o[a]).max() for a in range(2)) / us
        ea = abs(sw.amplitude(phi_g, n) - sw.amplitude(phi_o, n)) / sw.A0
        print(f"  {c['model']}/{c['force']}: |dphi| {ephi:.2e} |du|/|u| {eu:.2e} |dA|/A0 {ea:.2e}", flush=True)
        assert ephi < 1e-12 and eu < 1e-10 and ea < 1e-12
