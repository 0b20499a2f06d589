"""The standing-wave study: the exact small-amplitude solution against its
limits and symmetries, the mirrored initial state, and a short batched run on
the GPU."""
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


def test_mirrored_initial_state():
    n = 32
    phi = sw.initial_phi(n, sw.eps_of("fixed", n))
    assert phi.shape == (2 * n, n)
    # even about the plane y = 2 pi (a cell face) and periodic: a mirror image
    assert np.abs(phi - phi[::-1, :]).max() < 1e-14
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
