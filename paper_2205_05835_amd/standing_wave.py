"""Standing-wave study (Sec. 3.2, Fig. 3 to 5) on the GPU, with every case of
the study in one batched launch per step, and the exact small-amplitude
solution it is compared with.

Setup (Sec. 3.2): a 2 pi x 2 pi box, periodic in x, free-slip walls at the
bottom and the top; the interface starts at y = y0 - A0 cos(x - dx/2) with
y0 = pi, A0 = 2 pi / 100 (wavelength 2 pi, k = 1); rho1 = rho2 = 1, kinematic
viscosity 0.064720863 in both phases, sigma = 2, dt = 0.003, u = 0 at t = 0.
The amplitude is measured at x = dx/2.

Every case runs on an N x N grid with free-slip walls on the y axis (walls =
2 in the case parameters): no flow through y = 0 and y = 2 pi, no shear and
no normal gradient of phi there.

Readings: eps = 1/32 is taken in units of the box edge (eps = 2 pi / 32, so
eps / dx = N / 32, which is 2 at N = 64 as the text states); the
sharp-interface panel uses dx / L = sqrt(32) (eps / L)^(3/2); gamma = 0.1 (on
the scale of the wave's peak velocity A0 omega0 = 0.063).

Writes one JSON file: for every case the amplitude A(t) and the kinetic and
surface energies (Sec. 3.2, energetics), the exact amplitude of
prosperetti() at the same times, and the l2 error of A against it.  Only
marshals arguments: every step runs in the HIP kernels of the batched form.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

MODELS = ("CDI", "SB", "ISODI")
FORCES = ("EB", "CSF", "LCSF")
L = 2.0 * math.pi
Y0, A0 = math.pi, 2.0 * math.pi / 100.0
RHO, NU, SIGMA, DT = 1.0, 0.064720863, 2.0, 0.003


def prosperetti(t, k, nu, rho1, rho2, sigma):
    """a(t) / a(0) of a small-amplitude standing wave between two viscous
    fluids of equal kinematic viscosity nu, started from rest with no gravity
    (Prosperetti, Phys. Fluids 24 (1981), the initial-value solution):

      a/a0 = 4 (1 - 4b) nu^2 k^4 / (8 (1 - 4b) nu^2 k^4 + w0^2) erfc((nu k^2 t)^1/2)
             + sum_i z_i / Z_i  w0^2 / (z_i^2 - nu k^2)  exp((z_i^2 - nu k^2) t) erfc(z_i t^1/2)

    with b = rho1 rho2 / (rho1 + rho2)^2, w0^2 = sigma k^3 / (rho1 + rho2),
    z_i the four roots of
      z^4 - 4b (k^2 nu)^1/2 z^3 + 2 (1 - 6b) k^2 nu z^2 + 4 (1 - 3b) (k^2 nu)^3/2 z
          + (1 - 4b) nu^2 k^4 + w0^2 = 0
    and Z_i = prod_{j != i} (z_j - z_i).  exp(z^2 t) erfc(z t^1/2) is
    evaluated as the Faddeeva function w(i z t^1/2), which stays finite for
    roots of either sign of real part."""
    from scipy.special import erfc, wofz
    b = rho1 * rho2 / (rho1 + rho2) ** 2
    w02 = sigma * k ** 3 / (rho1 + rho2)
    q = k * k * nu
    z = np.roots([1.0, -4.0 * b * math.sqrt(q), 2.0 * (1.0 - 6.0 * b) * q, 4.0 * (1.0 - 3.0 * b) * q ** 1.5,
                  (1.0 - 4.0 * b) * q * q + w02])
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    a = 4.0 * (1.0 - 4.0 * b) * q * q / (8.0 * (1.0 - 4.0 * b) * q * q + w02) * erfc(np.sqrt(q * t))
    a = a.astype(np.complex128)
    for i in range(4):
        zi = z[i]
        Zi = np.prod([z[j] - zi for j in range(4) if j != i])
        a += zi / Zi * w02 / (zi * zi - q) * np.exp(-q * t) * wofz(1j * zi * np.sqrt(t))
    return a.real


def eps_of(panel: str, n: int) -> float:
    if panel == "fixed":
        return L / 32.0
    return L * ((1.0 / n) / math.sqrt(32.0)) ** (2.0 / 3.0)


def initial_phi(n: int, eps: float) -> np.ndarray:
    """phi on the N x N grid (C order [y][x]): 1 below the interface, from
    the wave-height function of Sec. 3.2."""
    h = L / n
    x = (np.arange(n) + 0.5) * h
    y = (np.arange(n) + 0.5) * h
    height = y[:, None] - Y0 + A0 * np.cos(x - 0.5 * h)[None, :]
    return 0.5 * (1.0 - np.tanh(height / (2.0 * eps)))


def amplitude(phi: np.ndarray, n: int) -> float:
    """y0 minus the interface height in the first column (x = dx/2), the
    height being the column integral of phi from the bottom wall (phi goes
    from 1 to 0 across the interface; for a symmetric profile the integral is
    the height of its midpoint, and the midpoint rule is far more accurate
    than locating phi = 1/2 between two cell centres)."""
    h = L / n
    return Y0 - h * float(np.sum(phi[:n, 0]))


def build_cases(ns, gamma, precision):
    from . import tpf
    cases = []
    for panel in ("fixed", "sharp"):
        for n in ns:
            for model in MODELS:
                for force in FORCES:
                    eps = eps_of(panel, n)
                    p = tpf.make_params((n, n), length=L, model=model, force=force, precision=precision,
                                        sigma=SIGMA, eps=eps, gamma=gamma, rho1=RHO, rho2=RHO,
                                        visc1=NU * RHO, visc2=NU * RHO, walls=2)
                    cases.append({"panel": panel, "n": n, "model": model, "force": force, "eps": eps,
                                  "params": p})
    return cases


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, nargs="+", default=[16, 32, 64, 128])
    ap.add_argument("--t-end", type=float, default=20.0)
    ap.add_argument("--sample-steps", type=int, default=50, help="steps between samples (dt = 0.003)")
    ap.add_argument("--gamma", type=float, default=0.1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_mixed"])
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        sys.exit("the study runs on the GPU")
    from . import tpf
    tpf.lib()
    cases = build_cases(args.n, args.gamma, args.precision)
    batch = tpf.Batch([c["params"] for c in cases])
    for q, c in enumerate(cases):
        n = c["n"]
        zero = np.zeros((n, n))
        batch.set_state(q, initial_phi(n, c["eps"]), [zero, zero])
    nsamples = int(round(args.t_end / (DT * args.sample_steps)))
    print(f"{len(cases)} cases, dt = {DT}, {args.sample_steps} steps per sample, {nsamples} samples", flush=True)
    times = [0.0]
    amp = [[] for _ in cases]
    ke = [[] for _ in cases]
    se = [[] for _ in cases]

    def sample():
        d = batch.diagnostics()
        for q, c in enumerate(cases):
            phi, _, _ = batch.get_state(q)
            amp[q].append(amplitude(phi, c["n"]))
            ke[q].append(d[q]["ke"])
            se[q].append(d[q]["se"])

    sample()
    t0 = time.perf_counter()
    for s in range(1, nsamples + 1):
        batch.step(DT, args.sample_steps)
        st, _, _ = batch.status()
        if np.any(st != 0):
            bad = [f'{cases[q]["model"]}/{cases[q]["force"]}/{cases[q]["n"]}' for q in np.nonzero(st)[0]]
            sys.exit(f"cases stopped: {bad}")
        times.append(s * args.sample_steps * DT)
        sample()
        if s % 10 == 0 or s == nsamples:
            print(f"t = {times[-1]:7.3f}  wall {time.perf_counter() - t0:7.1f} s", flush=True)
    exact = (A0 * prosperetti(np.array(times), 1.0, NU, RHO, RHO, SIGMA)).tolist()
    out = {"setup": {"box": "2 pi x 2 pi, periodic in x, free-slip walls at y = 0 and 2 pi",
                     "rho": RHO, "nu": NU, "sigma": SIGMA, "dt": DT, "A0": A0, "gamma": args.gamma,
                     "precision": args.precision},
           "t": times, "exact": exact, "cases": []}
    ex = np.array(exact)
    for q, c in enumerate(cases):
        a = np.array(amp[q])
        out["cases"].append({"panel": c["panel"], "n": c["n"], "model": c["model"], "force": c["force"],
                             "eps": c["eps"], "amplitude": amp[q], "ke": ke[q], "se": se[q],
                             "l2_error": float(np.sqrt(np.mean((a - ex) ** 2)) / A0)})
    with open(args.out, "w") as f:
        json.dump(out, f)
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
