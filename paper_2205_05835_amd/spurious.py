"""Spurious-current study of the static drop (Sec. 3.1, Fig. 1 and Fig. 2) on
the GPU, with every case of the study in one batched launch per step.

Setup (Sec. 3.1): a drop of diameter D = 0.4 at the centre of the unit box,
equal densities rho = 300 and viscosities visc = 0.1, sigma = 1 (La =
sigma rho D / visc^2 = 12000), u = 0 at t = 0, free-slip walls on all four
sides (--box periodic runs the periodic unit box instead).  Readings where
the paper is silent: gamma = 1, and the time step is the smallest stable
step of all cases (every case takes the same steps).  The measured quantity is
Ca_inf = max|u| visc / sigma (max over cells of the cell-averaged velocity)
against t* = sigma t / (visc D).

Cases, for each of the nine model/force pairs (Table 1 x {Eq. 4, CSF,
Eq. 11}):
  * fixed eps = 1/32 on N x N grids, N in --n (Fig. 2a); the CDI rows at
    N = 64 give the history of Fig. 1;
  * eps = (dx / sqrt(32))^(2/3), i.e. dx = sqrt(32) eps^(3/2), on the same N
    (Fig. 2b).

Writes one JSON file: the parameters, Ca_inf(t*) of every case, and Ca_inf at
--t-report (t* = 250 in the paper).  Only marshals arguments: every step runs
in the HIP kernels of the batched form.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import tpf

MODELS = ("CDI", "SB", "ISODI")
FORCES = ("EB", "CSF", "LCSF")
RHO, VISC, SIGMA, DIAM = 300.0, 0.1, 1.0, 0.4


def eps_of(panel: str, n: int) -> float:
    if panel == "fixed":
        return 1.0 / 32.0
    return ((1.0 / n) / math.sqrt(32.0)) ** (2.0 / 3.0)


def stable_dt(n: int, eps: float, gamma: float, cfl: float = 0.1) -> float:
    """The smallest of the advective (gamma), regularisation-diffusion,
    viscous and capillary limits of the explicit step."""
    h = 1.0 / n
    nu = VISC / RHO
    return min(cfl * h / gamma, cfl * h * h / (gamma * eps), cfl * h * h / nu,
               0.5 * math.sqrt(2.0 * RHO * h ** 3 / (4.0 * math.pi * SIGMA)))


def build_cases(ns, gamma, precision, walls=3):
    cases = []
    for panel in ("fixed", "sharp"):
        for n in ns:
            for model in MODELS:
                for force in FORCES:
                    eps = eps_of(panel, n)
                    p = tpf.make_params((n, n), length=1.0, model=model, force=force, precision=precision,
                                        sigma=SIGMA, eps=eps, gamma=gamma, rho1=RHO, rho2=RHO,
                                        visc1=VISC, visc2=VISC, walls=walls)
                    cases.append({"panel": panel, "n": n, "model": model, "force": force, "eps": eps,
                                  "params": p})
    return cases


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, nargs="+", default=[16, 32, 64, 128])
    ap.add_argument("--t-end", type=float, default=400.0, help="last t* (Fig. 1 runs to 400)")
    ap.add_argument("--t-report", type=float, default=250.0, help="t* of the convergence plots")
    ap.add_argument("--t-sample", type=float, default=10.0, help="t* between history samples")
    ap.add_argument("--gamma", type=float, default=1.0)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_mixed"])
    ap.add_argument("--box", default="walls", choices=["walls", "periodic"],
                    help="free-slip walls on all sides (Sec. 3.1) or a periodic box")
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        sys.exit("the study runs on the GPU")
    tpf.lib()
    cases = build_cases(args.n, args.gamma, args.precision, 3 if args.box == "walls" else 0)
    dt = min(stable_dt(c["n"], c["eps"], args.gamma) for c in cases)
    tscale = VISC * DIAM / SIGMA            # t = t* visc D / sigma
    steps_per_sample = max(1, int(round(args.t_sample * tscale / dt)))
    dt = args.t_sample * tscale / steps_per_sample
    nsamples = int(round(args.t_end / args.t_sample))
    batch = tpf.Batch([c["params"] for c in cases])
    for q, c in enumerate(cases):
        batch.init_droplet(q, (0.5, 0.5), (DIAM / 2, DIAM / 2))
    print(f"{len(cases)} cases, dt = {dt:.4e}, {steps_per_sample} steps per t* = {args.t_sample:g}, "
          f"{nsamples} samples", flush=True)
    hist = [[] for _ in cases]
    tstar = [0.0]
    d0 = batch.diagnostics()
    for q in range(len(cases)):
        hist[q].append(d0[q]["ca_inf"])
    t0 = time.perf_counter()
    for s in range(1, nsamples + 1):
        batch.step(dt, steps_per_sample)
        st, steps, t = batch.status()
        d = batch.diagnostics()
        tstar.append(s * args.t_sample)
        for q in range(len(cases)):
            hist[q].append(d[q]["ca_inf"] if st[q] == 0 else float("nan"))
        bad = int(np.count_nonzero(st))
        print(f"t* = {s * args.t_sample:7.1f}  wall {time.perf_counter() - t0:7.1f} s  stopped cases {bad}",
              flush=True)
    k_rep = int(round(args.t_report / args.t_sample))
    box = "unit square, free-slip walls" if args.box == "walls" else "periodic unit square"
    out = {"setup": {"rho": RHO, "visc": VISC, "sigma": SIGMA, "diameter": DIAM, "gamma": args.gamma,
                     "precision": args.precision, "dt": dt, "box": box, "t_report": args.t_report},
           "tstar": tstar,
           "cases": [{"panel": c["panel"], "n": c["n"], "model": c["model"], "force": c["force"],
                      "eps": c["eps"], "ca_inf": hist[q],
                      "ca_report": hist[q][k_rep] if k_rep < len(hist[q]) else None}
                     for q, c in enumerate(cases)]}
    with open(args.out, "w") as f:
        json.dump(out, f)
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
