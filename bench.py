#!/usr/bin/env python3
"""Throughput of the two-phase phase-field step on one MI355X.

Workload: the 256^3 periodic oscillating drop (ellipsoid with semi-axes
0.30, 0.25, 0.25 in the unit box, density and viscosity ratio 10,
eps = 0.75 h, CDI phase field + energy-based surface tension force, FP32
state and stencils with an FP64 pressure / defect-correction residual),
time step from the explicit stability limits (capillary bound, 3.6e-5).
Inputs are synthetic and built on the GPU (tanh profile, u = 0) before the
timed region.

Prints ONE JSON line: cell-steps/s over the timed steps, the roofline of the
dominant kernel class (algorithmic bytes per launch / its mean launch time
from HIP events recorded on the solver stream during the timed steps),
the FP32-vs-FP64 error of the same workload over a few steps, and the plain
CPU oracle timed on a bounded sample of the workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, 8 TB/s

# HBM traffic of the dominant kernel from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE), each scaled by what the same counter reads
# for a plain device copy of known size; recorded with a hash of the kernel
# sources and reported only while the sources still match.
TRAFFIC_DIR = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ("paper_2205_05835_amd/csrc/tpf_poisson.hip", "paper_2205_05835_amd/csrc/tpf_device.hpp")


IMPLICIT_SOURCES = ("paper_2205_05835_amd/csrc/tpf_implicit.hip", "paper_2205_05835_amd/csrc/tpf_device.hpp",
                    "paper_2205_05835_amd/csrc/tpf_stage_ops.hpp")


def kernel_source_hash(kernel=""):
    import hashlib
    h = hashlib.sha256()
    for f in (IMPLICIT_SOURCES if kernel.startswith("imp_") else KERNEL_SOURCES):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel):
    """Traffic bytes per launch of kernel class `kernel` from the committed
    counter summary profiles/<class>_256cubed_traffic.json, or None if there
    is none or the kernel sources changed since."""
    try:
        with open(os.path.join(TRAFFIC_DIR, f"{kernel}_256cubed_traffic.json")) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("class") != kernel or rec.get("source_hash") != kernel_source_hash(kernel):
        return None
    return rec.get("traffic_bytes_per_launch")


def copy_calibration(nbytes=1 << 29, reps=5):
    """A plain device-to-device copy of known size (for scaling the HBM
    traffic counters): reps copies of nbytes."""
    import torch
    torch.cuda.set_device(0)
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}), flush=True)


def gpu_run(args):
    import numpy as np
    import torch

    import workloads
    from paper_2205_05835_amd import tpf

    torch.cuda.set_device(0)
    case = workloads.oscillating_drop_3d(args.n, "fp32_mixed")
    dt = case.dt()
    s = tpf.solver_for_case(case, poisson_rtol_inner=args.poisson_rtol_inner)
    s.init_droplet(case.center, case.semi_axes)
    s.step(dt, args.warmup)
    torch.cuda.synchronize()

    # attribution pass (all classes timed; not the measured region)
    s.profile_enable(-1)
    s.step(dt, 1)
    prof_all = s.profile_read()
    s.profile_enable(0)
    names = s.profile_classes()
    # the roofline is quoted for one kernel symbol: the aggregate classes
    # (all coarse levels, reduction finalizes, small vector kernels) are excluded
    single = {k: v for k, v in prof_all.items()
              if k not in ("mg_coarse_levels", "reduce_finalize", "vector") and v["launches"]}
    dominant = max(single, key=lambda k: single[k]["ms"])
    dom_bit = names.index(dominant)

    # timed region: K steps, events around the dominant class only
    s.profile_enable(1 << dom_bit)
    s.solver_stats(reset=True)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    s.step(dt, args.steps)
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ev_ms = ev0.elapsed_time(ev1)
    dom = s.profile_read()[dominant]
    s.profile_enable(0)
    stats = s.solver_stats()
    diag = s.diagnostics()

    cells = case.cells
    value = cells * args.steps / wall
    mean_launch_s = dom["ms"] / max(dom["launches"], 1) * 1e-3
    achieved = dom["bytes_per_launch"] / mean_launch_s / 1e9 if mean_launch_s > 0 else 0.0
    out = {
        "case": case, "dt": dt, "value": value, "wall": wall, "ev_ms": ev_ms, "diag": diag,
        "dominant": dominant, "dom": dom, "achieved": achieved, "stats": stats,
        "breakdown": {k: round(v["ms"], 4) for k, v in sorted(prof_all.items(), key=lambda kv: -kv[1]["ms"]) if v["launches"]},
        "breakdown_launches": {k: v["launches"] for k, v in prof_all.items() if v["launches"]},
    }
    out["step_ms_attribution"] = sum(v["ms"] for v in prof_all.values())
    # algorithmic bytes of one whole step (every working launch of the
    # attributed step), against the wall time per timed step
    out["step_bytes"] = sum(v["launches"] * v["bytes_per_launch"] for v in prof_all.values())

    if not args.no_fp64_compare:
        m = args.compare_steps
        s64 = tpf.solver_for_case(workloads.oscillating_drop_3d(args.n, "fp64"))
        s64.init_droplet(case.center, case.semi_axes)
        s64.step(dt, m)
        d64 = s64.diagnostics()
        phi64, u64, _ = s64.get_state()
        del s64
        s32 = tpf.solver_for_case(case)
        s32.init_droplet(case.center, case.semi_axes)
        s32.step(dt, m)
        d32 = s32.diagnostics()
        phi32, u32, _ = s32.get_state()
        del s32
        umax = max(float(np.abs(x).max()) for x in u64)
        out["fp32_vs_fp64"] = {
            "steps": m,
            "phi_max_abs": float(np.abs(phi32 - phi64).max()),
            "u_max_rel": float(max(np.abs(u32[a] - u64[a]).max() for a in range(3)) / umax),
            "dp_rel": abs(d32["dp"] - d64["dp"]) / abs(d64["dp"]),
            "mass_drift_fp32": abs(d32["mass"] - d32["mass0"]) / d32["mass0"],
            "mass_drift_fp64": abs(d64["mass"] - d64["mass0"]) / d64["mass0"],
        }
        del phi64, u64, phi32, u32
    del s
    torch.cuda.empty_cache()
    return out


def batch_run(args):
    """The batched form on the uneven many-droplet workload: 512 2D drops on
    grids of 64^2 to 192^2, FP32-mixed, one launch per RK4 step, each case
    with its own time step; launch shape picked by the tuner."""
    import numpy as np
    import torch

    import workloads
    from paper_2205_05835_amd import tpf

    cases = workloads.batched_cases(args.batch_cases)
    b = tpf.Batch([tpf.params_for_case(c) for c in cases])
    for q, c in enumerate(cases):
        b.init_droplet(q, c.center, c.semi_axes)
    dts = np.array([c.dt() for c in cases])
    config = b.tune(dts)
    threads, lds = tpf.batch_configs()[config]
    failed = None
    try:
        b.step(dts, args.batch_warmup)
        b.solver_stats(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(dts, args.batch_steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    except tpf.TpfError as e:
        failed = str(e)
        wall = float("nan")
    stats = b.solver_stats()
    st, nst, _ = b.status()
    dg = b.diagnostics()
    cells = sum(c.cells for c in cases)
    out = {"workload": f"{len(cases)} 2D drops, grids 64^2..192^2 (seeded), FP32-mixed",
           "cases": len(cases), "cells": cells, "steps": args.batch_steps,
           "value": round(cells * args.batch_steps / wall, 1) if failed is None else None,
           "unit": "cell-steps/s", "ms_per_step": round(wall / args.batch_steps * 1e3, 4),
           "launch_config": {"threads": threads, "lds_bytes": lds},
           "cases_stopped": int((st != 0).sum()), "error": failed,
           "phi_min": min(d["phi_min"] for d in dg), "phi_max": max(d["phi_max"] for d in dg),
           "mean_pcg_iterations_last_solve": float(np.mean([d["poisson_inner"] for d in dg]))}
    # Roofline by the 2D mixed-precision byte model (one pass per operator,
    # units of one FP32 field sweep): per RK stage 27 + 6 units for the stage
    # operators and the projection, and per pressure solve 42 units per
    # defect-correction pass plus 43 per PCG iteration (V-cycle included),
    # with each case's counted passes and iterations of the timed steps.
    units = np.array([132.0 * args.batch_steps + 42.0 * stats["outer"][q] + 43.0 * stats["inner"][q]
                      for q in range(len(cases))])
    cells_q = np.array([c.cells for c in cases], dtype=np.float64)
    alg_bytes = float((units * cells_q * 4.0).sum()) / args.batch_steps
    # FP32-mixed fields per case: 12 state + 10 stage + 3 solver (4 B), b, p and
    # 3 pressure histories (8 B), 5 per multigrid level (4/3 of the fine grid)
    ws_case = cells_q * (25 * 4 + 5 * 8 + 5 * 4 * 4.0 / 3.0)
    if failed is None:
        ach = alg_bytes / (wall / args.batch_steps) / 1e9
        out["roofline"] = {
            "bound": "hbm", "model": "2D byte model: 132 units/step + 42 per outer pass + 43 per PCG iteration",
            "algorithmic_gb_per_step": round(alg_bytes / 1e9, 3), "achieved": round(ach, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
            "pcg_iterations_per_solve": round(float(stats["inner"].sum() / max(stats["solves"].sum(), 1)), 3),
            "outer_per_solve": round(float(stats["outer"].sum() / max(stats["solves"].sum(), 1)), 3),
            "working_set_gb": round(float(ws_case.sum()) / 1e9, 3),
            "largest_case_working_set_mb": round(float(ws_case.max()) / 1e6, 2),
            "cache_resident": False,
            "note": "the batch's working set is several times the 256 MB last-level cache and all cases "
                    "run at once, so the model's bytes come from HBM"}
    del b
    if args.batch_compare:
        # FP32-mixed vs FP64 on a seeded sample of the cases
        m = args.batch_compare
        sample = cases[:m]
        res = {}
        for prec in ("fp64", "fp32_mixed"):
            bb = tpf.Batch([tpf.params_for_case(c, precision=prec) for c in sample])
            for q, c in enumerate(sample):
                bb.init_droplet(q, c.center, c.semi_axes)
            bb.step(dts[:m], 5)
            res[prec] = [bb.get_state(q) for q in range(m)]
            del bb
        ephi = max(float(np.abs(res["fp32_mixed"][q][0] - res["fp64"][q][0]).max()) for q in range(m))
        eu = max(float(max(np.abs(res["fp32_mixed"][q][1][a] - res["fp64"][q][1][a]).max() for a in range(2)) /
                       (max(np.abs(x).max() for x in res["fp64"][q][1]) + 1e-300)) for q in range(m))
        out["fp32_vs_fp64_sample"] = {"cases": m, "steps": 5, "phi_max_abs": ephi, "u_max_rel": eu}
    torch.cuda.empty_cache()
    return out


def adjoint_run(args):
    """Adjoint/forward time on the 256^2 oscillating ellipse (0.30, 0.22),
    density ratio 10, FP32-mixed: a rollout of K steps with a checkpoint every
    `every` steps, loss = h^2/2 sum (phi_T - phi_target)^2 with the target a
    seeded perturbed ellipse; backward = checkpoint reloads, recomputation
    with a tape and the hand-written adjoint sweep."""
    import numpy as np
    import torch

    import workloads
    from paper_2205_05835_amd import adjoint, tpf

    case = workloads.oscillating_drop_2d(256, args.adjoint_precision)
    dt = case.dt()
    params = tpf.params_for_case(case)
    s0 = tpf.solver_for_case(case)
    s0.init_droplet(case.center, case.semi_axes)
    phi0, u0 = s0.get_state_device()
    xi = np.random.default_rng(1).normal(size=2)
    axes = (case.semi_axes[0] * (1 + 0.05 * xi[0]), case.semi_axes[1] * (1 + 0.05 * xi[1]))
    s0.init_droplet(case.center, axes)
    tgt, _ = s0.get_state_device()
    del s0
    f0 = phi0.clone().requires_grad_(True)
    uu = [x.clone().requires_grad_(True) for x in u0]
    sig = torch.tensor(case.sigma, dtype=torch.float64, requires_grad=True)
    eps = torch.tensor(case.eps, dtype=torch.float64, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi, u = adjoint.rollout(f0, uu, sig, eps, params, dt, args.adjoint_steps, args.adjoint_every)
    loss = 0.5 * case.h ** 2 * ((phi - tgt) ** 2).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out = {"workload": f"{case.name}, {args.adjoint_precision}, {args.adjoint_steps} steps, "
                       f"checkpoint every {args.adjoint_every}",
           "forward_s": round(t1 - t0, 4), "backward_s": round(t2 - t1, 4),
           "adjoint_over_forward": round((t2 - t1) / (t1 - t0), 4),
           "loss": float(loss.detach()), "dL_dsigma": float(sig.grad), "dL_deps": float(eps.grad),
           "dL_dphi0_norm": float(f0.grad.norm())}
    torch.cuda.empty_cache()
    return out


def fixed_run(args):
    """The same 256^3 step with a fixed amount of pressure-solver work
    (TPF_FIXED_PCG=outer,inner: that many defect-correction passes of that
    many PCG iterations each, no convergence test), so that cell-steps/s can
    be compared across solver versions whatever their iteration counts."""
    import torch

    import workloads
    from paper_2205_05835_amd import tpf

    case = workloads.oscillating_drop_3d(args.n, "fp32_mixed")
    dt = case.dt()
    os.environ["TPF_FIXED_PCG"] = args.fixed_pcg
    try:
        s = tpf.solver_for_case(case)
    finally:
        del os.environ["TPF_FIXED_PCG"]
    s.init_droplet(case.center, case.semi_axes)
    s.step(dt, 1)
    s.profile_enable(-1)
    s.step(dt, 1)
    prof = s.profile_read()
    s.profile_enable(0)
    step_bytes = sum(v["launches"] * v["bytes_per_launch"] for v in prof.values())
    s.solver_stats(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(dt, args.fixed_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stats = s.solver_stats()
    out = {"outer_inner": args.fixed_pcg, "steps": args.fixed_steps,
           "value": round(case.cells * args.fixed_steps / wall, 1), "unit": "cell-steps/s",
           "ms_per_step": round(wall / args.fixed_steps * 1e3, 4),
           "pcg_iterations_per_solve": round(stats["inner"] / max(stats["solves"], 1), 3),
           "outer_per_solve": round(stats["outer"] / max(stats["solves"], 1), 3),
           "step_hbm": {"algorithmic_gb_per_step": round(step_bytes / 1e9, 3),
                        "achieved": round(step_bytes / (wall / args.fixed_steps) / 1e9, 1), "unit": "GB/s",
                        "frac": round(step_bytes / (wall / args.fixed_steps) / 1e9 / HBM_PEAK_GBS, 4)}}
    del s
    torch.cuda.empty_cache()
    return out


def implicit_run(args):
    """Backward-Euler ISODI phase-field steps (Newton + BiCGStab, FP64) on the
    n^3 drop of radius 0.3 in the unit box, eps = 1.5 h, gamma = 1, under a
    seeded divergence-free velocity with max |u_a| = 0.5, dt = `mult` x the
    forward-Euler limit of the regularisation diffusion.  One untimed step,
    one attributed step (every kernel class timed), then the timed steps with
    events around the dominant kernel class only."""
    import torch

    import workloads
    from paper_2205_05835_amd import tpf

    n = args.implicit_n
    case = workloads.implicit_drop((n, n, n))
    dt = workloads.implicit_dt(case, args.implicit_mult)
    s = tpf.solver_for_case(case)
    s.init_droplet(case.center, case.semi_axes)
    phi, _ = s.get_state_device()
    u = [torch.from_numpy(x).to(s.device) for x in
         workloads.implicit_velocity(tuple(reversed(case.n)), seed=21)]
    s.set_state(phi, u)
    del phi, u
    s.implicit_phase_step(dt, 1)
    s.profile_enable(-1)
    s.implicit_phase_step(dt, 1)
    prof_all = s.profile_read()
    s.profile_enable(0)
    names = s.profile_classes()
    single = {k: v for k, v in prof_all.items()
              if k.startswith("imp_") and k not in ("imp_vector", "imp_finalize") and v["launches"]}
    dominant = max(single, key=lambda k: single[k]["ms"])
    s.profile_enable(1 << names.index(dominant))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = s.implicit_phase_step(dt, args.implicit_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dom = s.profile_read()[dominant]
    s.profile_enable(0)
    mean_s = dom["ms"] / max(dom["launches"], 1) * 1e-3
    achieved = dom["bytes_per_launch"] / mean_s / 1e9 if mean_s > 0 else 0.0
    steps = args.implicit_steps
    out = {"workload": f"{case.name}, ISODI, FP64, dt = {args.implicit_mult} x h^2/(2 dim gamma eps)",
           "dt": dt, "steps": steps, "value": round(case.cells * steps / wall, 1), "unit": "cell-steps/s",
           "ms_per_step": round(wall / steps * 1e3, 3),
           "newton_per_step": round(info["newton_total"] / steps, 3),
           "krylov_per_step": round(info["krylov_total"] / steps, 3),
           "residual": info["residual"],
           "roofline": {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": recorded_traffic(dominant),
                        "bytes_per_launch": dom["bytes_per_launch"],
                        "mean_launch_us": round(mean_s * 1e6, 3), "launches": dom["launches"]},
           "breakdown_ms_one_step": {k: round(v["ms"], 3) for k, v in
                                     sorted(prof_all.items(), key=lambda kv: -kv[1]["ms"]) if v["launches"]}}
    del s
    torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(args):
    """The oracle as it stands, on the host cores, on a bounded sample: the
    same oscillating-drop configuration at 64^3 for 2 RK4 steps on all the
    oracle's threads (the value), and at 48^3 for 1 step on one thread and
    on all of them (the parallel speed-up of the oracle on this host)."""
    import numpy as np

    import oracle
    import workloads

    def run(n, steps):
        c = workloads.oscillating_drop_3d(n, "fp64")
        P = oracle.Params(n=c.n, eps=c.eps, rho1=c.rho1, rho2=c.rho2, visc1=c.visc1, visc2=c.visc2,
                          sigma=c.sigma)
        phi = oracle.init_droplet(P, c.center, c.semi_axes)
        zero = [np.zeros(P.shape)] * 3
        t0 = time.perf_counter()
        oracle.step(P, c.dt(), steps, phi, zero)
        t = time.perf_counter() - t0
        return c.cells * steps / t, t

    n, steps = args.cpu_n, args.cpu_steps
    cores = oracle.threads()
    value, t = run(n, steps)
    out = {"value": value, "unit": "cell-steps/s", "cores": cores, "kind": "oracle",
           "sample": f"{steps} RK4 steps of the same drop configuration at {n}^3 "
                     f"(FP64, Jacobi-PCG pressure to 1e-14), {t:.1f} s",
           "cpu_model": cpu_model()}
    if args.cpu_single_n > 0:
        many, t_many = run(args.cpu_single_n, 1)
        prev = oracle.set_threads(1)
        try:
            one, t_one = run(args.cpu_single_n, 1)
        finally:
            oracle.set_threads(prev)
        out["threads_1_vs_all"] = {
            "sample": f"1 RK4 step at {args.cpu_single_n}^3", "unit": "cell-steps/s",
            "threads_1": one, "seconds_1": round(t_one, 2),
            f"threads_{cores}": many, f"seconds_{cores}": round(t_many, 2)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256, help="cells per axis of the drop workload")
    ap.add_argument("--compare-steps", type=int, default=3)
    ap.add_argument("--poisson-rtol-inner", type=float, default=0.0,
                    help="floor of the FP32 inner PCG tolerance (0: library default)")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=64)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--cpu-single-n", type=int, default=48,
                    help="grid of the one-thread vs all-threads oracle sample (0: skip)")
    ap.add_argument("--breakdown-out", default="")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched many-droplet measurement")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward measurement")
    ap.add_argument("--adjoint-steps", type=int, default=500)
    ap.add_argument("--adjoint-every", type=int, default=50)
    ap.add_argument("--adjoint-precision", default="fp32_mixed", choices=["fp32_mixed", "fp64"])
    ap.add_argument("--batch-cases", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--batch-warmup", type=int, default=2)
    ap.add_argument("--batch-compare", type=int, default=16,
                    help="cases of the FP32-vs-FP64 batch comparison (0: skip)")
    ap.add_argument("--no-fixed", action="store_true",
                    help="skip the fixed-iteration (comparable-work) measurement")
    ap.add_argument("--fixed-pcg", default="2,6", help="outer,inner of the fixed-iteration measurement")
    ap.add_argument("--fixed-steps", type=int, default=5)
    ap.add_argument("--no-implicit", action="store_true",
                    help="skip the backward-Euler ISODI phase-field measurement")
    ap.add_argument("--implicit-n", type=int, default=256)
    ap.add_argument("--implicit-steps", type=int, default=3)
    ap.add_argument("--implicit-mult", type=float, default=10.0)
    ap.add_argument("--implicit-only", action="store_true",
                    help="only the backward-Euler ISODI measurement (its own JSON line; for profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design, not an implementation)", file=sys.stderr)
        sys.exit(2)

    if args.implicit_only:
        print(json.dumps({"implicit_isodi": implicit_run(args)}))
        return
    g = gpu_run(args)
    case = g["case"]
    batch = None if args.no_batch else batch_run(args)
    adj = None if args.no_adjoint else adjoint_run(args)
    imp = None if args.no_implicit else implicit_run(args)
    fixed = None if args.no_fixed else fixed_run(args)
    cpu = None if args.no_cpu_baseline else cpu_baseline(args)
    dom = g["dom"]
    line = {
        "metric": "cell-steps/s at 256^3 + % HBM roofline; adjoint/forward time; FP32 vs FP64 err",
        "value": round(g["value"], 1),
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(g["wall"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": case.name, "grid": list(case.n), "cells": case.cells,
                   "phase_field": case.model, "surface_force": case.force,
                   "precision": "fp32 state/stencils/smoothers, fp64 pressure residual",
                   "density_ratio": case.rho1 / case.rho2, "eps_over_h": case.eps_over_h,
                   "dt": g["dt"]},
        "roofline": {"bound": "hbm", "kernel": g["dominant"],
                     "achieved": round(g["achieved"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(g["achieved"] / HBM_PEAK_GBS, 4),
                     "traffic": recorded_traffic(g["dominant"]),
                     "bytes_per_launch": dom["bytes_per_launch"],
                     "mean_launch_us": round(dom["ms"] / max(dom["launches"], 1) * 1e3, 3),
                     "launches": dom["launches"]},
        "cpu_baseline": cpu,
        "poisson_last_solve": {"outer": g["diag"]["poisson_outer"], "inner": g["diag"]["poisson_inner"],
                               "relres": g["diag"]["poisson_relres"]},
        "poisson_timed": {"solves": g["stats"]["solves"],
                          "outer_per_solve": round(g["stats"]["outer"] / max(g["stats"]["solves"], 1), 3),
                          "pcg_iterations_per_solve": round(g["stats"]["inner"] / max(g["stats"]["solves"], 1), 3)},
        "fp32_vs_fp64": g.get("fp32_vs_fp64"),
        "adjoint_over_forward": adj["adjoint_over_forward"] if adj else None,
        "adjoint": adj,
        "batched": batch,
        "implicit_isodi": imp,
        "fixed_iterations": fixed,
        "event_ms_per_step": round(g["ev_ms"] / args.steps, 4),
        "step_hbm": {"algorithmic_gb_per_step": round(g["step_bytes"] / 1e9, 3),
                     "achieved": round(g["step_bytes"] / (g["wall"] / args.steps) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(g["step_bytes"] / (g["wall"] / args.steps) / 1e9 / HBM_PEAK_GBS, 4)},
    }
    if args.breakdown_out:
        with open(args.breakdown_out, "w") as f:
            json.dump({"ms_one_step": g["breakdown"], "launches": g["breakdown_launches"]}, f, indent=1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
