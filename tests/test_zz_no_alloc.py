"""tpf_diagnostics_noalloc (the entry point for callers that cannot allocate)
against tpf_diagnostics of a context holding the same state, through the C
ABI: two calls in a row on one device, the second on a smaller grid, to the
FP64 parity bound (1e-12 relative); a NULL pressure gives dp = NaN; a grid
beyond the static scratch is rejected before any device work."""
import ctypes
import math
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

KEYS = ("mass", "ke", "se", "dp", "umax", "ca_inf", "div_max", "phi_min", "phi_max")


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


def noalloc(gpu, params, phi, u, p, stream):
    d = gpu.tpf_diag()
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    uu = [ptr(x) for x in u] + [None] * (3 - len(u))
    st = gpu.lib().tpf_diagnostics_noalloc(ctypes.byref(params), ptr(phi), *uu, ptr(p),
                                           ctypes.c_void_p(stream.cuda_stream), ctypes.byref(d))
    return st, d.as_dict()


def compare_one(gpu, case):
    import torch
    say(f"noalloc diagnostics {case.n} {case.model} {case.force}")
    s = gpu.solver_for_case(case, poisson_rtol=1e-13)
    s.init_droplet(case.center, case.semi_axes)
    shape = tuple(reversed(case.n))
    phi, u, _ = s.get_state()
    u = workloads.random_velocity(shape, 3, amplitude=0.05)
    s.set_state(phi, u)
    s.step(case.dt(umax0=0.05), 2)
    ref = s.diagnostics()                          # also leaves the projection pressure in the view
    vphi, vu, vp = s.state_views()
    assert vphi.dtype == torch.float64
    st, got = noalloc(gpu, s.params, vphi, vu, vp, s.stream)
    assert st == gpu.TPF_OK, gpu.lib().tpf_last_error()
    for k in KEYS:
        scale = max(abs(ref[k]), 1e-300)
        assert abs(got[k] - ref[k]) <= 1e-12 * scale, (k, got[k], ref[k])
    assert math.isnan(got["mass0"]) and got["step"] == 0
    return s, vphi, vu


def test_noalloc_matches_diagnostics_twice_smaller_second(gpu):
    C = workloads.Case
    big = C("na3d", (96, 40, 32), (0.5, 0.2, 0.17), (0.3, 0.15, 0.12), 10.0, 1.0, 0.02, 0.004, 1.0, 1.0,
            "SB", "LCSF", "fp64")
    small = C("na2d", (40, 24), (0.5, 0.3), (0.3, 0.2), 1.0, 0.1, 2e-3, 2e-4, 1.0, 1.0, "CDI", "EB", "fp64")
    compare_one(gpu, big)
    s, vphi, vu = compare_one(gpu, small)
    # no pressure: dp is NaN, the rest unchanged
    st, got = noalloc(gpu, s.params, vphi, vu, None, s.stream)
    assert st == gpu.TPF_OK and math.isnan(got["dp"])


def test_noalloc_rejects_grids_beyond_scratch(gpu):
    import torch
    p = gpu.make_params((8192, 8192))              # 128 x 2048 tiles > 65536
    dummy = torch.zeros(1, dtype=torch.float64, device="cuda")
    st, _ = noalloc(gpu, p, dummy, [dummy, dummy], None, torch.cuda.current_stream())
    assert st == gpu.TPF_EINVAL
    assert b"static scratch" in gpu.lib().tpf_last_error()
