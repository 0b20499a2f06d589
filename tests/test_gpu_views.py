"""Zero-copy state access through tpf_field_offset (the boundary's view of
the state of the problem statement, Sec. 3.1: given phi and u, advance and
report).

A view of the workspace must see exactly what tpf_get_state copies out, move
with the state slot at every step, and a state written through the views
followed by tpf_state_changed must behave exactly as the same state set by
tpf_set_state.
"""
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


def make_case(dim, precision):
    if dim == 2:
        return workloads.Case("views2d", (40, 24), (0.5, 0.5), (0.3, 0.22), 10.0, 1.0, 0.02, 0.004,
                              1.0, 1.0, "CDI", "EB", precision)
    return workloads.Case("views3d", (24, 16, 16), (0.5, 0.5, 0.5), (0.3, 0.25, 0.22), 10.0, 1.0,
                          0.02, 0.004, 1.0, 1.0, "SB", "LCSF", precision)


def seeded_state(case, gpu):
    import oracle
    P = oracle.Params(n=case.n, eps=case.eps)
    phi = oracle.init_droplet(P, case.center, case.semi_axes)
    shape = tuple(reversed(case.n))
    u = workloads.random_velocity(shape, 5, amplitude=0.02)
    return phi, u


@pytest.mark.parametrize("dim,precision", [(2, "fp64"), (3, "fp64"), (2, "fp32_mixed"), (3, "fp32_mixed")])
def test_views_match_get_state_and_follow_steps(gpu, dim, precision):
    import torch
    case = make_case(dim, precision)
    say(f"views: {case.n} {precision}")
    s = gpu.solver_for_case(case, poisson_rtol=1e-13 if precision == "fp64" else 0.0)
    phi0, u0 = seeded_state(case, gpu)
    s.set_state(phi0, u0)
    want = torch.float64 if precision == "fp64" else torch.float32
    for nstep in range(3):
        vphi, vu, vp = s.state_views()
        assert vphi.dtype == want and all(x.dtype == want for x in vu) and vp.dtype == torch.float64
        assert len(vu) == dim and vphi.shape == s.shape
        phi, u, p = s.get_state(with_pressure=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(vphi.double().cpu().numpy(), phi)
        for a in range(dim):
            np.testing.assert_array_equal(vu[a].double().cpu().numpy(), u[a])
        # after get_state(p) the pressure view holds the zero-mean projection pressure
        np.testing.assert_array_equal(vp.cpu().numpy(), p)
        s.step(case.dt(umax0=0.02), 1)
    # bad fields
    with pytest.raises(gpu.TpfError):
        s.field_offset(99)
    if dim == 2:
        with pytest.raises(gpu.TpfError):
            s.field_offset(gpu.TPF_STATE_U2)


@pytest.mark.parametrize("dim,precision", [(2, "fp64"), (3, "fp32_mixed")])
def test_write_through_views_equals_set_state(gpu, dim, precision):
    import torch
    case = make_case(dim, precision)
    say(f"write views: {case.n} {precision}")
    phi0, u0 = seeded_state(case, gpu)
    a = gpu.solver_for_case(case)
    a.set_state(phi0, u0)
    b = gpu.solver_for_case(case)
    b.init_droplet(case.center, case.semi_axes)      # some other state first
    b.step(case.dt(), 1)
    vphi, vu, _ = b.state_views()
    vphi.copy_(torch.from_numpy(phi0))
    for k in range(dim):
        vu[k].copy_(torch.from_numpy(u0[k]))
    b.state_changed()
    da, db = a.diagnostics(), b.diagnostics()
    assert db["t"] == 0.0 and db["step"] == 0
    assert da["mass0"] == db["mass0"]
    dt = case.dt(umax0=0.02)
    a.step(dt, 3)
    b.step(dt, 3)
    pa, ua, qa = a.get_state(with_pressure=True)
    pb, ub, qb = b.get_state(with_pressure=True)
    np.testing.assert_array_equal(pa, pb)
    for k in range(dim):
        np.testing.assert_array_equal(ua[k], ub[k])
    np.testing.assert_array_equal(qa, qb)
