"""GPU tests of the hand-written adjoint (2D and 3D, every model and force).

Checks, all through the C ABI:
  * the transpose of one stage evaluation against central differences of
    the forward stage (the dot-product test <l, J v> = <J^T l, v>), for the
    state and for sigma and eps, for all nine model/force pairs in 2D and
    three in 3D;
  * the adjoint of several RK4 steps against central differences of the GPU
    forward and of the FP64 oracle's forward (the oracle's gradient);
  * checkpointed rollouts through torch.autograd equal one-segment adjoints;
  * the FP32-mixed adjoint against the FP64 one (stated bound).
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

PAIRS_2D = [(m, f) for m in ("CDI", "SB", "ISODI") for f in ("EB", "CSF", "LCSF")]
PAIRS_3D = [("CDI", "EB"), ("SB", "CSF"), ("ISODI", "LCSF")]


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


def small_case(n=(32, 24), precision="fp64", model="CDI", force="EB"):
    if len(n) == 2:
        return workloads.Case(f"adj_{n[0]}x{n[1]}", n, (0.5, 0.3), (0.3, 0.17), 1.0, 0.1, 0.02, 0.004,
                              1.0, 1.0, model, force, precision)
    return workloads.Case(f"adj_{n[0]}x{n[1]}x{n[2]}", n, (0.5, 0.35, 0.3), (0.27, 0.2, 0.17), 1.0, 0.1,
                          0.02, 0.004, 1.0, 1.0, model, force, precision)


def oparams(ora, case, **kw):
    base = dict(n=case.n, length=case.length, model=ora.MODELS[case.model],
                force=ora.FORCES[case.force], sigma=case.sigma, eps=case.eps, gamma=case.gamma,
                rho1=case.rho1, rho2=case.rho2, visc1=case.visc1, visc2=case.visc2,
                poisson_rtol=1e-14)
    base.update(kw)
    return ora.Params(**base)


def state(ora, case, seed=0):
    """A drop with a smooth perturbation (phi stays in (0, 1)) and a smooth
    velocity field, so every stage operator is active."""
    P = oparams(ora, case)
    phi = ora.init_droplet(P, case.center, case.semi_axes)
    shape = P.shape
    phi = phi + 0.3 * phi * (1 - phi) * workloads.smooth_field(shape, seed + 1)
    u = workloads.random_velocity(shape, seed + 2, amplitude=0.2)
    return phi, u


def direction(case, phi, seed):
    shape = tuple(reversed(case.n))
    v = 4 * phi * (1 - phi) * workloads.smooth_field(shape, seed)
    v = v / np.abs(v).max()
    vu = workloads.random_velocity(shape, seed + 5, amplitude=1.0)
    return v, vu


def solver(gpu, case, **kw):
    kw.setdefault("poisson_rtol", 1e-14)
    kw.setdefault("poisson_maxit", 2000)
    kw.setdefault("adjoint", 1)
    return gpu.solver_for_case(case, **kw)


def stage_out(s, phi, u):
    s.set_state(phi, u)
    return s.eval_field("DPHI"), [s.eval_field(f"DU{a}") for a in range(len(u))]


def dot(a, b):
    return float(sum(np.vdot(x.ravel(), y.ravel()) for x, y in zip(a, b)))


@pytest.mark.parametrize("n,model,force", [((32, 24), m, f) for m, f in PAIRS_2D] +
                         [((16, 12, 10), m, f) for m, f in PAIRS_3D])
def test_stage_adjoint_dot_product(gpu, ora, n, model, force):
    case = small_case(n, model=model, force=force)
    dim = len(n)
    say(f"stage adjoint dot-product test {case.n} {model} {force}")
    phi, u = state(ora, case)
    shape = phi.shape
    lphi = workloads.smooth_field(shape, 11)
    lu = workloads.random_velocity(shape, 12, amplitude=1.0)
    v, vu = direction(case, phi, 13)
    s = solver(gpu, case)
    s.set_state(phi, u)
    gphi, gu, gp = s.stage_adjoint(lphi, lu)
    h = 1e-5
    fp = stage_out(s, phi + h * v, [u[a] + h * vu[a] for a in range(dim)])
    fm = stage_out(s, phi - h * v, [u[a] - h * vu[a] for a in range(dim)])
    jv = [(fp[0] - fm[0]) / (2 * h)] + [(fp[1][a] - fm[1][a]) / (2 * h) for a in range(dim)]
    lhs = dot([lphi] + lu, jv)
    rhs = dot([gphi] + gu, [v] + vu)
    say(f"  <l, J v> {lhs:.12e}  <J^T l, v> {rhs:.12e}  rel {abs(lhs - rhs) / abs(lhs):.2e}")
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs)
    # parameters: sigma (absolute step) and eps (relative step)
    for k, name in enumerate(("sigma", "eps")):
        base = getattr(case, name)
        dh = 1e-5 if name == "sigma" else 1e-5 * base
        outs = []
        for sgn in (1, -1):
            kw = {"sigma": base + sgn * dh} if name == "sigma" else {"eps": base + sgn * dh}
            s2 = solver(gpu, case, adjoint=0, **kw)
            outs.append(stage_out(s2, phi, u))
        jp = [(outs[0][0] - outs[1][0]) / (2 * dh)] + [(outs[0][1][a] - outs[1][1][a]) / (2 * dh)
                                                       for a in range(dim)]
        fd = dot([lphi] + lu, jp)
        say(f"  d/d{name}: FD {fd:.12e}  adjoint {gp[k]:.12e}  rel {abs(fd - gp[k]) / abs(fd):.2e}")
        assert abs(fd - gp[k]) <= 1e-6 * abs(fd)


def test_adjoint_needs_scratch(gpu):
    """A context created without params.adjoint refuses the adjoint calls."""
    case = small_case()
    s = solver(gpu, case, adjoint=0)
    s.init_droplet(case.center, case.semi_axes)
    with pytest.raises(gpu.TpfError) as e:
        s.tape_bytes(1)
    assert e.value.status == gpu.TPF_EINVAL


def loss_and_seed(case, phi_t, u_t, tgt, c_u=0.1):
    hd = case.h ** case.dim
    L = 0.5 * hd * float(np.sum((phi_t - tgt) ** 2)) + 0.5 * c_u * hd * sum(float(np.sum(x * x)) for x in u_t)
    return L, hd * (phi_t - tgt), [c_u * hd * x for x in u_t]


def target_of(ora, case):
    P = oparams(ora, case)
    rng = np.random.default_rng(1)
    xi = rng.normal(size=case.dim)
    ax = tuple(case.semi_axes[a] * (1 + 0.05 * xi[a]) for a in range(case.dim))
    return ora.init_droplet(P, case.center, ax)


def gpu_loss(gpu, case, phi0, u0, tgt, steps, dt, **kw):
    s = solver(gpu, case, adjoint=0, **kw)
    s.set_state(phi0, u0)
    s.step(dt, steps)
    phi, u, _ = s.get_state()
    return loss_and_seed(case, phi, u, tgt)[0]


def ora_loss(ora, case, phi0, u0, tgt, steps, dt, **kw):
    P = oparams(ora, case, **kw)
    phi, u, _ = ora.step(P, dt, steps, phi0, u0)
    return loss_and_seed(case, phi, u, tgt)[0]


STEP_CASES = [
    ("gpu", (32, 24), "CDI", "EB"), ("gpu", (32, 24), "SB", "CSF"), ("gpu", (32, 24), "ISODI", "LCSF"),
    ("gpu", (16, 12, 8), "CDI", "EB"), ("gpu", (16, 12, 8), "SB", "LCSF"),
    ("oracle", (24, 20), "CDI", "EB"), ("oracle", (24, 20), "ISODI", "CSF"), ("oracle", (24, 20), "SB", "LCSF"),
    ("oracle", (12, 10, 8), "ISODI", "EB"),
]


@pytest.mark.parametrize("reference,n,model,force", STEP_CASES)
def test_step_adjoint_against_finite_differences(gpu, ora, reference, n, model, force):
    case = small_case(n, model=model, force=force)
    dim = case.dim
    steps = 4 if reference == "gpu" else 3
    dt = case.dt(umax0=0.2)
    say(f"step adjoint vs {reference} central differences {case.n} {model} {force} x {steps}")
    phi0, u0 = state(ora, case, seed=3)
    tgt = target_of(ora, case)
    s = solver(gpu, case)
    s.set_state(phi0, u0)
    s.step(dt, steps)
    phi_t, u_t, _ = s.get_state()
    _, gphi, gu = loss_and_seed(case, phi_t, u_t, tgt)
    s.set_state(phi0, u0)
    g0, gu0, gp = s.step_adjoint(dt, steps, gphi, gu)
    v, vu = direction(case, phi0, 21)
    if reference == "gpu":
        L = lambda f, u, **kw: gpu_loss(gpu, case, f, u, tgt, steps, dt, **kw)
    else:
        L = lambda f, u, **kw: ora_loss(ora, case, f, u, tgt, steps, dt, **kw)
    h = 1e-4
    # phi0 direction, u0 direction
    fd_phi = (L(phi0 + h * v, u0) - L(phi0 - h * v, u0)) / (2 * h)
    ad_phi = float(np.vdot(g0.ravel(), v.ravel()))
    fd_u = (L(phi0, [u0[a] + h * vu[a] for a in range(dim)]) -
            L(phi0, [u0[a] - h * vu[a] for a in range(dim)])) / (2 * h)
    ad_u = dot(gu0, vu)
    fd_s = (L(phi0, u0, sigma=case.sigma + h) - L(phi0, u0, sigma=case.sigma - h)) / (2 * h)
    he = h * case.eps
    fd_e = (L(phi0, u0, eps=case.eps + he) - L(phi0, u0, eps=case.eps - he)) / (2 * he)
    for name, fd, ad in (("phi0.v", fd_phi, ad_phi), ("u0.v", fd_u, ad_u), ("sigma", fd_s, gp[0]),
                         ("eps", fd_e, gp[1])):
        rel = abs(fd - ad) / max(abs(fd), 1e-300)
        say(f"  {name}: FD {fd:.10e} adjoint {ad:.10e} rel {rel:.2e}")
        assert rel < 2e-5, name


@pytest.mark.parametrize("n,model,force,steps,every", [((32, 24), "CDI", "EB", 12, 5),
                                                       ((16, 12, 8), "SB", "CSF", 5, 2)])
def test_rollout_checkpoints_and_autograd(gpu, ora, n, model, force, steps, every):
    import torch
    from paper_2205_05835_amd import adjoint
    case = small_case(n, model=model, force=force)
    dim = case.dim
    dt = case.dt(umax0=0.2)
    say(f"autograd rollout {case.n} {model} {force} x {steps}, checkpoints every {every} vs one segment")
    phi0, u0 = state(ora, case, seed=4)
    tgt = torch.tensor(target_of(ora, case), device="cuda")
    params = gpu.params_for_case(case, poisson_rtol=1e-14, poisson_maxit=2000)
    hd = case.h ** dim
    grads = []
    for ev in (every, steps):
        f0 = torch.tensor(phi0, device="cuda", requires_grad=True)
        uu = [torch.tensor(x, device="cuda", requires_grad=True) for x in u0]
        sig = torch.tensor(case.sigma, dtype=torch.float64, requires_grad=True)
        eps = torch.tensor(case.eps, dtype=torch.float64, requires_grad=True)
        phi, u = adjoint.rollout(f0, uu, sig, eps, params, dt, steps, ev)
        loss = 0.5 * hd * ((phi - tgt) ** 2).sum() + 0.05 * hd * sum((x * x).sum() for x in u)
        loss.backward()
        grads.append([f0.grad.cpu().numpy()] + [x.grad.cpu().numpy() for x in uu] +
                     [float(sig.grad), float(eps.grad)])
    for k in range(1 + dim):
        scale = np.abs(grads[1][k]).max()
        assert np.abs(grads[0][k] - grads[1][k]).max() <= 1e-12 * scale, k
    for k in (1 + dim, 2 + dim):
        assert abs(grads[0][k] - grads[1][k]) <= 1e-12 * abs(grads[1][k]), k
    say(f"  dL/dsigma {grads[0][1 + dim]:.10e} dL/deps {grads[0][2 + dim]:.10e}")


@pytest.mark.parametrize("n,model,force", [((32, 24), "CDI", "EB"), ((16, 12, 8), "ISODI", "LCSF")])
def test_mixed_precision_adjoint(gpu, ora, n, model, force):
    case64 = small_case(n, model=model, force=force)
    case32 = small_case(n, precision="fp32_mixed", model=model, force=force)
    steps = 4
    dt = case64.dt(umax0=0.2)
    say(f"FP32-mixed adjoint vs FP64 adjoint {n} {model} {force}")
    phi0, u0 = state(ora, case64, seed=5)
    phi0 = phi0.astype(np.float32).astype(np.float64)
    u0 = [x.astype(np.float32).astype(np.float64) for x in u0]
    tgt = target_of(ora, case64)
    out = {}
    for name, case in (("fp64", case64), ("fp32", case32)):
        s = solver(gpu, case) if name == "fp64" else gpu.solver_for_case(case, adjoint=1)
        s.set_state(phi0, u0)
        s.step(dt, steps)
        phi_t, u_t, _ = s.get_state()
        _, gphi, gu = loss_and_seed(case, phi_t, u_t, tgt)
        s.set_state(phi0, u0)
        out[name] = s.step_adjoint(dt, steps, gphi, gu)
    e_phi = np.abs(out["fp32"][0] - out["fp64"][0]).max() / np.abs(out["fp64"][0]).max()
    e_s = abs(out["fp32"][2][0] - out["fp64"][2][0]) / abs(out["fp64"][2][0])
    e_e = abs(out["fp32"][2][1] - out["fp64"][2][1]) / abs(out["fp64"][2][1])
    say(f"  dL/dphi0 rel {e_phi:.2e}  dL/dsigma rel {e_s:.2e}  dL/deps rel {e_e:.2e}")
    assert e_phi < 1e-2 and e_s < 1e-2 and e_e < 1e-2
