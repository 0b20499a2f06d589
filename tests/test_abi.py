"""CPU checks of the C ABI: the library loads, exports every function that
include/tpf.h declares, and validates parameters without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def tpf():
    from paper_2205_05835_amd import tpf as t
    if not os.path.exists(t.LIB_PATH):
        pytest.fail("libtpf.so is not built: run __graft_entry__.build()")
    return t


def declared_functions():
    src = open(os.path.join(ROOT, "include", "tpf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tpf_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_binding_exports(tpf):
    assert declared_functions() == sorted(tpf.EXPORTS)


def test_library_exports_every_declared_symbol(tpf):
    L = tpf.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert L.tpf_version().decode().startswith("tpf")
    assert L.tpf_profile_classes() > 0


def test_struct_layout_matches_header(tpf):
    # tpf_params: 4 int32 + 1 double ... ; check a few offsets against C rules
    P = tpf.tpf_params
    assert P.length.offset == 16
    assert P.sigma.offset == 40
    assert P.poisson_maxit.offset == 120 and P.adjoint.offset == 128 and P.walls.offset == 132
    assert ctypes.sizeof(P) == 136
    D = tpf.tpf_diag
    assert D.poisson_outer.offset == 104 and ctypes.sizeof(D) == 112
    O = tpf.tpf_implicit_opts
    assert O.newton_maxit.offset == 16 and ctypes.sizeof(O) == 24
    info = tpf.tpf_implicit_info
    assert info.residual.offset == 8 and info.krylov_total.offset == 24 and ctypes.sizeof(info) == 32


@pytest.mark.parametrize("bad", [
    dict(eps=-1.0), dict(rho1=0.0), dict(rho2=-2.0), dict(sigma=-1.0), dict(model=7), dict(force=-1),
    dict(precision=5), dict(mg_levels=-1)])
def test_invalid_parameters_rejected(tpf, bad):
    p = tpf.make_params((32, 32), **{k: v for k, v in bad.items() if k in ("eps", "sigma", "rho1", "rho2", "mg_levels")})
    for k, v in bad.items():
        if k in ("model", "force", "precision"):
            setattr(p, k, v)
    with pytest.raises(tpf.TpfError) as e:
        tpf.workspace_bytes(p)
    assert e.value.status == tpf.TPF_EINVAL
    assert tpf.lib().tpf_last_error().decode() != ""


def test_invalid_dim_rejected(tpf):
    p = tpf.make_params((32, 32))
    p.dim = 4
    with pytest.raises(tpf.TpfError):
        tpf.workspace_bytes(p)


def test_workspace_size_scales(tpf):
    small = tpf.workspace_bytes(tpf.make_params((64, 64)))
    big = tpf.workspace_bytes(tpf.make_params((128, 128)))
    mixed = tpf.workspace_bytes(tpf.make_params((128, 128), precision="fp32_mixed"))
    assert 3.5 < big / small < 4.5
    assert mixed < big
    b3 = tpf.workspace_bytes(tpf.make_params((256, 256, 256), precision="fp32_mixed"))
    # about 45 FP32-equivalent fields of 64 MiB at 256^3
    assert 2.5 * 2 ** 30 < b3 < 4 * 2 ** 30


def test_create_rejects_null_or_small_workspace(tpf):
    p = tpf.make_params((16, 16))
    ctx = ctypes.c_void_p()
    st = tpf.lib().tpf_create(ctypes.byref(p), None, 0, None, ctypes.byref(ctx))
    assert st == tpf.TPF_EINVAL
    st = tpf.lib().tpf_create(ctypes.byref(p), ctypes.c_void_p(256), 16, None, ctypes.byref(ctx))
    assert st == tpf.TPF_ENOMEM
    assert "workspace too small" in tpf.lib().tpf_last_error().decode()


def test_batch_workspace_validation(tpf):
    """Batched cases must be 2D and share one precision; the workspace grows
    with the cases."""
    a = tpf.make_params((32, 32))
    b = tpf.make_params((64, 48))
    n1 = tpf.batch_workspace_bytes([a])
    n2 = tpf.batch_workspace_bytes([a, b])
    assert n2 > n1 > 0
    with pytest.raises(tpf.TpfError):
        tpf.batch_workspace_bytes([a, tpf.make_params((8, 8, 8))])
    with pytest.raises(tpf.TpfError):
        tpf.batch_workspace_bytes([a, tpf.make_params((32, 32), precision="fp32_mixed")])
    assert len(tpf.batch_configs()) == tpf.lib().tpf_batch_configs() >= 1
    for threads, lds in tpf.batch_configs():
        # LDS per workgroup on gfx950: 160 KiB, less the kernel's reduction scratch
        assert threads in (256, 512, 1024) and 0 <= lds <= 160 * 1024 - 1024


def test_grid_size_limits(tpf):
    """n >= 2 per axis and at most 2^29 cells (32-bit byte offsets of FP64 fields)."""
    for n in [(1, 16), (16, 1), (8, 8, 1)]:
        with pytest.raises(tpf.TpfError):
            tpf.workspace_bytes(tpf.make_params(n))
    with pytest.raises(tpf.TpfError) as e:
        tpf.workspace_bytes(tpf.make_params((1024, 1024, 1024), precision="fp32_mixed"))
    assert "too large" in str(e.value)
    assert tpf.workspace_bytes(tpf.make_params((512, 512, 512), precision="fp32_mixed")) > 0
    assert tpf.workspace_bytes(tpf.make_params((2, 2))) > 0


def test_adjoint_scratch_is_opt_in(tpf):
    """params.adjoint = 1 adds 11 + 8 dim FP64 fields of N values (plus 256
    bytes of accumulators) to the workspace; other values are rejected."""
    for n in [(64, 48), (16, 12, 8)]:
        N = 1
        for x in n:
            N *= x
        base = tpf.workspace_bytes(tpf.make_params(n))
        adj = tpf.workspace_bytes(tpf.make_params(n, adjoint=1))
        fields = 11 + 8 * len(n)
        stride = (N * 8 + 255) // 256 * 256
        assert fields * stride <= adj - base <= fields * stride + 512
    with pytest.raises(tpf.TpfError) as e:
        tpf.workspace_bytes(tpf.make_params((32, 32), adjoint=2))
    assert e.value.status == tpf.TPF_EINVAL


def test_walls_validation(tpf):
    """params.walls: one bit per axis of the grid; batched cases only (the
    single-case calls reject any wall)."""
    for bad in (-1, 4, 8):
        with pytest.raises(tpf.TpfError) as e:
            tpf.batch_workspace_bytes([tpf.make_params((32, 32), walls=bad)])
        assert e.value.status == tpf.TPF_EINVAL
    with pytest.raises(tpf.TpfError):
        tpf.batch_workspace_bytes([tpf.make_params((8, 8, 8), walls=4)])
    ok = tpf.batch_workspace_bytes([tpf.make_params((32, 32), walls=w) for w in range(4)])
    assert ok == tpf.batch_workspace_bytes([tpf.make_params((32, 32))] * 4)
    for n, w in (((32, 32), 1), ((16, 16, 16), 4)):
        assert tpf.workspace_bytes(tpf.make_params(n, walls=w)) == tpf.workspace_bytes(tpf.make_params(n))
        # the adjoint calls need a periodic box
        with pytest.raises(tpf.TpfError) as e:
            tpf.workspace_bytes(tpf.make_params(n, walls=w, adjoint=1))
        assert e.value.status == tpf.TPF_EINVAL and "periodic" in str(e.value)
