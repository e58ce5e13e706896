"""C ABI checks that need no GPU: the library loads, exports every declared entry
point, and rejects invalid parameters with MFL_EINVAL before touching a device."""
import ctypes
import os
import re

import pytest

import paper_1611_03029_amd as mfl
from paper_1611_03029_amd import _mfl

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "mfl.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mfl_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 15
    lib = mfl.lib()
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_mfl.SIGNATURES)


def test_default_params():
    p = _mfl.Params()
    assert mfl.lib().mfl_default_params(ctypes.byref(p)) == 0
    assert (p.degree, p.cheb_degree, p.eig_iters) == (2, 5, 15)
    assert abs(p.cheb_lo - 0.06) < 1e-15 and abs(p.cheb_hi - 1.2) < 1e-15
    assert abs(p.coarse_tol - 1e-3) < 1e-18


@pytest.mark.parametrize("k,Nc,disc,dofs", [(2, 8, mfl.CG, 17 ** 3), (4, 64, mfl.CG, 257 ** 3),
                                            (3, 32, mfl.SIPG, 32 ** 3 * 64), (5, 32, mfl.SIPG, 7077888)])
def test_query_dof_counts(k, Nc, disc, dofs):
    n, c, ws = mfl.query(mfl.make_params(k, Nc, disc=disc))
    assert n == dofs and c == Nc ** 3 and ws > 0


def test_workspace_scales_with_geometry_and_multigrid():
    cart = mfl.query(mfl.make_params(4, 64))[2]
    curved = mfl.query(mfl.make_params(4, 64, geometry=mfl.CURVED, metric_mode=mfl.METRIC_STORED))[2]
    # stored metric: FP64 + FP32 copies of 6 metric entries per quadrature point
    assert curved - cart >= 262144 * 125 * 6 * 12
    # on the fly: FP64 + FP32 node displacements only (one value per DoF)
    otf = mfl.query(mfl.make_params(4, 64, geometry=mfl.CURVED, metric_mode=mfl.METRIC_ON_THE_FLY))[2]
    assert 257 ** 3 * 12 <= otf - cart < 257 ** 3 * 12 + 4096
    assert mfl.query(mfl.make_params(4, 64, geometry=mfl.CURVED))[2] == otf   # AUTO, cellwise kappa
    cos = mfl.query(mfl.make_params(4, 64, geometry=mfl.CURVED, kappa_field=mfl.KAPPA_COSINE))[2]
    assert cos == curved                                                       # AUTO, kappa field
    assert mfl.query(mfl.make_params(4, 64, metric_mode=mfl.METRIC_STORED))[2] == cart   # Cartesian: no metric
    mg = mfl.query(mfl.make_params(4, 64, build_mg=True))[2]
    assert mg > cart


@pytest.mark.parametrize("kw", [dict(degree=0), dict(degree=9), dict(cells_per_dim=0),
                                dict(disc=2), dict(geometry=5), dict(bc=3), dict(bc=-1), dict(mg_precision=7),
                                dict(disc=mfl.SIPG, geometry=mfl.CURVED),
                                dict(disc=mfl.SIPG, build_mg=True, bc=mfl.NEUMANN),
                                dict(cells_per_dim=12, build_mg=True, min_level_cells=2),
                                dict(build_mg=True, bc=mfl.NEUMANN),
                                dict(geometry=mfl.CURVED, curve_amp=0.5),
                                dict(build_mg=True, cheb_lo=1.5),
                                dict(domain_len=0.0), dict(domain_len=-2.0),
                                dict(dg_jacobi_basis=2),
                                dict(domain_lo=float("nan")),
                                dict(geometry=mfl.CURVED, domain_lo=-1.0, domain_len=2.0),
                                dict(kappa_field=2),
                                dict(kappa_field=mfl.KAPPA_COSINE),
                                dict(kappa_field=mfl.KAPPA_COSINE, disc=mfl.SIPG),
                                dict(kappa_field=mfl.KAPPA_COSINE, geometry=mfl.CURVED, kappa_field_amp=-1.0),
                                dict(kappa_field=mfl.KAPPA_COSINE, geometry=mfl.CURVED,
                                     kappa_field_amp=float("inf")),
                                dict(metric_mode=3), dict(metric_mode=-1),
                                dict(geometry=mfl.CURVED, kappa_field=mfl.KAPPA_COSINE,
                                     metric_mode=mfl.METRIC_ON_THE_FLY),
                                dict(degree=8, cells_per_dim=4, build_mg=True, min_level_cells=4),
                                dict(degree=7, cells_per_dim=4, build_mg=True, min_level_cells=4,
                                     disc=mfl.SIPG)])
def test_invalid_params_rejected(kw):
    base = dict(degree=2, cells_per_dim=8)
    base.update(kw)
    deg, nc = base.pop("degree"), base.pop("cells_per_dim")
    with pytest.raises(mfl.MflError) as e:
        mfl.query(mfl.make_params(deg, nc, **base))
    assert e.value.code == _mfl.MFL_EINVAL


def test_setup_rejects_null_workspace_without_gpu():
    p = mfl.make_params(2, 8)
    h = ctypes.c_void_p()
    rc = mfl.lib().mfl_setup(ctypes.byref(p), None, 0, None, None, ctypes.byref(h))
    assert rc == _mfl.MFL_EINVAL and not h.value
    assert b"workspace" in mfl.lib().mfl_last_error()
    rc = mfl.lib().mfl_setup(ctypes.byref(p), ctypes.c_void_p(1024 + 8), 1 << 20, None, None, ctypes.byref(h))
    assert rc == _mfl.MFL_EINVAL and b"aligned" in mfl.lib().mfl_last_error()
    rc = mfl.lib().mfl_setup(ctypes.byref(p), ctypes.c_void_p(1024), 16, None, None, ctypes.byref(h))
    assert rc == _mfl.MFL_EINVAL and b"too small" in mfl.lib().mfl_last_error()


def test_null_handle_rejected():
    assert mfl.lib().mfl_apply(None, -1, 0, None, None, None) == _mfl.MFL_EINVAL
    assert mfl.lib().mfl_destroy(None) == _mfl.MFL_EINVAL


def test_mixed_conditions_and_domain_accepted():
    n, c, ws = mfl.query(mfl.make_params(3, 8, bc=mfl.MIXED, build_mg=True, domain_lo=-1.0,
                                         domain_len=2.0))
    assert n == 25 ** 3 and c == 512 and ws > 0
    n2, _, ws2 = mfl.query(mfl.make_params(3, 8, bc=mfl.MIXED, disc=mfl.SIPG))
    assert n2 == 512 * 64 and ws2 > 0


def test_coarse_size_limit():
    """The coarsest level takes at most 20000 unknowns (CG: without the Dirichlet DoFs)."""
    # Q8 on 2^3 cells: 15^3 interior unknowns; Q6 on 3^3 cells: 17^3; both accepted
    for k, nc in ((8, 2), (6, 3)):
        mfl.query(mfl.make_params(k, nc, build_mg=True, min_level_cells=nc))
    # Q8 on 3^3 cells: 23^3 = 12167 accepted; SIPG Q5 on 4^3 cells: 13824 accepted
    mfl.query(mfl.make_params(8, 3, build_mg=True, min_level_cells=3, bc=mfl.MIXED))
    mfl.query(mfl.make_params(5, 4, build_mg=True, min_level_cells=4, disc=mfl.SIPG, bc=mfl.MIXED))


def test_kappa_field_accepted_on_curved_cg():
    n, c, ws = mfl.query(mfl.make_params(4, 8, geometry=mfl.CURVED, curve_amp=0.0,
                                         kappa_field=mfl.KAPPA_COSINE, build_mg=True))
    assert n == 33 ** 3 and ws > 0


def test_default_kappa_field():
    p = _mfl.Params()
    assert mfl.lib().mfl_default_params(ctypes.byref(p)) == 0
    assert p.kappa_field == mfl.KAPPA_CELLWISE and p.kappa_field_amp == 1e6
    assert p.metric_mode == mfl.METRIC_AUTO


@pytest.mark.parametrize("bad", ["cpu", "dtype", "size", "strided", "not_tensor"])
def test_check_vector_rejects_without_gpu(bad):
    """The binding validates every tensor the library writes through (output vectors of
    apply, vcycle, solve, adjoint_solve and transfer) before calling it."""
    import torch
    t = {"cpu": torch.zeros(10, dtype=torch.float64),
         "dtype": torch.zeros(10, dtype=torch.float32),
         "size": torch.zeros(9, dtype=torch.float64),
         "strided": torch.zeros(20, dtype=torch.float64)[::2],
         "not_tensor": [0.0] * 10}[bad]
    with pytest.raises(ValueError):
        mfl.check_vector(t, 10, torch.float64, "x")
