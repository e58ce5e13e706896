"""More multigrid parity cases against the oracle: curved meshes, high degree, a one-cell
coarsest level, FP32 cycles at higher degree, and SIPG at high degree.

Tolerances as in test_gpu_cg.py: solutions within 1e-8 of the oracle's, FP64 multigrid
iteration counts equal to the oracle's (FP32 cycles within one).
"""
import numpy as np
import pytest
import torch

import paper_1611_03029_amd as mfl
from oracle import dgmg, mg as o_mg
from oracle import gaussians as G

pytestmark = pytest.mark.gpu


def rel_err(a, b):
    a = a.detach().cpu().numpy() if torch.is_tensor(a) else a
    return float(np.abs(a - b).max() / np.abs(b).max())


def check(prob, b, ref, prec):
    x, its, res = prob.solve(b, rtol=1e-10, maxit=100)
    assert res <= 1e-10
    if prec == mfl.F64:
        assert its == ref["iterations"], (its, ref["iterations"])
    else:
        assert abs(its - ref["iterations"]) <= 1, (its, ref["iterations"])
    assert rel_err(x, ref["x"]) <= 1e-8


@pytest.mark.parametrize("prec", [mfl.F64, mfl.F32])
def test_curved_mesh_multigrid(prec):
    k, nc = 3, 8
    ref = o_mg.solve(nc, k, curve_amp=0.1, tol=1e-10)
    prob = mfl.Problem(k, nc, geometry=mfl.CURVED, curve_amp=0.1, build_mg=True, mg_precision=prec)
    lev = prob.level_info(-1)
    assert abs(lev["lambda_max"] - ref["mg"].levels[-1]["lambda"]) <= 1e-10 * lev["lambda_max"]
    check(prob, prob.rhs_sine(), ref, prec)


@pytest.mark.parametrize("k", [6])
def test_high_degree_multigrid(k):
    nc = 4
    ref = o_mg.solve(nc, k, tol=1e-10)
    prob = mfl.Problem(k, nc, build_mg=True)
    check(prob, prob.rhs_sine(), ref, mfl.F64)


@pytest.mark.parametrize("prec", [mfl.F64, mfl.F32])
def test_one_cell_coarsest_level(prec):
    k, nc = 3, 8
    bx = G.box(nc, k)
    b = G.rhs(bx)
    ref = o_mg.solve(nc, k, b=b, tol=1e-10, min_cells=1, bc="mixed", lo=-1.0, length=2.0)
    prob = mfl.Problem(k, nc, build_mg=True, mg_precision=prec, min_level_cells=1, bc=mfl.MIXED,
                       domain_lo=-1.0, domain_len=2.0)
    assert prob.num_levels == 4
    c0 = prob.level_info(0)
    assert c0["coarse_steps"] == ref["mg"].levels[0]["steps"]
    check(prob, prob.rhs_gaussians(), ref, prec)


def test_fp32_cycle_at_degree_six():
    k, nc = 6, 4
    ref = o_mg.solve(nc, k, tol=1e-10)
    prob = mfl.Problem(k, nc, build_mg=True, mg_precision=mfl.F32)
    check(prob, prob.rhs_sine(), ref, mfl.F32)


@pytest.mark.parametrize("k", [5])
def test_sipg_multigrid_high_degree(k):
    nc = 4
    dg = G.dg_box(nc, k)
    b = G.dg_rhs(dg)
    ref = dgmg.solve(nc, k, b, c_pen=3.0, tol=1e-10, bc="mixed", lo=-1.0, length=2.0, jacobi_basis="gll")
    prob = mfl.Problem(k, nc, disc=mfl.SIPG, bc=mfl.MIXED, build_mg=True, penalty_factor=3.0,
                       domain_lo=-1.0, domain_len=2.0)
    check(prob, prob.rhs_gaussians(), ref, mfl.F64)
