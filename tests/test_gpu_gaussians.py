"""GPU parity for mixed boundary conditions on (-1,1)^3 and the smooth-solution example
(three Gaussians, Sec. 4.3) against the oracle and the errors the paper prints.

Tolerances: FP64 operator and right-hand side within 1e-12 relative (max norm) of the
oracle; FP32 operator within 2e-5; solutions within 1e-8 of the oracle's; L2 errors of the
GPU solutions within 0.5% of the paper's values on resolved meshes (the oracle itself
reproduces them to that accuracy, tests/test_oracle_gaussians.py).
"""
import os

import numpy as np
import pytest
import torch

import paper_1611_03029_amd as mfl
from oracle import cg as o_cg
from oracle import gaussians as G
from oracle import mg as o_mg
from oracle.mesh import Box
from seeded_inputs import SEED_MIXED_BC, uniform_vector

pytestmark = pytest.mark.gpu
DEV = "cuda"
DOMAIN = dict(domain_lo=-1.0, domain_len=2.0)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_gaussian_errors.txt")


def paper_table():
    rows = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        k, nc, qit, fel2, dgit, dgl2 = line.split()
        rows[(int(k), int(nc))] = (int(qit), float(fel2))
    return rows


def rel_err(a, b):
    a = a.detach().cpu().numpy() if torch.is_tensor(a) else a
    b = b.detach().cpu().numpy() if torch.is_tensor(b) else b
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("k,nc", [(1, 6), (2, 5), (3, 4), (4, 3), (5, 3), (6, 2)])
@pytest.mark.parametrize("bc", ["mixed", "dirichlet"])
def test_apply_on_shifted_domain_matches_csr(k, nc, bc):
    bx = Box(nc, k, lo=-1.0, length=2.0)
    A = o_cg.assemble(bx, bc=bc)
    u = uniform_vector(bx.n_dofs, SEED_MIXED_BC)
    ref = A @ u
    prob = mfl.Problem(k, nc, bc=mfl.MIXED if bc == "mixed" else mfl.DIRICHLET, **DOMAIN)
    y = prob.apply(torch.tensor(u, device=DEV))
    assert rel_err(y, ref) <= 1e-12
    y32 = prob.apply(torch.tensor(u, dtype=torch.float32, device=DEV))
    assert rel_err(y32.double(), ref) <= 2e-5


@pytest.mark.parametrize("k,nc", [(1, 12), (2, 8), (3, 6), (4, 4), (5, 3)])
def test_rhs_gaussians_matches_oracle(k, nc):
    bx = G.box(nc, k)
    ref = G.rhs(bx)
    prob = mfl.Problem(k, nc, bc=mfl.MIXED, **DOMAIN)
    b = prob.rhs_gaussians()
    assert rel_err(b, ref) <= 1e-12


def test_rhs_gaussians_with_dirichlet_everywhere():
    bx = G.box(6, 3)
    ref = G.rhs(bx, bc="dirichlet")
    prob = mfl.Problem(3, 6, bc=mfl.DIRICHLET, **DOMAIN)
    assert rel_err(prob.rhs_gaussians(), ref) <= 1e-12


def test_rhs_gaussians_rejects_curved_meshes():
    with pytest.raises(mfl.MflError) as e:
        mfl.Problem(2, 4, geometry=mfl.CURVED).rhs_gaussians()
    assert e.value.code == mfl._mfl.MFL_EUNSUPPORTED


@pytest.mark.parametrize("prec", [mfl.F64, mfl.F32])
def test_mixed_multigrid_solve_matches_oracle(prec):
    k, nc = 2, 8
    bx, u_direct = G.solve_direct(nc, k)
    ref = o_mg.solve(nc, k, b=G.rhs(bx), tol=1e-10, bc="mixed", **{"lo": -1.0, "length": 2.0})
    prob = mfl.Problem(k, nc, bc=mfl.MIXED, build_mg=True, mg_precision=prec, **DOMAIN)
    lev = prob.level_info(-1)
    assert abs(lev["lambda_max"] - ref["mg"].levels[-1]["lambda"]) <= 1e-10 * lev["lambda_max"]
    u, its, res = prob.solve(prob.rhs_gaussians(), rtol=1e-10, maxit=50)
    assert res <= 1e-10
    if prec == mfl.F64:
        assert its == ref["iterations"]
    else:
        assert abs(its - ref["iterations"]) <= 1
    assert rel_err(u, u_direct) <= 1e-8


@pytest.mark.parametrize("k,nc", [(2, 32), (3, 32), (4, 32), (5, 32), (2, 64)])
def test_l2_error_matches_paper_at_scale(k, nc):
    """GMG-PCG on the GPU at the paper's tolerance (1e-9) reproduces the paper's iteration
    counts within one and, solved further, its printed L2 errors."""
    qit, fel2 = paper_table()[(k, nc)]
    prob = mfl.Problem(k, nc, bc=mfl.MIXED, build_mg=True, mg_precision=mfl.F32, **DOMAIN)
    b = prob.rhs_gaussians()
    _, its, _ = prob.solve(b, rtol=1e-9, maxit=50)
    assert abs(its - qit) <= 1, (its, qit)
    u, _, res = prob.solve(b, rtol=1e-13, maxit=100)
    assert res <= 1e-13
    bx = G.box(nc, k)
    err = o_cg.l2_error(bx, u.cpu().numpy(), exact=G.solution)
    print("k=%d Nc=%d iterations %d (paper %d) L2 error %.5e (paper %.4e)" % (k, nc, its, qit, err, fel2))
    assert abs(err - fel2) <= 5e-3 * fel2
