"""Multigrid parity against the oracle at the degrees the solver workload is timed at, and the
preconditioner of the adjoint workload (Sec. 4.1).

- CG Q4 and Q5 on 8^3 cells (levels 8, 4, 2): one FP64 V-cycle within 1e-9 of the oracle's;
  PCG solutions within 1e-8 with FP64 and FP32 cycles, equal iteration counts with the FP64
  cycle and within one with the FP32 cycle.
- A seeded lognormal cellwise kappa (sigma 0.5; coarse levels take the mean of the 8 children)
  at Q3, Q4 and Q5 on 8^3 cells: the same bars, so the coarse-level kappa of every level is
  compared with the oracle's.
- Transfers for k = 1..8: prolongation and restriction equal the oracle's P and P^T (1e-13).
"""
import functools

import numpy as np
import pytest
import torch

import paper_1611_03029_amd as mfl
from oracle import mg as o_mg
from oracle.mesh import Box
from seeded_inputs import gaussian_field, uniform_vector

pytestmark = pytest.mark.gpu


def rel_err(a, b):
    a = a.detach().cpu().numpy() if torch.is_tensor(a) else a
    return float(np.abs(a - b).max() / np.abs(b).max())


def kappa_of(case):
    return None if case == "unit" else np.exp(gaussian_field(8 ** 3, 5, 0.5))


@functools.lru_cache(maxsize=None)
def oracle_solve(k, case):
    print("oracle GMG-PCG Q%d 8^3 kappa=%s" % (k, case), flush=True)
    return o_mg.solve(8, k, kappa=kappa_of(case), tol=1e-10)


CASES = [(4, "unit"), (5, "unit"), (3, "lognormal"), (4, "lognormal"), (5, "lognormal")]


@pytest.mark.parametrize("k,case", CASES)
def test_vcycle_fp64(k, case):
    ref = oracle_solve(k, case)
    mg = ref["mg"]
    prob = mfl.Problem(k, 8, kappa=kappa_of(case), build_mg=True)
    assert prob.num_levels == len(mg.levels) == 3
    for l, lev in enumerate(mg.levels):
        info = prob.level_info(l)
        if l == 0:
            assert abs(info["coarse_lmin"] - lev["lmin"]) <= 1e-10 * lev["lmax"]
            assert abs(info["coarse_lmax"] - lev["lmax"]) <= 1e-10 * lev["lmax"]
            assert info["coarse_steps"] == lev["steps"]
        else:
            assert abs(info["lambda_max"] - lev["lambda"]) <= 1e-10 * lev["lambda"]
    r = uniform_vector(prob.n_dofs, 500 + k)
    r[mg.levels[-1]["box"].boundary_mask()] = 0.0
    z = prob.vcycle(torch.tensor(r, device="cuda"))
    assert rel_err(z, mg.vcycle(r)) <= 1e-9


@pytest.mark.parametrize("prec", [mfl.F64, mfl.F32])
@pytest.mark.parametrize("k,case", CASES)
def test_pcg(k, case, prec):
    ref = oracle_solve(k, case)
    prob = mfl.Problem(k, 8, kappa=kappa_of(case), build_mg=True, mg_precision=prec)
    x, its, res = prob.solve(prob.rhs_sine(), rtol=1e-10, maxit=100)
    assert res <= 1e-10
    if prec == mfl.F64:
        assert its == ref["iterations"], (its, ref["iterations"])
    else:
        assert abs(its - ref["iterations"]) <= 1, (its, ref["iterations"])
    assert rel_err(x, ref["x"]) <= 1e-8


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8])
def test_transfer_matches_oracle_embedding(k):
    nf = 8 if k <= 4 else 4
    prob = mfl.Problem(k, nf, build_mg=True, min_level_cells=nf // 2 if k > 4 else 2)
    lev = prob.num_levels - 1
    fine, coarse = Box(nf, k), Box(nf // 2, k)
    P = o_mg.prolongation(coarse, fine)
    uc = uniform_vector(coarse.n_dofs, 11 + k)
    uf = uniform_vector(fine.n_dofs, 12 + k)
    out = torch.tensor(uf.copy(), device="cuda")
    prob.transfer(lev, 0, torch.tensor(uc, device="cuda"), out)
    assert rel_err(out, uf + P @ uc) <= 1e-13
    rc = torch.empty(coarse.n_dofs, dtype=torch.float64, device="cuda")
    prob.transfer(lev, 1, torch.tensor(uf, device="cuda"), rc)
    assert rel_err(rc, P.T @ uf) <= 1e-13


@pytest.mark.parametrize("k,nf", [(1, 128), (2, 64), (3, 64), (4, 64), (5, 64)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_transfer_rows_full_size(k, nf, dtype):
    """Transfers on a fine level large enough that a work-group takes a row of coarse cells
    (the meshes above take one cell per work-group), checked by properties that hold at any
    size, with mixed boundary conditions (Dirichlet DoFs masked on both levels):
    - prolongation reproduces, at the fine nodes, a polynomial of degree k per direction that
      vanishes on the Dirichlet faces (it lies in the coarse space);
    - restriction is its transpose: <P c, f> = <c, P^T f> for seeded random c and f."""
    print("transfer rows Q%d fine %d^3 %s" % (k, nf, dtype), flush=True)
    prob = mfl.Problem(k, nf, bc=mfl.MIXED, build_mg=True)
    lev = prob.num_levels - 1
    fine, coarse = Box(nf, k), Box(nf // 2, k)
    rng = np.random.default_rng(300 + k)

    def poly_values(box, coef):
        # prod_d (1 - x_d) r_d(x_d), r_d of degree k - 1: zero on the faces x_d = 1
        x = box.node_coords_1d()
        q = [torch.tensor((1 - x) * np.polyval(coef[d], x), device="cuda") for d in range(3)]
        return (q[2][:, None, None] * q[1][None, :, None] * q[0][None, None, :]).reshape(-1)

    coef = rng.uniform(-1, 1, (3, k))
    pc, pf = poly_values(coarse, coef), poly_values(fine, coef)
    out = torch.zeros(fine.n_dofs, dtype=dtype, device="cuda")
    prob.transfer(lev, 0, pc.to(dtype), out)
    tol = 1e-12 if dtype == torch.float64 else 2e-6
    assert (out.double() - pf).abs().max().item() <= tol * pf.abs().max().item()

    c = torch.tensor(uniform_vector(coarse.n_dofs, 320 + k), device="cuda").to(dtype)
    f = torch.tensor(uniform_vector(fine.n_dofs, 330 + k), device="cuda").to(dtype)
    pcv = torch.zeros(fine.n_dofs, dtype=dtype, device="cuda")
    prob.transfer(lev, 0, c, pcv)
    rf = torch.empty(coarse.n_dofs, dtype=dtype, device="cuda")
    prob.transfer(lev, 1, f, rf)
    lhs = torch.dot(pcv.double(), f.double()).item()
    rhs = torch.dot(c.double(), rf.double()).item()
    scale = (pcv.double().abs() * f.double().abs()).sum().item()
    assert abs(lhs - rhs) <= (1e-13 if dtype == torch.float64 else 1e-6) * scale
