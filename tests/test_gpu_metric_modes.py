"""The two representations of the curved geometry (Sec. 3, non-affine cells): the metric
G_q = w det J J^{-1} J^{-T} stored per quadrature point at setup, and the metric formed on the
fly in every apply from the node displacements of the map x = X + d(X) (1,1,1).  Both against
the oracle's assembled operator (which evaluates the Jacobian of the isoparametric map at
every quadrature point, without either representation), and against each other at the
size the operator is timed at.

Bars: FP64 operator, diagonal and gradient within 1e-12 of the oracle; the two modes within
1e-13 of each other in FP64 and 2e-5 in FP32 at full size; multigrid solves of the two modes
with equal iteration counts and solutions within 1e-9.
"""
import numpy as np
import pytest
import torch

import paper_1611_03029_amd as mfl
from oracle import adjoint as o_adj
from oracle import cg as o_cg
from oracle.mesh import Box
from seeded_inputs import SEED_CG_Q4_CURVED, SEED_KAPPA_FIELD, gaussian_field, uniform_vector

pytestmark = pytest.mark.gpu
MODES = [mfl.METRIC_STORED, mfl.METRIC_ON_THE_FLY]


def rel_err(a, b):
    a = a.detach().cpu().numpy() if torch.is_tensor(a) else a
    b = b.detach().cpu().numpy() if torch.is_tensor(b) else b
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def t(x, dtype=torch.float64):
    return torch.as_tensor(np.asarray(x), dtype=dtype, device="cuda")


def kappa_field(n):
    return np.exp(gaussian_field(n, SEED_KAPPA_FIELD, 0.5))


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8])
def test_curved_apply_matches_oracle(k, mode):
    Nc = 4 if k <= 4 else 3
    print("curved apply Q%d %d^3 metric mode %d" % (k, Nc, mode), flush=True)
    box = Box(Nc, k, 0.1)
    kap = kappa_field(box.n_cells)
    prob = mfl.Problem(k, Nc, kappa=kap, geometry=mfl.CURVED, curve_amp=0.1, metric_mode=mode)
    u = uniform_vector(box.n_dofs, 40 + k)
    ref = o_cg.assemble(box, kap) @ u
    assert rel_err(prob.apply(t(u)), ref) <= 1e-12
    assert rel_err(prob.apply(t(u, torch.float32)).double(), ref) <= 2e-5


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("k,Nc", [(2, 6), (4, 4)])
def test_curved_mixed_conditions_match_oracle(k, Nc, mode):
    """Neumann lower faces (the node displacements there are not masked: the geometry is not
    a Dirichlet datum) and Dirichlet upper faces, FP64 and FP32."""
    box = Box(Nc, k, 0.1)
    kap = kappa_field(box.n_cells)
    prob = mfl.Problem(k, Nc, kappa=kap, geometry=mfl.CURVED, curve_amp=0.1, bc=mfl.MIXED, metric_mode=mode)
    u = uniform_vector(box.n_dofs, 50 + k)
    ref = o_cg.assemble(box, kap, bc="mixed") @ u
    assert rel_err(prob.apply(t(u)), ref) <= 1e-12
    assert rel_err(prob.apply(t(u, torch.float32)).double(), ref) <= 2e-5


@pytest.mark.parametrize("mode", MODES)
def test_curved_diagonal_and_gradient_match_oracle(mode):
    k, Nc = 3, 4
    box = Box(Nc, k, 0.1)
    kap = kappa_field(box.n_cells)
    prob = mfl.Problem(k, Nc, kappa=kap, geometry=mfl.CURVED, curve_amp=0.1, build_mg=True, metric_mode=mode)
    assert rel_err(prob.diagonal(), o_cg.assemble(box, kap).diagonal()) <= 1e-12
    u = uniform_vector(box.n_dofs, 31)
    lam = uniform_vector(box.n_dofs, 32)
    assert rel_err(prob.kappa_gradient(t(u), t(lam)), o_adj.gradient(box, u, lam)) <= 1e-12


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_modes_agree_at_full_size(dtype):
    """CG Q4 on 64^3 curved cells (257^3 DoFs): the applies of the two modes on the whole
    vector, and both against oracle rows computed one by one."""
    print("metric modes Q4 64^3 %s" % dtype, flush=True)
    u = uniform_vector(257 ** 3, SEED_CG_Q4_CURVED)
    ys = []
    for mode in MODES:
        prob = mfl.Problem(4, 64, geometry=mfl.CURVED, curve_amp=0.1, metric_mode=mode)
        ys.append(prob.apply(t(u, dtype)).double())
        del prob
        torch.cuda.empty_cache()
    tol = 1e-13 if dtype == torch.float64 else 2e-5
    assert (ys[0] - ys[1]).abs().max().item() <= tol * ys[0].abs().max().item()
    rows = np.random.default_rng(23).choice(257 ** 3, 60, replace=False)
    ref = o_cg.apply_rows(Box(64, 4, 0.1), u, rows)
    for y in ys:
        assert np.abs(y.cpu().numpy()[rows] - ref).max() <= (1e-12 if dtype == torch.float64 else 2e-5) * np.abs(ref).max()


def test_multigrid_solves_of_both_modes_agree():
    """Curved Q3 on 16^3 cells, FP32 V-cycle: the same iteration counts and solutions."""
    sols, its = [], []
    for mode in MODES:
        prob = mfl.Problem(3, 16, geometry=mfl.CURVED, curve_amp=0.1, build_mg=True, mg_precision=mfl.F32,
                           metric_mode=mode)
        x, it, res = prob.solve(prob.rhs_sine(), rtol=1e-10)
        assert res <= 1e-10
        sols.append(x)
        its.append(it)
    assert its[0] == its[1]
    assert (sols[0] - sols[1]).abs().max().item() <= 1e-9 * sols[0].abs().max().item()


def test_on_the_fly_needs_cellwise_kappa():
    with pytest.raises(mfl.MflError):
        mfl.Problem(4, 4, geometry=mfl.CURVED, kappa_field=mfl.KAPPA_COSINE, metric_mode=mfl.METRIC_ON_THE_FLY)
