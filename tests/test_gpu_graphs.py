"""The V-cycle captured as a HIP graph (use_graphs, the default) against the same cycle
launched kernel by kernel: every replay, with eager work and synchronizations between the
replays, matches the eager result (the CG restriction adds with atomics, so the order of
additions may differ: relative 1e-13), and PCG solves agree.
"""
import numpy as np
import pytest
import torch

import paper_1611_03029_amd as mfl
from seeded_inputs import SEED_MIXED_BC, uniform_vector

pytestmark = pytest.mark.gpu
DEV = "cuda"
DOMAIN = dict(domain_lo=-1.0, domain_len=2.0)

CASES = {
    "cg_dirichlet": dict(degree=3, cells_per_dim=8),
    "cg_mixed": dict(degree=2, cells_per_dim=8, bc=mfl.MIXED, **DOMAIN),
    "sipg_mixed": dict(degree=3, cells_per_dim=4, disc=mfl.SIPG, bc=mfl.MIXED, penalty_factor=3.0, **DOMAIN),
}


def rel(a, b):
    return ((a - b).abs().max() / b.abs().max()).item()


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", [mfl.F64, mfl.F32])
def test_graph_replays_match_eager_cycles(case, prec):
    kw = dict(CASES[case])
    k, nc = kw.pop("degree"), kw.pop("cells_per_dim")
    g = mfl.Problem(k, nc, build_mg=True, mg_precision=prec, use_graphs=True, **kw)
    e = mfl.Problem(k, nc, build_mg=True, mg_precision=prec, use_graphs=False, **kw)
    tol = 1e-13 if prec == mfl.F64 else 1e-6
    for rep in range(4):
        r = torch.tensor(uniform_vector(g.n_dofs, SEED_MIXED_BC + rep), device=DEV)
        zg = g.vcycle(r)
        # eager work between the replays, on the same stream and after a synchronization
        torch.cuda.synchronize()
        y = g.apply(r)
        ze = e.vcycle(r)
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
        assert rel(zg, ze) <= tol, (rep, rel(zg, ze))


@pytest.mark.parametrize("case", list(CASES))
def test_graph_solves_match_eager_solves(case):
    kw = dict(CASES[case])
    k, nc = kw.pop("degree"), kw.pop("cells_per_dim")
    g = mfl.Problem(k, nc, build_mg=True, use_graphs=True, **kw)
    e = mfl.Problem(k, nc, build_mg=True, use_graphs=False, **kw)
    b = torch.tensor(uniform_vector(g.n_dofs, SEED_MIXED_BC), device=DEV)
    for _ in range(2):
        ug, itg, resg = g.solve(b, rtol=1e-10, maxit=100)
        ue, ite, rese = e.solve(b, rtol=1e-10, maxit=100)
        assert itg == ite
        assert rel(ug, ue) <= 1e-9


def test_graph_is_rebuilt_when_kappa_changes():
    k, nc = 2, 8
    g = mfl.Problem(k, nc, build_mg=True, use_graphs=True)
    e = mfl.Problem(k, nc, build_mg=True, use_graphs=False)
    r = torch.tensor(uniform_vector(g.n_dofs, SEED_MIXED_BC), device=DEV)
    g.vcycle(r)
    kappa = np.exp(np.linspace(-1.0, 1.0, g.n_cells))
    g.set_kappa(kappa)
    e.set_kappa(kappa)
    assert rel(g.vcycle(r), e.vcycle(r)) <= 1e-13


@pytest.mark.parametrize("prec", [mfl.F64, mfl.F32])
@pytest.mark.parametrize("k,nc", [(3, 8), (4, 64)])
def test_caller_vectors_off_16_byte_alignment(k, nc, prec):
    """Caller vectors 8 bytes off a 16-byte boundary take the vector kernels' one-entry-per-lane
    forms (the work vectors keep the four-entry forms): cycles and solves agree with those
    on aligned vectors.  On 64^3 cells (257^3 DoFs, one DoF past a multiple of four) the
    fine level's smoother updates run four DoFs per lane, the last one of the cycle on an
    unaligned output one per lane."""
    print("unaligned caller vectors Q%d %d^3 precision %d" % (k, nc, prec), flush=True)
    e = mfl.Problem(k, nc, build_mg=True, mg_precision=prec, use_graphs=False)
    n = e.n_dofs
    r = torch.tensor(uniform_vector(n, SEED_MIXED_BC), device=DEV)
    rbuf = torch.empty(n + 1, dtype=torch.float64, device=DEV)
    zbuf = torch.empty(n + 1, dtype=torch.float64, device=DEV)
    r_off, z_off = rbuf[1:], zbuf[1:]
    r_off.copy_(r)
    assert r_off.data_ptr() % 16 == 8 and z_off.data_ptr() % 16 == 8
    z = e.vcycle(r)
    e.vcycle(r_off, z_off)
    tol = 1e-13 if prec == mfl.F64 else 1e-6
    assert rel(z_off, z) <= tol
    x, it, res = e.solve(r, rtol=1e-10)
    e.solve(r, rtol=1e-10, x=z_off)
    assert rel(z_off, x) <= 1e-9
    assert res <= 1e-10
