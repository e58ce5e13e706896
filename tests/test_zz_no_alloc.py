"""The allocation-free apply (mfl_apply_noalloc) against the handle-based mfl_apply, through the
C ABI: two calls in a row, the second on a smaller mesh, FP64 within 1e-12 and FP32 within
2e-5 (relative, max norm), plus the host-side rejection of a mesh that needs more scratch
than the fixed array holds."""
import numpy as np
import pytest
import torch

import paper_1611_03029_amd as mfl
from paper_1611_03029_amd import _mfl
from seeded_inputs import gaussian_field, uniform_vector

pytestmark = pytest.mark.gpu


def rel_err(a, b):
    return (a.double() - b.double()).abs().max().item() / b.double().abs().max().item()


def run_case(k, nc, bc, with_kappa, seed):
    kap = np.exp(gaussian_field(nc ** 3, seed, 0.5)) if with_kappa else None
    ref = mfl.Problem(k, nc, kappa=kap, bc=bc)
    params = mfl.make_params(k, nc, bc=bc)
    kt = None if kap is None else torch.tensor(kap, device="cuda")
    for dtype, tol in ((torch.float64, 1e-12), (torch.float32, 2e-5)):
        u = torch.tensor(uniform_vector(ref.n_dofs, seed + 1), dtype=dtype, device="cuda")
        y_ref = ref.apply(u)
        y = torch.full_like(u, float("nan"))
        mfl.apply_noalloc(params, u, y, kappa=kt)
        torch.cuda.synchronize()
        err = rel_err(y, y_ref)
        print("noalloc Q%d %d^3 bc=%d kappa=%s %s: rel err %.2e" % (k, nc, bc, with_kappa, dtype, err), flush=True)
        assert err <= tol


def test_two_calls_second_smaller():
    run_case(4, 16, mfl.DIRICHLET, True, 800)
    run_case(3, 7, mfl.MIXED, False, 810)


def test_larger_after_smaller_and_tall_bricks():
    run_case(2, 5, mfl.DIRICHLET, False, 820)
    run_case(2, 40, mfl.MIXED, True, 830)


def test_rejects_mesh_beyond_scratch():
    params = mfl.make_params(6, 64)
    n, _, _ = mfl.query(params)
    u = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(mfl.MflError) as e:
        mfl.apply_noalloc(params, u, torch.empty_like(u))
    assert e.value.code == _mfl.MFL_EINVAL and "scratch" in str(e.value)
    with pytest.raises(mfl.MflError) as e:
        mfl.apply_noalloc(mfl.make_params(3, 4, geometry=mfl.CURVED), torch.zeros(13 ** 3, dtype=torch.float64,
                          device="cuda"), torch.zeros(13 ** 3, dtype=torch.float64, device="cuda"))
    assert e.value.code == _mfl.MFL_EUNSUPPORTED
