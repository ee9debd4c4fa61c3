"""toeplitz_matvec_static (workspace in the library's static device array, no
allocation) against toeplitz_matvec (plan workspace) on the same plan and
inputs: the kernels are the same, so the results agree bit for bit.  Two calls
in a row, the second on a smaller input; a request beyond the static limit is
refused before any device work."""
import ctypes

import numpy as np
import pytest

import oracle
from synth import arrays as sa
from helpers import assert_parity, banner, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2506_04710_amd as tp
    tp.load()
    return torch


def _plan(prob, R):
    import paper_2506_04710_amd as tp
    return tp.Plan.create(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr,
                          prec="mixed", max_rhs=R, restart=4)


def _both(torch, plan, X, which):
    dt = torch.complex64 if which == "fp32" else torch.complex128
    xd = to_dev(X, dt)
    y_ws = plan.matvec(xd, which=which)
    y_st = plan.matvec_static(xd, which=which)
    torch.cuda.synchronize()
    return y_ws.cpu().numpy(), y_st.cpu().numpy()


# (Nx, Ny, b, Nr, R): the first call runs several columns on a larger plan
# (multi-column kernels), the second one column on a smaller plan (fused
# single-column kernel, half spectrum, mirror parts)
SEQUENCE = [(12, 10, 24, 44, 3), (4, 4, 16, 24, 1)]


@pytest.mark.parametrize("which", ["fp64", "fp32", "mixed"])
def test_static_matvec_matches_workspace_matvec(torch_cuda, which):
    for i, (Nx, Ny, b, Nr, R) in enumerate(SEQUENCE):
        banner(f"matvec_static {which} call {i} {(Nx, Ny, b, Nr, R)}")
        prob = sa.make_problem(Nx, Ny, b, Nr, 7100 + i)
        X = sa.rhs_random(prob, R)
        if which == "fp32":
            X = X.astype(np.complex64)
        plan = _plan(prob, R)
        y_ws, y_st = _both(torch_cuda, plan, X, which)
        assert np.array_equal(y_ws.view(np.uint8), y_st.view(np.uint8)), f"call {i}: results differ"
        tol = 1e-10 if which == "fp64" else 1e-5
        assert_parity(y_st.astype(np.complex128).reshape(R, -1), oracle.matvec(prob, X.astype(np.complex128)),
                      tol, N=prob.N, what=f"static {which} call {i}")


def test_static_matvec_refuses_beyond_limit(torch_cuda):
    import paper_2506_04710_amd as tp
    from paper_2506_04710_amd import _lib
    L = _lib.lib()
    limit = L.toeplitz_static_scratch_bytes()
    assert limit == 64 << 20
    # 20 x 20, b = 64, 40 columns: grids of 39 * 39 * 64 * 40 complex128 values, twice: 125 MB
    prob = sa.make_problem(20, 20, 64, 0, 7200)
    R = 40
    plan = _plan(prob, R)
    x = torch_cuda.zeros((R, prob.Nt), dtype=torch_cuda.complex128, device="cuda:0")
    y = torch_cuda.full((R, prob.Nt), 3.0, dtype=torch_cuda.complex128, device="cuda:0")
    st = L.toeplitz_matvec_static(plan._h, _lib.TP_FP64, ctypes.c_void_p(x.data_ptr()), prob.Nt,
                                  ctypes.c_void_p(y.data_ptr()), prob.Nt, R, None)
    assert st == _lib.TP_E_INVAL
    assert b"static scratch" in L.toeplitz_last_error()
    torch_cuda.cuda.synchronize()
    assert bool((y == 3.0).all()), "a refused call wrote its output"
    # the same plan at a size within the limit runs and agrees with the plan workspace
    X = sa.rhs_random(prob, 2)
    plan2 = _plan(prob, 2)
    y_ws, y_st = _both(torch_cuda, plan2, X, "fp64")
    assert np.array_equal(y_ws.view(np.uint8), y_st.view(np.uint8))
    del tp
