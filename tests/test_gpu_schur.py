"""GPU parity of the Schur-complement elimination of the rim (solves with the
element operator A, dense C - B A^-1 B_er) against the oracle's dense LU."""
import numpy as np
import pytest

import oracle
from synth import arrays as sa
from helpers import banner, random_rim_er, rel_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2506_04710_amd as tp
    tp.load()
    return tp


def _pair(tp, prob, rim_er=None, max_rhs=4, precond=True):
    plan = tp.Plan.create(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, rim_er=rim_er,
                          prec="mixed", max_rhs=max_rhs, restart=40)
    elem = tp.Plan.create(prob.Nx, prob.Ny, prob.b, 0, prob.gen, prec="mixed", max_rhs=8, restart=40)
    if precond:
        elem.precond_create()
    return plan, elem


@pytest.mark.parametrize("mode,precond", [("mixed", True), ("fp64", False)])
def test_schur_solve_matches_lu(tp, mode, precond):
    banner(f"schur solve {mode} precond={precond}")
    prob, V = sa.make_config(1)
    V = np.concatenate([V, sa.rhs_random(prob, 2, np.random.default_rng(11))])
    plan, elem = _pair(tp, prob, precond=precond)
    plan.schur_create(elem, mode=mode, tol=1e-11, precond=precond)
    x, info = plan.schur_solve(to_dev(V), mode=mode, tol=1e-8, precond=precond)
    X = x.cpu().numpy()
    rr = oracle.relres(prob, X, V)
    assert all(i["status"] == 0 for i in info), info
    assert np.all(rr <= 1e-8), rr
    # the library's reported residual is the true one
    assert np.allclose([i["relres"] for i in info], rr, rtol=1e-3, atol=1e-14)
    Xlu = oracle.lu_solve(oracle.assemble(prob), V)
    assert rel_err(X, Xlu) <= 1e-6


def test_schur_solve_nonreciprocal_rim(tp):
    banner("schur solve non-reciprocal rim")
    prob = sa.make_problem(5, 3, 12, 10, 61)
    rim_er = random_rim_er(prob, 62)
    V = sa.rhs_random(prob, 3, np.random.default_rng(63))
    plan, elem = _pair(tp, prob, rim_er=rim_er)
    plan.schur_create(elem, tol=1e-11, precond=True)
    x, info = plan.schur_solve(to_dev(V), tol=1e-8, precond=True)
    op = oracle.Operator(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, rim_er)
    rr = oracle.relres(op, x.cpu().numpy(), V)
    assert all(i["status"] == 0 for i in info) and np.all(rr <= 1e-8), (info, rr)


def test_schur_errors(tp):
    banner("schur argument errors")
    prob, V = sa.make_config(1)
    plan, elem = _pair(tp, prob, precond=False)
    with pytest.raises(tp.ToeplitzError):        # no elimination built yet
        plan.schur_solve(to_dev(V))
    other = tp.Plan.create(prob.Nx, prob.Ny, 8, 0, np.zeros((2 * prob.Ny - 1, 2 * prob.Nx - 1, 8, 8), complex),
                           prec="mixed", max_rhs=2, restart=4)
    with pytest.raises(tp.ToeplitzError):        # element plan of another shape
        plan.schur_create(other)
    with pytest.raises(tp.ToeplitzError):        # element plan with a rim
        plan.schur_create(plan)


def test_schur_one_rim_function_strided_columns(tp):
    banner("schur solve Nr=1, ldv > Nt")
    prob = sa.make_problem(3, 2, 4, 1, 71)          # the single rim function sits in a corner
    V = sa.rhs_random(prob, 2, np.random.default_rng(72))
    plan, elem = _pair(tp, prob, max_rhs=2, precond=False)
    plan.schur_create(elem, mode="fp64", tol=1e-12)
    import torch
    wide = torch.zeros((2, prob.Nt + 3), dtype=torch.complex128, device="cuda:0")
    wide[:, :prob.Nt] = to_dev(V)
    x, info = plan.schur_solve(wide[:, :prob.Nt], mode="fp64", tol=1e-10)
    X = x.cpu().numpy()
    assert all(i["status"] == 0 for i in info), info
    Xlu = oracle.lu_solve(oracle.assemble(prob), V)
    assert rel_err(X, Xlu) <= 1e-8


def test_schur_needs_fp64_operator(tp):
    banner("schur rejects an FP32-only plan")
    prob, _ = sa.make_config(1)
    plan = tp.Plan.create(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, prec="fp32",
                          max_rhs=1, restart=8)
    elem = tp.Plan.create(prob.Nx, prob.Ny, prob.b, 0, prob.gen, prec="mixed", max_rhs=1, restart=8)
    with pytest.raises(tp.ToeplitzError):
        plan.schur_create(elem)
