"""The dense rim's matrix-core slabs and the forward 2-D tiles in one launch
(TP_OPT_RIM_OVERLAP) against the two launches bit for bit and against the
oracle: reciprocal and separate element-rim blocks, three precisions, ragged
column blocks, idle solver columns."""
import numpy as np
import pytest

import oracle
from synth import arrays as sa
from helpers import assert_parity, banner, random_rim_er, to_dev

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-10, "fp32": 1e-5, "mixed": 1e-5}


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2506_04710_amd as tp
    tp.load()
    return tp


def _bits(y):
    return y.view(np.uint32 if y.dtype == np.complex64 else np.uint64)


CASES = [(4, 4, 16, 24, 16, False), (6, 5, 33, 70, 40, True), (5, 4, 64, 36, 20, False), (9, 9, 96, 72, 81, False)]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}b{c[2]}r{c[3]}R{c[4]}{'er' if c[5] else ''}"
                                             for c in CASES])
@pytest.mark.parametrize("which", ["fp64", "fp32", "mixed"])
def test_rim_overlap_bitwise(tp, case, which):
    import torch
    from paper_2506_04710_amd import _lib
    Nx, Ny, b, Nr, R, er = case
    banner(f"rim overlap {which} {case}")
    prob = sa.make_problem(Nx, Ny, b, Nr, 9400 + b)
    rim_er = random_rim_er(prob, 5) if er else None
    plan = tp.Plan.create(Nx, Ny, b, Nr, prob.gen, prob.rim_re, prob.rim_rr, rim_er=rim_er, prec="mixed",
                          max_rhs=R, restart=4)
    X = sa.rhs_random(prob, R, rng=np.random.default_rng(R))
    dt = torch.complex64 if which == "fp32" else torch.complex128
    if which == "fp32":
        X = X.astype(np.complex64).astype(np.complex128)
    x = to_dev(X, dt)
    assert plan.get_option(_lib.TP_OPT_RIM_OVERLAP) == 1          # the default
    assert "rim_overlap" in plan.path(which, R), plan.path(which, R)
    y1 = plan.matvec(x, which=which).cpu().numpy()
    plan.set_option(_lib.TP_OPT_RIM_OVERLAP, 0)
    assert "rim_overlap" not in plan.path(which, R)
    y0 = plan.matvec(x, which=which).cpu().numpy()
    assert np.array_equal(_bits(y0), _bits(y1))
    op = oracle.Operator(Nx, Ny, b, Nr, prob.gen, prob.rim_re, prob.rim_rr, rim_er)
    assert_parity(y1.astype(np.complex128).reshape(X.shape), oracle.matvec(op, X), TOL[which], N=prob.N,
                  what=which)
    plan.close()


def test_rim_overlap_solve(tp):
    """A 24-column preconditioned mixed solve with the shared launch (columns
    that finish early leave idle slots in both halves of it)."""
    from paper_2506_04710_amd import _lib
    banner("rim overlap in a 24-column solve")
    prob = sa.make_problem(6, 6, 32, 40, 9450)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=24, restart=30)
    assert "rim_overlap" in plan.path("mixed", 24)
    plan.precond_create()
    V = sa.rhs_random(prob, 24, rng=np.random.default_rng(8))
    V[::4] *= 1e-3
    x, info = plan.solve(to_dev(V), mode="mixed", tol=1e-8, precond=True)
    rr = oracle.relres(prob, x.cpu().numpy().reshape(24, -1), V)
    assert all(i["status"] == 0 for i in info) and np.all(rr <= 1e-8), (info, rr)
    with pytest.raises(tp.ToeplitzError):
        plan.set_option(_lib.TP_OPT_RIM_OVERLAP, 3)
    plan.close()
