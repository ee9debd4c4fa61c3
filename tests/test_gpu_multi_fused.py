"""The persistent multi-column launch (TP_OPT_MULTI_FUSED = 1: rim slabs,
forward 2-D tiles, matrix-core products, inverse tiles and the rim finish as
tasks of one launch, ordered by completion counters) against the separate
launches bit for bit and against the oracle: dense reciprocal rims, placed
rims, no rim, odd b and separate B_er (which keep the separate launches), the
preconditioner, the static-workspace entry point and a multi-column solve."""
import numpy as np
import pytest

import oracle
from synth import arrays as sa
from helpers import assert_parity, banner, to_dev

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-10, "fp32": 1e-5, "mixed": 1e-5}
WHICH = ["fp64", "fp32", "mixed"]


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2506_04710_amd as tp
    tp.load()
    return tp


def _input(prob, R, which, seed):
    X = sa.rhs_random(prob, R, rng=np.random.default_rng(seed))
    return X.astype(np.complex64).astype(np.complex128) if which == "fp32" else X


def _run(plan, X, which, fn="matvec"):
    import torch
    dt = torch.complex64 if which == "fp32" else torch.complex128
    y = getattr(plan, fn)(to_dev(X, dt), which=which).cpu().numpy()
    return y.reshape(X.shape)


def _bits(y):
    return y.view(np.uint32 if y.dtype == np.complex64 else np.uint64)


def _both(tp, plan, X, which, fn="matvec"):
    from paper_2506_04710_amd import _lib
    plan.set_option(_lib.TP_OPT_MULTI_FUSED, 0)
    y0 = _run(plan, X, which, fn)
    plan.set_option(_lib.TP_OPT_MULTI_FUSED, 1)
    assert plan.get_option(_lib.TP_OPT_MULTI_FUSED) == 1
    y1 = _run(plan, X, which, fn)
    return y0, y1


# (Nx, Ny, b, Nr, R): 2-D tile grids; R spans one and several column blocks
# with a ragged last one
CASES = [(4, 4, 16, 24, 16), (6, 5, 8, 44, 33), (5, 4, 64, 36, 20), (9, 7, 12, 32, 81), (3, 3, 96, 40, 17),
         (7, 6, 24, 0, 48)]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}b{c[2]}r{c[3]}R{c[4]}" for c in CASES])
@pytest.mark.parametrize("placed", [False, True])
@pytest.mark.parametrize("which", WHICH)
def test_fused_operator(tp, case, placed, which):
    Nx, Ny, b, Nr, R = case
    if placed and Nr == 0:
        pytest.skip("no rim to place")
    banner(f"persistent multi-column operator {which} {case} placed={placed}")
    prob = sa.make_problem(Nx, Ny, b, Nr, 9800 + Nx * 10 + b)
    kw = {"rim_place": sa.rim_placement(prob)} if placed else {}
    plan = tp.Plan.create(Nx, Ny, b, Nr, prob.gen, prob.rim_re, prob.rim_rr, prec="mixed", max_rhs=R, restart=4,
                          **kw)
    X = _input(prob, R, which, 31 + R)
    y0, y1 = _both(tp, plan, X, which)
    path = plan.path(which, R)
    assert ("persistent" in path) == (plan.info()["bc"] % 2 == 0), path
    assert {"mfma", "tiles2d"} <= path and ("dense_rim" in path) == (not placed and Nr > 0), path
    assert np.array_equal(_bits(y0), _bits(y1)), f"{which} {case}: persistent launch differs from separate launches"
    assert_parity(y1.astype(np.complex128), oracle.matvec(prob, X), TOL[which], N=prob.N, what=f"{which} {case}")
    plan.close()


@pytest.mark.parametrize("which", WHICH)
def test_fused_not_applicable(tp, which):
    """Odd b and a separate B_er keep the separate launches (same results)."""
    banner(f"persistent multi-column launch not applicable {which}")
    for Nx, Ny, b, Nr, nonrecip in [(4, 3, 9, 20, False), (4, 4, 16, 24, True)]:
        prob = sa.make_problem(Nx, Ny, b, Nr, 9900 + b)
        kw = {}
        if nonrecip:
            rng = np.random.default_rng(3)
            rim_er = prob.rim_re.T + 0.1 * (rng.standard_normal(prob.rim_re.T.shape)
                                            + 1j * rng.standard_normal(prob.rim_re.T.shape))
            kw["rim_er"] = rim_er
        plan = tp.Plan.create(Nx, Ny, b, Nr, prob.gen, prob.rim_re, prob.rim_rr, prec="mixed", max_rhs=20,
                              restart=4, **kw)
        X = _input(prob, 20, which, 5)
        y0, y1 = _both(tp, plan, X, which)
        assert "persistent" not in plan.path(which, 20)
        assert np.array_equal(_bits(y0), _bits(y1))
        op = oracle.Operator(Nx, Ny, b, Nr, prob.gen, prob.rim_re, prob.rim_rr, kw.get("rim_er"))
        assert_parity(y1.astype(np.complex128), oracle.matvec(op, X), TOL[which], N=prob.N, what=which)
        plan.close()


@pytest.mark.parametrize("placed", [False, True])
@pytest.mark.parametrize("which", WHICH)
def test_fused_preconditioner(tp, placed, which):
    Nx, Ny, b, Nr, R = 6, 5, 16, 30, 24
    banner(f"persistent multi-column preconditioner {which} placed={placed}")
    prob = sa.make_problem(Nx, Ny, b, Nr, 9950 + placed)
    kw = {"rim_place": sa.rim_placement(prob)} if placed else {}
    plan = tp.Plan.create(Nx, Ny, b, Nr, prob.gen, prob.rim_re, prob.rim_rr, prec="mixed", max_rhs=R, restart=4,
                          **kw)
    plan.precond_create()
    info = plan.info()
    X = _input(prob, R, which, 77)
    y0, y1 = _both(tp, plan, X, which, "precond_apply")
    assert "persistent" in plan.path(which, R, precond=True)
    assert np.array_equal(_bits(y0), _bits(y1))
    if placed:
        place, nrc = sa.rim_placement(prob)
        ref = oracle.placed_precond_apply(prob, X, place, nrc, info["Px"], info["Py"])
    else:
        ref = oracle.precond_apply(prob, X, info["Px"], info["Py"])
    assert_parity(y1.astype(np.complex128), ref, TOL[which], N=prob.N, what=which)
    plan.close()


def test_fused_static_entry(tp):
    """The static-workspace entry point takes the same launch (its counters
    live in the static array): equal bit for bit to the plan's own, twice."""
    from paper_2506_04710_amd import _lib
    banner("persistent multi-column launch through the static entry point")
    prob = sa.make_problem(5, 4, 32, 28, 9977)
    plan = tp.Plan.create(5, 4, 32, 28, prob.gen, prob.rim_re, prob.rim_rr, prec="mixed", max_rhs=40, restart=4)
    plan.set_option(_lib.TP_OPT_MULTI_FUSED, 1)
    for R in (40, 18):
        X = _input(prob, R, "mixed", R)
        y = _run(plan, X, "mixed")
        ys = _run(plan, X, "mixed", "matvec_static")
        assert np.array_equal(_bits(y), _bits(ys)), R
    plan.close()


def test_fused_solve(tp):
    """Preconditioned mixed solve of 20 columns: the solver's idle columns go
    through the persistent launch's column checks."""
    from paper_2506_04710_amd import _lib
    import torch
    banner("persistent multi-column launch in a 20-column solve")
    prob = sa.make_problem(8, 7, 24, 36, 9988)
    plan = tp.Plan.create(8, 7, 24, 36, prob.gen, prob.rim_re, prob.rim_rr, prec="mixed", max_rhs=20, restart=30)
    plan.set_option(_lib.TP_OPT_MULTI_FUSED, 1)
    plan.precond_create()
    V = sa.rhs_random(prob, 20, rng=np.random.default_rng(12))
    x, info = plan.solve(to_dev(V), mode="mixed", tol=1e-8, precond=True)
    rr = oracle.relres(prob, x.cpu().numpy().reshape(20, -1), V)
    assert all(i["status"] == 0 for i in info) and np.all(rr <= 1e-8), (info, rr)
    print(f"persistent launch solve: iters {[i['iters'] for i in info]} max relres {rr.max():.2e}")
    torch.cuda.synchronize()
    plan.close()


def test_fused_option_checks(tp):
    from paper_2506_04710_amd import _lib
    banner("persistent multi-column option checks")
    prob = sa.make_problem(3, 3, 4, 0, 9990)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=1, restart=4)
    assert plan.get_option(_lib.TP_OPT_MULTI_FUSED) == 0
    with pytest.raises(tp.ToeplitzError):
        plan.set_option(_lib.TP_OPT_MULTI_FUSED, 2)
    assert "fused" in plan.path("fp64", 1)
    with pytest.raises(tp.ToeplitzError):
        plan.path("fp64", 2)                      # beyond max_rhs
    with pytest.raises(tp.ToeplitzError):
        plan.path("fp64", 1, precond=True)        # no preconditioner
    plan.close()
