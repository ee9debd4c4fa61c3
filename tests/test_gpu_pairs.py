"""The pair-stream spectrum pass (TP_PASS_PAIRS: y transforms in passes of
their own, each stored block of a half spectrum read once and applied to its
frequency and, transposed, to the mirror frequency) against the oracle: the
operator of a placed rim, the preconditioner of dense and placed plans, on
small grids (2-D tile transforms) and the 63 x 63 headline grid (separate x
and y passes), and a solve."""
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


def _plan(tp, prob, placed, R=1, restart=4):
    from paper_2506_04710_amd import _lib
    kw = {"rim_place": sa.rim_placement(prob)} if placed else {}
    plan = tp.Plan.create(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, prec="mixed",
                          max_rhs=R, restart=restart, **kw)
    plan.set_option(_lib.TP_OPT_SPECTRUM_PASS, _lib.TP_PASS_PAIRS)
    assert plan.get_option(_lib.TP_OPT_SPECTRUM_PASS) == _lib.TP_PASS_PAIRS
    return plan


def _apply(plan, X, which, fn):
    import torch
    dt = torch.complex64 if which == "fp32" else torch.complex128
    return getattr(plan, fn)(to_dev(X, dt), which=which).cpu().numpy().astype(np.complex128).reshape(X.shape)


def _input(X, which):
    return X.astype(np.complex64).astype(np.complex128) if which == "fp32" else X


# (Nx, Ny, b, Nr): channels per cell 28, 16, 72, 78 (placed); grids up to 18 x 13
SHAPES = [(4, 4, 16, 24), (6, 5, 8, 44), (5, 4, 64, 36), (7, 3, 70, 40), (9, 7, 12, 32)]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{s[0]}x{s[1]}b{s[2]}r{s[3]}" for s in SHAPES])
@pytest.mark.parametrize("which", WHICH)
def test_pairs_placed_operator(tp, shape, which):
    banner(f"pairs placed operator {which} {shape}")
    prob = sa.make_problem(*shape, 9500 + shape[0] * 10 + shape[2])
    plan = _plan(tp, prob, True)
    X = _input(sa.rhs_random(prob, 1), which)
    assert_parity(_apply(plan, X, which, "matvec"), oracle.matvec(prob, X), TOL[which], N=prob.N,
                  what=f"{which} {shape}")
    plan.close()


@pytest.mark.parametrize("placed", [False, True])
@pytest.mark.parametrize("shape", SHAPES[:3], ids=[f"{s[0]}x{s[1]}b{s[2]}r{s[3]}" for s in SHAPES[:3]])
@pytest.mark.parametrize("which", WHICH)
def test_pairs_preconditioner(tp, shape, which, placed):
    banner(f"pairs preconditioner {which} {shape} placed={placed}")
    prob = sa.make_problem(*shape, 9600 + shape[0] * 10 + shape[2])
    plan = _plan(tp, prob, placed)
    plan.precond_create()
    info = plan.info()
    X = _input(sa.rhs_random(prob, 1), which)
    if placed:
        place, nrc = sa.rim_placement(prob)
        ref = oracle.placed_precond_apply(prob, X, place, nrc, info["Px"], info["Py"])
    else:
        ref = oracle.precond_apply(prob, X, info["Px"], info["Py"])
    assert_parity(_apply(plan, X, which, "precond_apply"), ref, TOL[which], N=prob.N, what=f"{which} {shape}")
    plan.close()


@pytest.fixture(scope="module")
def config2():
    prob, V = sa.make_config(2)
    X = sa.rhs_random(prob, 1, rng=np.random.default_rng(7022)).astype(np.complex64).astype(np.complex128)
    return prob, V, X, oracle.matvec(prob, X)


@pytest.mark.parametrize("tile", [0, 163840])
@pytest.mark.parametrize("which", WHICH)
def test_pairs_config2_every_row(tp, config2, which, tile):
    """The headline grid (63 x 63: separate x and y transform passes, or with
    160 KB tiles both directions in one launch for FP32), placed rim with 72
    channels: every output row."""
    from paper_2506_04710_amd import _lib
    banner(f"pairs placed config 2 every row {which} tile={tile}")
    prob, _, X, ref = config2
    plan = _plan(tp, prob, True)
    plan.set_option(_lib.TP_OPT_FFT2_LDS, tile)
    assert_parity(_apply(plan, X, which, "matvec"), ref, TOL[which], N=prob.N, what=f"config 2 {which}")
    plan.close()


@pytest.mark.parametrize("placed,tile", [(False, 0), (True, 0), (True, 163840)])
def test_pairs_config2_solve(tp, config2, placed, tile):
    """The headline preconditioned mixed solve with the pair-stream pass (the
    dense plan uses it for its preconditioner, the placed plan for both)."""
    from paper_2506_04710_amd import _lib
    banner(f"pairs config 2 solve placed={placed} tile={tile}")
    prob, V, _, _ = config2
    plan = _plan(tp, prob, placed, restart=40)
    plan.set_option(_lib.TP_OPT_FFT2_LDS, tile)
    plan.precond_create()
    x, info = plan.solve(to_dev(V), mode="mixed", tol=1e-8, precond=True)
    rr = oracle.relres(prob, x.cpu().numpy().reshape(1, -1), V)[0]
    assert info[0]["status"] == 0 and rr <= 1e-8, (info, rr)
    print(f"pairs config 2 placed={placed}: iters={info[0]['iters']} relres={rr:.2e}")
    plan.close()


def test_option_checks(tp):
    from paper_2506_04710_amd import _lib
    banner("plan option checks")
    prob = sa.make_problem(3, 3, 4, 0, 9700)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=1, restart=4)
    assert plan.get_option(_lib.TP_OPT_SPECTRUM_PASS) == _lib.TP_PASS_AUTO
    with pytest.raises(tp.ToeplitzError):
        plan.set_option(_lib.TP_OPT_SPECTRUM_PASS, 7)
    with pytest.raises(tp.ToeplitzError):
        plan.set_option(99, 0)
    with pytest.raises(tp.ToeplitzError):
        plan.set_option(_lib.TP_OPT_FFT2_LDS, 200000)
    plan.close()
