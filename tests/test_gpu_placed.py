"""GPU parity of plans with a placed (structured) rim: the rim functions are
extra channels of element cells and the plan holds the spectrum of the
extended two-level block-Toeplitz operator, no dense B or C.  Every product,
preconditioner application and solve is checked against the oracle's dense
Z (assembled from the unchanged rim blocks) or its placed preconditioner."""
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


def _input(X, which):
    return X.astype(np.complex64).astype(np.complex128) if which == "fp32" else X


def _plan(tp, prob, R, rim_er=None, restart=4):
    place, nrc = sa.rim_placement(prob)
    return tp.Plan.create(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, rim_er=rim_er,
                          prec="mixed", max_rhs=R, restart=restart, rim_place=(place, nrc)), place, nrc


def _apply(plan, X, which, fn="matvec"):
    import torch
    dt = torch.complex64 if which == "fp32" else torch.complex128
    y = getattr(plan, fn)(to_dev(X, dt), which=which)
    return y.cpu().numpy().astype(np.complex128).reshape(X.shape)


# (Nx, Ny, b, Nr, R): channels per cell b + nrc of 28 (corners), 16, 72 (the
# headline's width, 9 row chunks), 64, 78 and 104 (wider than the fused
# single-column path: multi-column kernels at R = 1); 2-15 columns (2-D tiles
# or the product kernel) and 16+ (matrix cores)
CASES = [(4, 4, 16, 24, 1), (6, 5, 8, 44, 1), (5, 4, 64, 36, 1), (3, 4, 60, 14, 1), (7, 3, 70, 40, 1),
         (9, 9, 96, 72, 1), (4, 4, 16, 24, 3), (5, 4, 24, 36, 5), (17, 9, 8, 52, 2), (4, 4, 16, 24, 17),
         (5, 3, 33, 32, 20)]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}b{c[2]}r{c[3]}R{c[4]}" for c in CASES])
@pytest.mark.parametrize("which", WHICH)
def test_placed_matvec_parity(tp, case, which):
    Nx, Ny, b, Nr, R = case
    banner(f"placed matvec {which} {case}")
    prob = sa.make_problem(Nx, Ny, b, Nr, 9100 + Nx * 100 + Ny * 10 + b)
    plan, place, nrc = _plan(tp, prob, R)
    info = plan.info()
    assert info["nrc"] == nrc and info["bc"] == b + nrc and info["half_spectrum"] == 1
    assert info["rim_bytes"] == 0
    assert info["spectrum_bytes"] == (info["Px"] // 2 + 1) * info["Py"] * (b + nrc) ** 2 * 16
    X = _input(sa.rhs_random(prob, R, rng=np.random.default_rng(R + b)), which)
    Y = _apply(plan, X, which)
    assert_parity(Y, oracle.matvec(prob, X), TOL[which], N=prob.N, what=f"{which} {case}")
    plan.close()


@pytest.mark.parametrize("R", [1, 3, 17])
@pytest.mark.parametrize("which", WHICH)
def test_placed_matvec_nonreciprocal(tp, which, R):
    """A non-reciprocal rim (B_er = 1.5 B^T, still block Toeplitz): the
    extended generators are not symmetric, so the whole spectrum is stored."""
    banner(f"placed matvec non-reciprocal {which} R={R}")
    prob = sa.make_problem(6, 4, 12, 40, 9201)
    rim_er = 1.5 * prob.rim_re.T
    plan, _, _ = _plan(tp, prob, R, rim_er=rim_er)
    assert plan.info()["half_spectrum"] == 0
    X = _input(sa.rhs_random(prob, R), which)
    Y = _apply(plan, X, which)
    op = oracle.Operator(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, rim_er)
    assert_parity(Y, oracle.matvec(op, X), TOL[which], N=prob.N, what=which)
    plan.close()


def test_placed_spectrum_parity(tp):
    """The plan's extended spectrum at every frequency against the oracle's DFT
    of the placed generators (mirrored columns read back transposed)."""
    banner("placed spectrum parity")
    prob, _ = sa.make_config(1)
    plan, place, nrc = _plan(tp, prob, 1)
    info = plan.info()
    Px, Py = info["Px"], info["Py"]
    ext = oracle.Operator(prob.Nx, prob.Ny, prob.b + nrc, 0, oracle.placed_generator(prob, place, nrc))
    kx, ky = np.meshgrid(np.arange(Px), np.arange(Py), indexing="ij")
    ref = oracle.spectrum(ext, Px, Py, kx.ravel(), ky.ravel())
    for which, tol in (("fp64", 1e-13), ("fp32", 1e-6)):
        got = np.stack([plan.spectrum(int(a), int(c), which) for a, c in zip(kx.ravel(), ky.ravel())])
        assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref)), which
    plan.close()


PRE_CASES = [(4, 4, 16, 24, 1), (5, 4, 24, 36, 1), (4, 4, 16, 24, 3), (4, 4, 16, 24, 17), (6, 5, 8, 44, 2)]


@pytest.mark.parametrize("case", PRE_CASES, ids=[f"{c[0]}x{c[1]}b{c[2]}r{c[3]}R{c[4]}" for c in PRE_CASES])
@pytest.mark.parametrize("which", WHICH)
def test_placed_precond_parity(tp, case, which):
    Nx, Ny, b, Nr, R = case
    banner(f"placed preconditioner {which} {case}")
    prob = sa.make_problem(Nx, Ny, b, Nr, 9300 + Nx * 10 + b)
    plan, place, nrc = _plan(tp, prob, R)
    plan.precond_create()
    info = plan.info()
    X = _input(sa.rhs_random(prob, R, rng=np.random.default_rng(R)), which)
    Y = _apply(plan, X, which, "precond_apply")
    ref = oracle.placed_precond_apply(prob, X, place, nrc, info["Px"], info["Py"])
    tol = 1e-10 if which == "fp64" else 1e-5
    assert_parity(Y, ref, tol, N=prob.N, what=f"{which} {case}")
    plan.close()


@pytest.mark.parametrize("mode,precond", [("fp64", False), ("mixed", True), ("fp64", True)])
def test_placed_solve_against_lu(tp, mode, precond):
    """Config 1 (4 x 4, b = 16, 24 rim functions with corners): the solve on
    the placed plan matches the oracle's dense LU solution."""
    banner(f"placed solve config 1 {mode} precond={precond}")
    prob, V = sa.make_config(1)
    plan, _, _ = _plan(tp, prob, 1, restart=40)
    if precond:
        plan.precond_create()
    x, info = plan.solve(to_dev(V), mode=mode, tol=1e-10, precond=precond)
    x = x.cpu().numpy().reshape(1, -1)
    ref = oracle.lu_solve(oracle.assemble(prob), V)
    rr = oracle.relres(prob, x, V)[0]
    assert info[0]["status"] == 0 and rr <= 1e-10, (info, rr)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 1e-8
    plan.close()


@pytest.fixture(scope="module")
def config2_placed():
    prob, V = sa.make_config(2)
    X = sa.rhs_random(prob, 1, rng=np.random.default_rng(7012)).astype(np.complex64).astype(np.complex128)
    return prob, V, X, oracle.matvec(prob, X)


@pytest.mark.parametrize("which", WHICH)
def test_placed_config2_every_row(tp, config2_placed, which):
    """The 32 x 32, b = 64, 256-rim operator from its placed form (72 channels
    per cell, half spectrum, no dense rim) on every output row."""
    banner(f"placed config 2 every row {which}")
    prob, _, X, ref = config2_placed
    plan, _, nrc = _plan(tp, prob, 1)
    assert nrc == 8 and plan.info()["bc"] == 72
    Y = _apply(plan, X, which)
    e = assert_parity(Y, ref, TOL[which], N=prob.N, what=f"placed config 2 {which}")
    print(f"placed config 2 {which}: {e}")
    plan.close()


@pytest.mark.parametrize("mode", ["mixed", "fp64"])
def test_placed_config2_solve(tp, config2_placed, mode):
    """The headline solve (broadside plane wave, tol 1e-8, preconditioned) on
    the placed plan: the oracle's residual over every row."""
    banner(f"placed config 2 solve {mode}")
    prob, V, _, _ = config2_placed
    plan, _, _ = _plan(tp, prob, 1, restart=40)
    plan.precond_create()
    x, info = plan.solve(to_dev(V), mode=mode, tol=1e-8, precond=True)
    rr = oracle.relres(prob, x.cpu().numpy().reshape(1, -1), V)[0]
    assert info[0]["status"] == 0 and rr <= 1e-8, (info, rr)
    print(f"placed config 2 {mode}: iters={info[0]['iters']} outer={info[0]['outer_iters']} relres={rr:.2e}")
    plan.close()


def test_placed_schur_refused(tp):
    banner("placed plan: rim elimination refused")
    prob, _ = sa.make_config(1)
    plan, _, _ = _plan(tp, prob, 1)
    elem = tp.Plan.create(prob.Nx, prob.Ny, prob.b, 0, prob.gen, prec="mixed", max_rhs=4, restart=8)
    with pytest.raises(tp.ToeplitzError) as ei:
        plan.schur_create(elem, mode="mixed", tol=1e-10)
    assert ei.value.status == 6
    plan.close()
    elem.close()
