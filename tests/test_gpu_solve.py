"""GPU solves (plain FP64 GMRES and mixed-precision refinement) checked by the
oracle's FP64 residual, and against the oracle's dense LU where it fits."""
import numpy as np
import pytest

import oracle
from synth import arrays as sa
from helpers import banner, rel_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available()
    import paper_2506_04710_amd as tp
    tp.load()
    return tp


def _solve(tp, prob, V, mode, tol=1e-8, restart=40, **kw):
    R = V.shape[0]
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=R, restart=restart)
    x, info = plan.solve(to_dev(V), mode=mode, tol=tol, **kw)
    return x.cpu().numpy().reshape(R, prob.Nt), info, plan


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_solve_config1_vs_lu(tp, mode):
    banner(f"solve config 1 {mode}")
    prob, V = sa.make_config(1)
    X, info, _ = _solve(tp, prob, V, mode)
    rr = oracle.relres(prob, X, V)
    assert info[0]["status"] == 0 and rr[0] <= 1e-8, (info, rr)
    assert abs(info[0]["relres"] - rr[0]) <= 1e-12 + 1e-3 * rr[0]       # library's own FP64 residual
    Xlu = oracle.lu_solve(oracle.assemble(prob), V)
    assert rel_err(X, Xlu) <= 1e-6
    print(f"config1 {mode}: iters={info[0]['iters']} outer={info[0]['outer_iters']} relres={rr[0]:.2e} "
          f"fwd_err={rel_err(X, Xlu):.2e}")


def test_solve_scaled_identity_one_step(tp):
    """Z = alpha I: the first Krylov vector is the solution (one Arnoldi step)."""
    banner("solve scaled identity")
    Nx, Ny, b = 3, 2, 4
    gen = np.zeros((2 * Ny - 1, 2 * Nx - 1, b, b), dtype=complex)
    gen[Ny - 1, Nx - 1] = (2 - 1j) * np.eye(b)
    plan = tp.Plan.create(Nx, Ny, b, 0, gen, prec="mixed", max_rhs=1, restart=10)
    v = np.random.default_rng(1).standard_normal(Nx * Ny * b) + 0j
    x, info = plan.solve(to_dev(v), mode="fp64", tol=1e-12)
    assert info[0]["iters"] == 1 and info[0]["status"] == 0
    assert np.allclose(x.cpu().numpy(), v / (2 - 1j), rtol=1e-13, atol=0)


def test_solve_block_diagonal_minimal_polynomial(tp):
    """Only Z_{0,0} != 0: Z = I (x) Z00, so GMRES ends within b steps."""
    banner("solve block diagonal")
    Nx, Ny, b = 4, 3, 6
    rng = np.random.default_rng(2)
    gen = np.zeros((2 * Ny - 1, 2 * Nx - 1, b, b), dtype=complex)
    gen[Ny - 1, Nx - 1] = rng.standard_normal((b, b)) + 1j * rng.standard_normal((b, b)) + 6 * np.eye(b)
    plan = tp.Plan.create(Nx, Ny, b, 0, gen, prec="mixed", max_rhs=1, restart=20)
    v = rng.standard_normal(Nx * Ny * b) + 1j * rng.standard_normal(Nx * Ny * b)
    x, info = plan.solve(to_dev(v), mode="fp64", tol=1e-12)
    assert info[0]["status"] == 0 and info[0]["iters"] <= b
    op = oracle.Operator(Nx, Ny, b, 0, gen)
    assert oracle.relres(op, x.cpu().numpy()[None], v[None])[0] <= 1e-12


def test_solve_x0_exact_needs_no_iterations(tp):
    banner("solve with exact x0")
    prob, V = sa.make_config(1)
    Xlu = oracle.lu_solve(oracle.assemble(prob), V)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=1, restart=40)
    x, info = plan.solve(to_dev(V), mode="fp64", tol=1e-8, x0=to_dev(Xlu))
    assert info[0]["iters"] == 0 and info[0]["status"] == 0


def test_solve_noconv_reports(tp):
    banner("solve no-convergence path")
    prob, V = sa.make_config(1)
    _, info, _ = _solve(tp, prob, V, "fp64", tol=1e-14, max_iter=2)
    assert info[0]["status"] == 4 and info[0]["iters"] <= 2 and info[0]["relres"] > 1e-14


def test_solve_rejects_bad_requests(tp):
    banner("solve argument errors")
    import torch
    prob, V = sa.make_config(1)
    plan = tp.Plan.from_problem(prob, prec="fp64", max_rhs=1, restart=10)
    with pytest.raises(tp.ToeplitzError) as e:
        plan.solve(to_dev(V), mode="mixed")           # no FP32 copy in this plan
    assert e.value.status == 6
    with pytest.raises(tp.ToeplitzError):
        plan.solve(to_dev(np.vstack([V, V])), mode="fp64")   # more columns than max_rhs
    with pytest.raises(tp.ToeplitzError):
        plan.solve(to_dev(V), mode="fp64", restart=11)        # beyond the plan's restart
    with pytest.raises(tp.ToeplitzError):
        plan.matvec(to_dev(V, torch.complex64), which="fp32")  # no FP32 copy


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_solve_batch_matches_single(tp, mode):
    """Independent Krylov spaces.  Batches of two or more columns run the same
    kernels whatever the batch holds, so a column's iterates, and its solution,
    are the same bit for bit in any such batch.  A single column runs the
    fused single-column operator, whose sums run in another order: its
    solution is a different iterate meeting the same tolerance, so the two
    differ by at most the residual bound ||Z (x1 - xb)|| <= 2 tol ||v||."""
    banner(f"solve batch vs single {mode}")
    prob = sa.make_problem(6, 5, 16, 20, 77)
    V = sa.rhs_random(prob, 4)
    Xb, ib, _ = _solve(tp, prob, V, mode)
    assert np.all(oracle.relres(prob, Xb, V) <= 1e-8)
    X2, i2, _ = _solve(tp, prob, V[[3, 0]], mode)
    assert np.array_equal(X2[0], Xb[3]) and np.array_equal(X2[1], Xb[0])
    assert [i["iters"] for i in i2] == [ib[3]["iters"], ib[0]["iters"]]
    for r in (0, 3):
        X1, i1, _ = _solve(tp, prob, V[r:r + 1], mode)
        assert oracle.relres(prob, X1, V[r:r + 1])[0] <= 1e-8
        # ||Z (x1 - xb)|| / ||v|| by the oracle's product (v cancels)
        D = oracle.matvec(prob, X1 - Xb[r:r + 1])
        assert np.linalg.norm(D) / np.linalg.norm(V[r]) <= 2e-8


def test_solve_config3_ports_batched(tp):
    """81 port excitations solved together (mixed precision), residual by the oracle."""
    banner("solve config 3 batched ports")
    prob, V = sa.make_config(3)
    X, info, _ = _solve(tp, prob, V, "mixed")
    rr = oracle.relres(prob, X, V)
    assert all(i["status"] == 0 for i in info)
    assert np.max(rr) <= 1e-8, np.max(rr)
    print(f"config3: iters max={max(i['iters'] for i in info)} outer max={max(i['outer_iters'] for i in info)}")


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_solve_config2_full_size(tp, mode):
    banner(f"solve config 2 full size {mode}")
    prob, V = sa.make_config(2)
    X, info, _ = _solve(tp, prob, V, mode)
    rr = oracle.relres(prob, X, V)
    assert info[0]["status"] == 0 and rr[0] <= 1e-8, (info, rr)
    print(f"config2 {mode}: iters={info[0]['iters']} outer={info[0]['outer_iters']} relres={rr[0]:.2e}")


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_solve_graph_replays_deterministic(tp, mode):
    """Solves replay a captured graph: repeated solves on one plan, with eager
    operator applications in between, give bit-identical results."""
    banner(f"solve graph replay determinism {mode}")
    import torch
    prob = sa.make_problem(7, 6, 24, 30, 91)
    V = sa.rhs_random(prob, 2)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=2, restart=40)
    v = to_dev(V)
    ref, info0 = plan.solve(v, mode=mode)
    ref = ref.cpu().numpy()
    for rep in range(3):
        plan.matvec(v)                                  # eager work between replays
        torch.cuda.synchronize()
        x, info = plan.solve(v, mode=mode)
        assert np.array_equal(x.cpu().numpy(), ref), rep
        assert [i["iters"] for i in info] == [i["iters"] for i in info0]
    assert np.all(oracle.relres(prob, ref, V) <= 1e-8)


def test_config4_mixed_to_1e10_against_fp64():
    """64 x 64 array, b = 48, 8 scan-angle plane waves: the mixed solve reaches
    relative residual 1e-10 per column; its error against the plain FP64 solve
    is reported and bounded; the oracle's rows agree on a row sample."""
    banner("config 4 mixed 1e-10, 8 RHS")
    import torch
    import paper_2506_04710_amd as tp
    prob, V = sa.make_config(4)
    R = V.shape[0]
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=R, restart=40, device=torch.device("cuda:0"))
    v = to_dev(V)
    x, info = plan.solve(v, mode="mixed", tol=1e-10)
    assert all(i["status"] == 0 and i["relres"] <= 1e-10 for i in info), info
    x64, info64 = plan.solve(v, mode="fp64", tol=1e-10)
    assert all(i["status"] == 0 for i in info64), info64
    X, X64 = x.cpu().numpy(), x64.cpu().numpy()
    errs = [rel_err(X[r], X64[r]) for r in range(R)]
    print(f"config 4: mixed iters {[i['iters'] for i in info]} outer {[i['outer_iters'] for i in info]}, "
          f"fp64 iters {[i['iters'] for i in info64]}, max rel diff mixed vs fp64 {max(errs):.2e}")
    assert max(errs) <= 1e-8
    # the oracle's FP64 residual over all 196,608 rows, for the first and the
    # last scan angle
    for r in (0, R - 1):
        rr = oracle.relres(prob, X[r:r + 1], V[r:r + 1])[0]
        print(f"config 4 column {r}: oracle relres {rr:.3e}, library {info[r]['relres']:.3e}")
        assert rr <= 1e-10
    plan.close()


def test_solve_nonfinite_rhs_stops():
    """A right-hand side holding NaN or Inf ends its column at the first
    residual with TP_E_INVAL; a finite column in the same call still solves."""
    banner("solve non-finite right-hand side")
    import ctypes
    import torch
    import paper_2506_04710_amd as tp
    from paper_2506_04710_amd import _lib
    prob, V = sa.make_config(1)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=3, restart=40)
    V3 = np.vstack([V, V, V])
    V3[1, 7] = np.nan
    V3[2, 3] = np.inf
    v = to_dev(V3)
    x = torch.empty_like(v)
    o = _lib.SolveOpts()
    _lib.lib().toeplitz_solve_opts_default(ctypes.byref(o))
    o.mode = _lib.PREC["mixed"]
    info = (_lib.SolveInfo * 3)()
    st = _lib.lib().toeplitz_solve(plan._h, ctypes.c_void_p(v.data_ptr()), prob.Nt, ctypes.c_void_p(x.data_ptr()),
                                   prob.Nt, 3, ctypes.byref(o), info, None)
    assert st == _lib.TP_E_INVAL
    assert info[0].status == 0 and info[0].relres <= 1e-8
    assert info[1].status == _lib.TP_E_INVAL and info[1].iters == 0
    assert info[2].status == _lib.TP_E_INVAL and info[2].iters == 0
    assert oracle.relres(prob, x[:1].cpu().numpy(), V)[0] <= 1e-8
    plan.close()


@pytest.mark.parametrize("shape", [(12, 10, 24, 40), (40, 36, 16, 24)])
def test_mixed_solve_shared_launches_bitwise(tp, shape):
    """A one-column mixed solve whose FP32 and FP64 operators share each stage's
    launch, and whose preconditioner's last pass shares a launch with the
    operator's first (TP_OPT_DUAL_LAUNCH, placed rim, pair-stream pass), gives
    the same bits as the solve with one launch sequence per precision."""
    from paper_2506_04710_amd import _lib
    Nx, Ny, b, Nr = shape
    banner(f"mixed solve, shared FP32/FP64 launches, {Nx}x{Ny} b{b} Nr{Nr}")
    prob = sa.make_problem(Nx, Ny, b, Nr, 9555)
    V = sa.rhs_random(prob, 1, rng=np.random.default_rng(4))
    out = {}
    for dual in (1, 0):
        plan = tp.Plan.create(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, prec="mixed",
                              max_rhs=1, restart=30, rim_place=sa.rim_placement(prob))
        plan.set_option(_lib.TP_OPT_SPECTRUM_PASS, _lib.TP_PASS_PAIRS)
        assert plan.get_option(_lib.TP_OPT_DUAL_LAUNCH) == 1
        plan.set_option(_lib.TP_OPT_DUAL_LAUNCH, dual)
        plan.precond_create()
        # on the larger grid (separate x and y passes) the preconditioner's last
        # pass and the operator's first share a launch; the small grid's
        # preconditioner runs on 2-D tiles
        assert ("joined" in plan.path("mixed", nrhs=1, precond=True)) == (bool(dual) and Nx >= 20)
        x, info = plan.solve(to_dev(V), mode="mixed", tol=1e-8, precond=True)
        out[dual] = (x.cpu().numpy().reshape(1, -1), info[0])
        plan.close()
    (x1, i1), (x0, i0) = out[1], out[0]
    assert i1["status"] == 0 and i1["iters"] == i0["iters"] and i1["outer_iters"] == i0["outer_iters"]
    assert np.array_equal(x1.view(np.uint64), x0.view(np.uint64))
    assert oracle.relres(prob, x1, V)[0] <= 1e-8


@pytest.mark.parametrize("shape,R,placed", [((12, 10, 24, 40), 16, True), ((12, 10, 24, 40), 40, True),
                                            ((40, 36, 16, 24), 20, True), ((40, 36, 16, 0), 33, False)])
def test_mixed_solve_shared_launches_multi_bitwise(tp, shape, R, placed):
    """Many columns: the shared FP32/FP64 launches (matrix-core product at its
    default column tiles, on 2-D tiles for the small grid and on separate
    passes for the larger one; ragged column blocks) give the same bits,
    iteration counts and statuses as one launch sequence per precision."""
    from paper_2506_04710_amd import _lib
    Nx, Ny, b, Nr = shape
    banner(f"mixed solve, shared launches, {Nx}x{Ny} b{b} Nr{Nr} R{R} placed={placed}")
    prob = sa.make_problem(Nx, Ny, b, Nr, 9556 + R)
    V = sa.rhs_random(prob, R, rng=np.random.default_rng(R))
    out = {}
    for dual in (1, 0):
        kw = {"rim_place": sa.rim_placement(prob)} if placed and Nr else {}
        plan = tp.Plan.create(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, prec="mixed",
                              max_rhs=R, restart=30, **kw)
        plan.set_option(_lib.TP_OPT_DUAL_LAUNCH, dual)
        p32, p64 = plan.path("fp32", nrhs=R), plan.path("fp64", nrhs=R)
        assert "mfma" in p32 and "mfma" in p64 and not (p32 | p64) & {"dense_rim", "persistent"}
        assert ("tiles2d" in p32) == ("tiles2d" in p64) == (Nx < 20)
        x, info = plan.solve(to_dev(V), mode="mixed", tol=1e-8)
        out[dual] = (x.cpu().numpy().reshape(R, -1), info)
        plan.close()
    (x1, i1), (x0, i0) = out[1], out[0]
    for a, c in zip(i1, i0):
        assert a["status"] == c["status"] == 0 and a["iters"] == c["iters"] and a["outer_iters"] == c["outer_iters"]
    assert np.array_equal(x1.view(np.uint64), x0.view(np.uint64))
    rr = oracle.relres(prob, x1, V)
    assert max(rr) <= 1e-8, rr
    print(f"R={R}: iters {[a['iters'] for a in i1][:4]} max relres {max(rr):.2e}")
