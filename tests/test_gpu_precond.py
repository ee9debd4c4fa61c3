"""Block-circulant preconditioner on the GPU: its application against the
oracle's dense circulant solve, and right-preconditioned GMRES (plain FP64 and
mixed) reaching the tolerance on the oracle's FP64 residual."""
import numpy as np
import pytest

import oracle
from synth import arrays as sa
from helpers import assert_parity, banner, random_rim_er, rel_err, to_dev

pytestmark = pytest.mark.gpu
TOL64, TOL32 = 1e-10, 1e-5
TOL = {"fp64": TOL64, "fp32": TOL32, "mixed": TOL32}


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available()
    import paper_2506_04710_amd as tp
    tp.load()
    return tp


CASES = [  # (Nx, Ny, b, Nr, R): fused single column, 2-D tiles, MFMA columns, large-grid passes
    (3, 2, 4, 5, 1), (3, 2, 4, 5, 3), (4, 3, 6, 0, 2), (5, 4, 8, 3, 17), (2, 5, 33, 4, 2),
    (22, 22, 1, 0, 2), (22, 22, 1, 3, 1)]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}b{c[2]}r{c[3]}R{c[4]}" for c in CASES])
@pytest.mark.parametrize("which", ["fp64", "fp32", "mixed"])
def test_precond_apply_parity(tp, case, which):
    """'mixed' is the FP32 copy on complex128 vectors, the form a mixed solve
    applies (its inputs are rounded by the kernel, so the oracle sees the
    unrounded X)."""
    import torch
    Nx, Ny, b, Nr, R = case
    banner(f"precond apply {which} {case}")
    prob = sa.make_problem(Nx, Ny, b, Nr, 5000 + Nx * 100 + Ny * 10 + b)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=R, restart=4).precond_create()
    inf = plan.info()
    X = sa.rhs_random(prob, R)
    if which == "fp32":
        X = X.astype(np.complex64).astype(np.complex128)
    dt = torch.complex64 if which == "fp32" else torch.complex128
    Y = plan.precond_apply(to_dev(X, dt), which=which).cpu().numpy().astype(np.complex128).reshape(R, prob.Nt)
    ref = oracle.precond_apply(prob, X, inf["Px"], inf["Py"])
    assert_parity(Y, ref, TOL[which], N=prob.N, what=f"{which} {case}")
    plan.close()


def test_precond_rebuild_then_solve(tp):
    """A second precond_create moves the preconditioner to a new buffer (the
    old one is freed): solves after it must use the new one, not graphs
    captured with the old pointers."""
    banner("precond rebuild then solve")
    import torch
    prob = sa.make_problem(6, 5, 12, 9, 48)
    V = sa.rhs_random(prob, 2)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=2, restart=20).precond_create()
    v = to_dev(V)
    for mode in ("mixed", "fp64"):
        x0, i0 = plan.solve(v, mode=mode, tol=1e-9, precond=True)
        assert all(i["status"] == 0 for i in i0)
    old = plan.pbuf
    plan.precond_create()
    del old
    junk = torch.full((1 << 22,), float("nan"), dtype=torch.float64, device="cuda:0")   # reuse freed memory
    for mode in ("mixed", "fp64"):
        x, info = plan.solve(v, mode=mode, tol=1e-9, precond=True)
        assert all(i["status"] == 0 for i in info), (mode, info)
        assert np.all(oracle.relres(prob, x.cpu().numpy(), V) <= 1e-9), mode
    del junk
    plan.close()


def test_precond_bytes_host_formula(tp):
    """The host-side size used for HBM admission equals the library's."""
    import ctypes
    from paper_2506_04710_amd import _lib
    for shape in [(3, 2, 4, 5), (8, 8, 32, 0), (9, 9, 96, 72), (17, 5, 7, 3)]:
        prob = sa.make_problem(*shape, 90)
        plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=1, restart=4)
        n = ctypes.c_size_t(0)
        _lib.check(_lib.lib().toeplitz_precond_bytes(plan._h, ctypes.byref(n)))
        assert n.value == tp.precond_bytes(*shape, "mixed", symmetric=True), shape
        plan.close()


def test_precond_errors(tp):
    banner("precond errors")
    import torch
    from paper_2506_04710_amd import _lib
    prob = sa.make_problem(3, 3, 4, 2, 77)
    p32 = tp.Plan.from_problem(prob, prec="fp32", max_rhs=1, restart=4)
    with pytest.raises(_lib.ToeplitzError) as ei:
        p32.precond_create()
    assert ei.value.status == _lib.TP_E_UNSUPPORTED
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=1, restart=8)
    x = to_dev(sa.rhs_random(prob, 1)[0])
    with pytest.raises(_lib.ToeplitzError):
        plan.precond_apply(x)
    with pytest.raises(_lib.ToeplitzError):
        plan.solve(x, precond=True)
    # a singular spectrum block: every generator zero
    z = tp.Plan.create(3, 3, 4, 0, np.zeros((5, 5, 4, 4)), prec="fp64", max_rhs=1, restart=4)
    with pytest.raises(_lib.ToeplitzError) as ei:
        z.precond_create()
    assert ei.value.status == _lib.TP_E_BREAKDOWN
    for p in (p32, plan, z):
        p.close()


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_preconditioned_solve_config1(tp, mode):
    banner(f"preconditioned solve config 1 {mode}")
    prob, V = sa.make_config(1)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=1, restart=40).precond_create()
    v = to_dev(V)
    x, info = plan.solve(v, mode=mode, tol=1e-10, precond=True)
    x0, info0 = plan.solve(v, mode=mode, tol=1e-10)
    assert info[0]["status"] == 0 and info[0]["relres"] <= 1e-10
    X = x.cpu().numpy().reshape(1, -1)
    assert oracle.relres(prob, X, V)[0] <= 1e-10
    ref = oracle.lu_solve(oracle.assemble(prob), V)
    assert rel_err(X, ref) <= 1e-8
    print(f"config 1 {mode}: preconditioned {info[0]['iters']} steps, plain {info0[0]['iters']} steps")
    assert info[0]["iters"] <= info0[0]["iters"]
    plan.close()


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_preconditioned_solve_multi_column_nonreciprocal(tp, mode):
    banner(f"preconditioned multi-column solve {mode}")
    prob = sa.make_problem(6, 5, 12, 9, 46)
    rim_er = random_rim_er(prob, 7)
    V = sa.rhs_random(prob, 3)
    plan = tp.Plan.create(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, rim_er=rim_er,
                          prec="mixed", max_rhs=3, restart=20).precond_create()
    x, info = plan.solve(to_dev(V), mode=mode, tol=1e-9, precond=True)
    assert all(i["status"] == 0 for i in info), info
    op = oracle.Operator(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, rim_er)
    assert np.all(oracle.relres(op, x.cpu().numpy(), V) <= 1e-9)
    plan.close()


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_preconditioned_solve_config2(tp, mode):
    """32 x 32, b = 64, 256 rim functions, broadside: fewer Arnoldi steps with the
    preconditioner, same accuracy (oracle rows sampled)."""
    banner(f"preconditioned solve config 2 {mode}")
    prob, V = sa.make_config(2)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=1, restart=40).precond_create()
    v = to_dev(V)
    x, info = plan.solve(v, mode=mode, tol=1e-8, precond=True)
    _, info0 = plan.solve(v, mode=mode, tol=1e-8)
    assert info[0]["status"] == 0 and info[0]["relres"] <= 1e-8
    print(f"config 2 {mode}: preconditioned {info[0]['iters']} steps / {info[0]['outer_iters']} refinements, "
          f"plain {info0[0]['iters']} / {info0[0]['outer_iters']}")
    assert info[0]["iters"] < info0[0]["iters"]
    # the oracle's FP64 residual over all 65,792 rows
    X = x.cpu().numpy().reshape(1, -1)
    rr = oracle.relres(prob, X, V)[0]
    print(f"config 2 {mode}: oracle relres {rr:.3e}, library {info[0]['relres']:.3e}")
    assert rr <= 1e-8
    assert abs(rr - info[0]["relres"]) <= 1e-3 * rr + 1e-14
    plan.close()


def test_preconditioned_batch_engine(tp):
    """Continuous batching with the preconditioner: columns admitted by hand
    converge to the tolerance."""
    banner("preconditioned batch engine")
    import ctypes
    import torch
    from paper_2506_04710_amd import _lib
    L = _lib.lib()
    prob = sa.make_problem(5, 4, 8, 0, 78)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=2, restart=20).precond_create()
    o = _lib.SolveOpts()
    L.toeplitz_solve_opts_default(ctypes.byref(o))
    o.restart, o.mode, o.tol, o.precond = 20, _lib.PREC["mixed"], 1e-9, 1
    V = sa.rhs_random(prob, 2)
    v = [to_dev(V[r]) for r in range(2)]
    x = [torch.empty_like(v[r]) for r in range(2)]
    vp = ctypes.c_void_p
    sh = vp(torch.cuda.current_stream().cuda_stream)
    _lib.check(L.toeplitz_batch_begin(plan._h, ctypes.byref(o)))
    for r in range(2):
        _lib.check(L.toeplitz_batch_admit(plan._h, r, vp(v[r].data_ptr()), vp(x[r].data_ptr()), 1e-9, 0, sh))
    phases = (ctypes.c_int * 2)()
    infos = (_lib.SolveInfo * 2)()
    for _ in range(300):
        _lib.check(L.toeplitz_batch_step(plan._h, 1))
        _lib.check(L.toeplitz_batch_poll(plan._h, 0, 1, phases, infos))
        if phases[0] == 2 and phases[1] == 2:
            break
    assert phases[0] == 2 and phases[1] == 2
    _lib.check(L.toeplitz_batch_end(plan._h))
    X = np.stack([x[r].cpu().numpy() for r in range(2)])
    assert np.all(oracle.relres(prob, X, V) <= 1e-9)
    plan.close()
