"""GPU parity of the operator application and of the plan-time spectrum,
through the C ABI, against the plain FP64 oracle."""
import numpy as np
import pytest

import oracle
from synth import arrays as sa
from helpers import assert_parity, banner, random_rim_er, rel_err, to_dev

pytestmark = pytest.mark.gpu
TOL64, TOL32 = 1e-10, 1e-5
TOL = {"fp64": TOL64, "fp32": TOL32, "mixed": TOL32}
WHICH = ["fp64", "fp32", "mixed"]


def _input(X, which):
    """The exact input a path reads: complex64 vectors for 'fp32'; 'fp64' and
    'mixed' take complex128 (the mixed path rounds them to FP32 itself, so its
    comparison against the oracle on the unrounded X includes that rounding)."""
    return X.astype(np.complex64).astype(np.complex128) if which == "fp32" else X


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2506_04710_amd as tp
    tp.load()
    return torch


def _matvec_case(torch, prob, X, rim_er=None, which="fp64", ld_pad=0):
    import paper_2506_04710_amd as tp
    R = X.shape[0]
    plan = tp.Plan.create(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, rim_er=rim_er,
                          prec="mixed", max_rhs=R, restart=4)
    dt = torch.complex64 if which == "fp32" else torch.complex128
    xd = torch.zeros((R, prob.Nt + ld_pad), dtype=dt, device="cuda:0")
    xd[:, :prob.Nt] = to_dev(X, dt)
    yd = torch.zeros((R, prob.Nt + ld_pad), dtype=dt, device="cuda:0")
    plan.matvec(xd[:, :prob.Nt], which=which, out=yd[:, :prob.Nt])
    torch.cuda.synchronize()
    return yd[:, :prob.Nt].cpu().numpy().astype(np.complex128), plan


CASES = [  # (Nx, Ny, b, Nr, R): ragged b against the 64-lane rows, prime and padded grids
    (4, 4, 16, 24, 1), (1, 1, 8, 0, 1), (1, 5, 4, 3, 2), (7, 2, 3, 0, 1), (5, 3, 33, 10, 3),
    (3, 4, 70, 5, 2), (17, 9, 8, 20, 1), (2, 3, 100, 7, 5), (9, 9, 96, 72, 1),
    # single columns take the fused path: multi-stage y lengths (18 = 2*3*3, 15, 9)
    (9, 8, 8, 0, 1), (5, 9, 40, 6, 1), (8, 5, 130, 3, 1),
    # 16 or more columns run on the matrix cores: ragged column blocks, b not a
    # multiple of 16 or 4, rim rows in several chunks, ragged 64-column slabs
    (4, 4, 16, 24, 16), (3, 4, 70, 5, 17), (5, 3, 33, 10, 33), (2, 3, 100, 70, 20), (9, 9, 96, 72, 40),
    (6, 4, 7, 0, 18)]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}b{c[2]}r{c[3]}R{c[4]}" for c in CASES])
@pytest.mark.parametrize("which", WHICH)
def test_matvec_parity(torch_cuda, case, which):
    Nx, Ny, b, Nr, R = case
    banner(f"matvec {which} {case}")
    prob = sa.make_problem(Nx, Ny, b, Nr, 3000 + Nx * 100 + Ny * 10 + b)
    X = _input(sa.rhs_random(prob, R), which)
    Y, _ = _matvec_case(torch_cuda, prob, X, which=which, ld_pad=3 if R > 1 else 0)
    assert_parity(Y, oracle.matvec(prob, X), TOL[which], N=prob.N, what=f"{which} {case}")


def _general_problem(Nx, Ny, b, Nr, seed):
    """A synthetic array with its generator blocks perturbed so that
    Z_{-m,-n} != Z_{m,n}^T: the plan keeps every spectrum column."""
    prob = sa.make_problem(Nx, Ny, b, Nr, seed)
    rng = np.random.default_rng(seed + 1)
    prob.gen = prob.gen + 0.05 * (rng.standard_normal(prob.gen.shape) + 1j * rng.standard_normal(prob.gen.shape))
    return prob


GENERAL_CASES = [(4, 4, 16, 24, 1), (7, 2, 3, 0, 1), (9, 8, 8, 0, 1), (5, 3, 33, 10, 3), (3, 4, 70, 5, 17),
                 (6, 4, 7, 0, 18)]


@pytest.mark.parametrize("case", GENERAL_CASES, ids=[f"{c[0]}x{c[1]}b{c[2]}r{c[3]}R{c[4]}" for c in GENERAL_CASES])
@pytest.mark.parametrize("which", WHICH)
def test_matvec_parity_general_generators(torch_cuda, case, which):
    """Generators without the symmetry: whole spectrum, every kernel path."""
    Nx, Ny, b, Nr, R = case
    banner(f"matvec general generators {which} {case}")
    prob = _general_problem(Nx, Ny, b, Nr, 5000 + Nx * 100 + Ny * 10 + b)
    X = _input(sa.rhs_random(prob, R), which)
    Y, plan = _matvec_case(torch_cuda, prob, X, which=which)
    assert plan.info()["half_spectrum"] == 0
    assert_parity(Y, oracle.matvec(prob, X), TOL[which], N=prob.N, what=f"{which} {case}")


def test_half_spectrum_storage(torch_cuda):
    """Symmetric generators: the plan stores the columns kx <= Px/2 only."""
    banner("half spectrum storage")
    import paper_2506_04710_amd as tp
    for shape in [(5, 4, 24, 12), (7, 2, 3, 0), (9, 9, 8, 0)]:
        prob = sa.make_problem(*shape, 46)
        plan = tp.Plan.from_problem(prob, prec="fp64", max_rhs=1, restart=4)
        info = plan.info()
        assert info["half_spectrum"] == 1
        assert info["spectrum_bytes"] == (info["Px"] // 2 + 1) * info["Py"] * prob.b ** 2 * 16
        gprob = _general_problem(*shape, 46)
        gplan = tp.Plan.from_problem(gprob, prec="fp64", max_rhs=1, restart=4)
        ginfo = gplan.info()
        assert ginfo["half_spectrum"] == 0
        assert ginfo["spectrum_bytes"] == ginfo["Px"] * ginfo["Py"] * prob.b ** 2 * 16
        plan.close()
        gplan.close()


@pytest.mark.parametrize("R", [1, 2])
@pytest.mark.parametrize("which", WHICH)
def test_matvec_nonreciprocal_rim(torch_cuda, which, R):
    banner(f"matvec non-reciprocal {which} R={R}")
    prob = sa.make_problem(6, 5, 12, 9, 41)
    rim_er = random_rim_er(prob, 5)
    X = _input(sa.rhs_random(prob, R), which)
    Y, _ = _matvec_case(torch_cuda, prob, X, rim_er=rim_er, which=which)
    op = oracle.Operator(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, rim_er)
    assert_parity(Y, oracle.matvec(op, X), TOL[which], N=prob.N, what=which)


def test_matvec_batch_invariant(torch_cuda):
    """A column's product does not depend on the other columns of its batch:
    batches of two or more columns run the same kernels and agree bit for bit;
    a single column runs the fused single-column path and agrees to rounding."""
    banner("matvec batch invariance")
    prob = sa.make_problem(5, 4, 24, 12, 42)
    X = sa.rhs_random(prob, 5)
    Yb, _ = _matvec_case(torch_cuda, prob, X)
    for r in range(4):
        Y2, _ = _matvec_case(torch_cuda, prob, X[r:r + 2])
        assert np.array_equal(Y2[0], Yb[r]) and np.array_equal(Y2[1], Yb[r + 1])
    for r in range(5):
        Y1, _ = _matvec_case(torch_cuda, prob, X[r:r + 1])
        assert rel_err(Y1[0], Yb[r]) <= 1e-14


def test_matvec_batch_invariant_mfma(torch_cuda):
    """From 16 columns on (matrix-core kernels) a column's product is the same
    bit for bit whatever its position in the batch and the batch's size."""
    banner("matvec batch invariance (MFMA)")
    prob = sa.make_problem(5, 4, 24, 12, 44)
    X = sa.rhs_random(prob, 21)
    for which in ("fp64", "fp32"):
        Xw = X if which == "fp64" else X.astype(np.complex64).astype(np.complex128)
        Ya, _ = _matvec_case(torch_cuda, prob, Xw, which=which)
        Yb, _ = _matvec_case(torch_cuda, prob, Xw[3:21], which=which)
        Yc, _ = _matvec_case(torch_cuda, prob, Xw[5:21], which=which)
        assert np.array_equal(Yb, Ya[3:21]) and np.array_equal(Yc, Ya[5:21]), which


@pytest.mark.parametrize("which", WHICH)
def test_matvec_nonreciprocal_rim_mfma(torch_cuda, which):
    banner(f"matvec non-reciprocal MFMA {which}")
    prob = sa.make_problem(6, 5, 12, 40, 45)
    rim_er = random_rim_er(prob, 6)
    X = _input(sa.rhs_random(prob, 19), which)
    Y, _ = _matvec_case(torch_cuda, prob, X, rim_er=rim_er, which=which)
    op = oracle.Operator(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, rim_er)
    assert_parity(Y, oracle.matvec(op, X), TOL[which], N=prob.N, what=which)


def test_matvec_repeat_bitwise(torch_cuda):
    banner("matvec repeat determinism")
    import paper_2506_04710_amd as tp
    prob = sa.make_problem(6, 6, 20, 16, 43)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=2, restart=4)
    x = to_dev(sa.rhs_random(prob, 2))
    y1 = plan.matvec(x).cpu().numpy()
    y2 = plan.matvec(x).cpu().numpy()
    assert np.array_equal(y1, y2)


def test_embed_crop_identity(torch_cuda):
    """Only Z_{0,0} = I: every stage (embed, transforms, product, crop) must return x."""
    banner("embed/crop identity")
    import paper_2506_04710_amd as tp
    Nx, Ny, b = 5, 7, 6
    gen = np.zeros((2 * Ny - 1, 2 * Nx - 1, b, b), dtype=complex)
    gen[Ny - 1, Nx - 1] = np.eye(b)
    plan = tp.Plan.create(Nx, Ny, b, 0, gen, prec="mixed", max_rhs=1, restart=4)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(Nx * Ny * b) + 1j * rng.standard_normal(Nx * Ny * b)
    y = plan.matvec(to_dev(x)).cpu().numpy()
    assert np.max(np.abs(y - x)) <= 1e-14 * np.max(np.abs(x))


def test_spectrum_parity(torch_cuda):
    banner("spectrum parity config 1")
    import paper_2506_04710_amd as tp
    prob, _ = sa.make_config(1)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=1, restart=4)
    info = plan.info()
    Px, Py = info["Px"], info["Py"]
    assert Px >= 2 * prob.Nx - 1 and Py >= 2 * prob.Ny - 1
    kx, ky = np.meshgrid(np.arange(Px), np.arange(Py), indexing="ij")
    ref = oracle.spectrum(prob, Px, Py, kx.ravel(), ky.ravel())
    got64 = np.stack([plan.spectrum(int(a), int(c), "fp64") for a, c in zip(kx.ravel(), ky.ravel())])
    got32 = np.stack([plan.spectrum(int(a), int(c), "fp32") for a, c in zip(kx.ravel(), ky.ravel())])
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got64 - ref)) <= 1e-13 * scale
    assert np.max(np.abs(got32 - ref)) <= 1e-6 * scale


def test_spectrum_parity_config2_sampled(torch_cuda):
    banner("spectrum parity config 2 sampled")
    import paper_2506_04710_amd as tp
    prob, _ = sa.make_config(2)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=1, restart=4)
    info = plan.info()
    Px, Py = info["Px"], info["Py"]
    assert (Px, Py) == (63, 63)
    ks = [(0, 0), (1, 0), (0, 1), (Px - 1, Py - 1), (31, 17), (62, 5)]
    ref = oracle.spectrum(prob, Px, Py, [k[0] for k in ks], [k[1] for k in ks])
    got = np.stack([plan.spectrum(a, c, "fp64") for a, c in ks])
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("cfg", [2, 3, 4])
@pytest.mark.parametrize("which", WHICH)
def test_matvec_full_size_sampled(torch_cuda, cfg, which):
    """Benchmark-size arrays with as many columns as the workload (config 3:
    81, the matrix-core path; config 4: 8), seeded random inputs: sampled
    output rows (element and rim) against the oracle's row sums."""
    banner(f"matvec full size config {cfg} {which}")
    import paper_2506_04710_amd as tp
    torch = torch_cuda
    prob, V = sa.make_config(cfg)
    R = V.shape[0]
    X = _input(sa.rhs_random(prob, R, rng=np.random.default_rng(700 + cfg)), which)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=R, restart=4)
    dt = torch.complex64 if which == "fp32" else torch.complex128
    Y = plan.matvec(to_dev(X, dt), which=which).cpu().numpy().astype(np.complex128).reshape(R, prob.Nt)
    rng = np.random.default_rng(cfg)
    rows = np.unique(np.concatenate([[0, prob.N - 1, prob.Nt - 1], rng.integers(0, prob.Nt, 40),
                                     prob.N + np.arange(min(prob.Nr, 8))]))
    ref = oracle.matvec(prob, X, rows=rows)
    assert_parity(Y[:, rows], ref, TOL[which], N=prob.N, rows=rows, what=f"config {cfg} {which}")
    plan.close()


@pytest.fixture(scope="module")
def config2_full():
    """The 32 x 32, b = 64, 256-rim operator on one seeded random input
    (rounded to complex64, so every path reads the same values) and the
    oracle's product over all 65,792 rows."""
    prob, _ = sa.make_config(2)
    X = sa.rhs_random(prob, 1, rng=np.random.default_rng(7002)).astype(np.complex64).astype(np.complex128)
    return prob, X, oracle.matvec(prob, X)


@pytest.mark.parametrize("which", WHICH)
def test_matvec_config2_every_row(torch_cuda, config2_full, which):
    """Headline operator (fused single-column half-spectrum path with the rim
    pass) checked on every output row, element and rim parts separately."""
    banner(f"matvec config 2 every row {which}")
    import paper_2506_04710_amd as tp
    torch = torch_cuda
    prob, X, ref = config2_full
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=1, restart=4)
    dt = torch.complex64 if which == "fp32" else torch.complex128
    Y = plan.matvec(to_dev(X, dt), which=which).cpu().numpy().astype(np.complex128).reshape(1, prob.Nt)
    e = assert_parity(Y, ref, TOL[which], N=prob.N, what=f"config 2 {which}")
    print(f"config 2 {which}: {e}")
    plan.close()


# Arrays with N >= 131072 use rim slabs of 256 columns (4 per lane): the
# fused single-column launch (b <= 64, half spectrum) and the multi-column
# rim pass, on seeded random inputs, sampled rows.
WIDE_SLAB_CASES = [(46, 46, 64, 184, 1), (64, 64, 32, 64, 3)]


@pytest.mark.parametrize("case", WIDE_SLAB_CASES, ids=[f"{c[0]}x{c[1]}b{c[2]}r{c[3]}R{c[4]}"
                                                       for c in WIDE_SLAB_CASES])
@pytest.mark.parametrize("which", WHICH)
def test_matvec_wide_rim_slabs(torch_cuda, case, which):
    Nx, Ny, b, Nr, R = case
    banner(f"matvec wide rim slabs {which} {case}")
    import paper_2506_04710_amd as tp
    torch = torch_cuda
    prob = sa.make_problem(Nx, Ny, b, Nr, 8000 + Nx + b)
    assert prob.N >= 131072
    X = _input(sa.rhs_random(prob, R, rng=np.random.default_rng(Nx * b)), which)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=R, restart=4)
    dt = torch.complex64 if which == "fp32" else torch.complex128
    Y = plan.matvec(to_dev(X, dt), which=which).cpu().numpy().astype(np.complex128).reshape(R, prob.Nt)
    rng = np.random.default_rng(b)
    rows = np.unique(np.concatenate([[0, prob.N - 1, prob.Nt - 1], rng.integers(0, prob.N, 40),
                                     prob.N + rng.integers(0, prob.Nr, 16)]))
    assert_parity(Y[:, rows], oracle.matvec(prob, X, rows=rows), TOL[which], N=prob.N, rows=rows,
                  what=f"{which} {case}")
    plan.close()
