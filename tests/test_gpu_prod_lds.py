"""The FP32 product with the spectrum block staged in LDS (TP_OPT_PROD_LDS),
per frequency and in the pair form (one workgroup per stored block of a half
spectrum, applied to its frequency and transposed to the mirror), against the
streaming product bit for bit, over row and column shapes, odd b, half and
full spectra, placed rims and solver-idle columns; the option's checks and
its fallback where the workgroup would not fit."""
import numpy as np
import pytest

import oracle
from synth import arrays as sa
from helpers import assert_parity, banner, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2506_04710_amd as tp
    tp.load()
    return tp


def _bits(y):
    return y.view(np.uint32 if y.dtype == np.complex64 else np.uint64)


# (Nx, Ny, b, Nr, R, full spectrum)
CASES = [(4, 4, 16, 24, 16, False), (5, 3, 33, 10, 40, True), (3, 3, 64, 20, 81, False), (4, 3, 96, 12, 20, True),
         (3, 2, 104, 8, 33, False), (2, 2, 128, 6, 17, False)]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}b{c[2]}R{c[4]}{'full' if c[5] else 'half'}"
                                             for c in CASES])
@pytest.mark.parametrize("which", ["fp32", "mixed"])
def test_prod_lds_bitwise(tp, case, which):
    import torch
    from paper_2506_04710_amd import _lib
    Nx, Ny, b, Nr, R, full = case
    banner(f"LDS product {which} {case}")
    prob = sa.make_problem(Nx, Ny, b, Nr, 9300 + b)
    gen = prob.gen.copy()
    if full:
        rng = np.random.default_rng(b)
        gen = gen + 0.01 * (rng.standard_normal(gen.shape) + 1j * rng.standard_normal(gen.shape))
    plan = tp.Plan.create(Nx, Ny, b, Nr, gen, prob.rim_re, prob.rim_rr, prec="mixed", max_rhs=R, restart=4)
    assert plan.info()["half_spectrum"] == (0 if full else 1)
    X = sa.rhs_random(prob, R, rng=np.random.default_rng(R))
    dt = torch.complex64 if which == "fp32" else torch.complex128
    if which == "fp32":
        X = X.astype(np.complex64).astype(np.complex128)
    x = to_dev(X, dt)
    plan.set_option(_lib.TP_OPT_MFMA_COLS, 32)
    y0 = plan.matvec(x, which=which).cpu().numpy()
    nrt = (b + 15) // 16
    ran = 0
    for pair in (0, 256):
        for cg in (1, 2, 3, 6, 15):
            for rt in (2, 3, 6):
                plan.set_option(_lib.TP_OPT_PROD_LDS, pair + cg * 16 + rt)
                y1 = plan.matvec(x, which=which).cpu().numpy()
                assert np.array_equal(_bits(y0), _bits(y1)), (pair, cg, rt)
                ran += cg * -(-nrt // rt) <= 16
    assert ran >= 18
    op = oracle.Operator(Nx, Ny, b, Nr, gen, prob.rim_re, prob.rim_rr)
    assert_parity(y1.astype(np.complex128).reshape(X.shape), oracle.matvec(op, X), 1e-5, N=prob.N, what=which)
    plan.close()


def test_prod_lds_placed_and_idle_columns(tp):
    """A placed plan (b + rim channels) in a 24-column preconditioned solve
    with the LDS product: columns that converge early go idle in the product."""
    from paper_2506_04710_amd import _lib
    banner("LDS product in a placed 24-column solve")
    prob = sa.make_problem(6, 5, 40, 30, 9390)
    plan = tp.Plan.create(6, 5, 40, 30, prob.gen, prob.rim_re, prob.rim_rr, prec="mixed", max_rhs=24, restart=30,
                          rim_place=sa.rim_placement(prob))
    plan.set_option(_lib.TP_OPT_PROD_LDS, 256 + 3 * 16 + 2)       # the pair form (half spectrum)
    plan.precond_create()
    V = sa.rhs_random(prob, 24, rng=np.random.default_rng(5))
    V[::3] *= 1e-3                      # a spread of norms: columns finish at different steps
    x, info = plan.solve(to_dev(V), mode="mixed", tol=1e-8, precond=True)
    rr = oracle.relres(prob, x.cpu().numpy().reshape(24, -1), V)
    assert all(i["status"] == 0 for i in info) and np.all(rr <= 1e-8), (info, rr)
    plan.close()


def test_prod_lds_option_checks(tp):
    from paper_2506_04710_amd import _lib
    banner("LDS product option checks")
    prob = sa.make_problem(3, 3, 8, 0, 9391)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=16, restart=4)
    assert plan.get_option(_lib.TP_OPT_PROD_LDS) == 0
    for bad in (16 * 3 + 4, 16 * 0 + 2, 256 + 2, 512 + 16 + 2, -1):
        with pytest.raises(tp.ToeplitzError):
            plan.set_option(_lib.TP_OPT_PROD_LDS, bad)
    plan.set_option(_lib.TP_OPT_PROD_LDS, 16 * 2 + 3)
    assert plan.get_option(_lib.TP_OPT_PROD_LDS) == 16 * 2 + 3
    # the persistent launch yields to it
    plan.set_option(_lib.TP_OPT_MULTI_FUSED, 1)
    assert "persistent" not in plan.path("fp32", 16)
    plan.close()
