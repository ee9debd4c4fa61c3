"""The autotuner on the device: the options it picks, the JSON cache, and that
every candidate it may pick computes the same operator (the matrix-core
column tiles bit for bit; the spectrum passes to the oracle's tolerance)."""
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


def test_tune_single_column_and_cache(tp, tmp_path):
    from paper_2506_04710_amd import _lib, tune
    banner("tune single column (placed rim, preconditioner) + cache")
    prob = sa.make_problem(5, 4, 24, 36, 9800)
    plan = tp.Plan.create(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, prec="mixed",
                          max_rhs=1, restart=4, rim_place=sa.rim_placement(prob)).precond_create()
    path = str(tmp_path / "tune.json")
    rec = tune.tune(plan, "mixed", 1, reps=5, path=path)
    assert rec["source"] == "measured" and rec["candidates"] == 2
    assert rec["spectrum_pass"] in (_lib.TP_PASS_FUSED, _lib.TP_PASS_PAIRS)
    assert plan.get_option(_lib.TP_OPT_SPECTRUM_PASS) == rec["spectrum_pass"]
    assert rec["ms"] > 0 and rec["ms_default"] > 0
    X = sa.rhs_random(prob, 1)
    assert_parity(plan.matvec(to_dev(X), which="mixed").cpu().numpy().reshape(1, -1), oracle.matvec(prob, X), 1e-5,
                  N=prob.N, what="tuned")
    # a second plan of the same key takes the stored choice
    plan2 = tp.Plan.create(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, prec="mixed",
                           max_rhs=1, restart=4, rim_place=sa.rim_placement(prob)).precond_create()
    rec2 = tune.tune(plan2, "mixed", 1, path=path)
    assert rec2["source"] == "cache" and plan2.get_option(_lib.TP_OPT_SPECTRUM_PASS) == rec["spectrum_pass"]
    plan.close()
    plan2.close()


def test_mfma_column_tiles_bitwise(tp):
    """16, 32 and 64 columns per matrix-core workgroup: the same bits."""
    from paper_2506_04710_amd import _lib
    banner("MFMA column tiles bit for bit")
    prob = sa.make_problem(5, 3, 33, 10, 9801)
    R = 40
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=R, restart=4)
    X = sa.rhs_random(prob, R)
    out = {}
    for which, dt in (("fp32", "c64"), ("fp64", "c128")):
        x = to_dev(X.astype(np.complex64) if dt == "c64" else X)
        for cols in (16, 32, 64):
            plan.set_option(_lib.TP_OPT_MFMA_COLS, cols)
            out[(which, cols)] = plan.matvec(x, which=which).cpu().numpy()
        assert np.array_equal(out[(which, 16)], out[(which, 32)]) and np.array_equal(out[(which, 16)],
                                                                                     out[(which, 64)]), which
    Xr = X.astype(np.complex64).astype(np.complex128)
    assert_parity(out[("fp32", 64)].astype(np.complex128), oracle.matvec(prob, Xr), 1e-5, N=prob.N, what="fp32")
    plan.close()


def test_tune_many_columns(tp, tmp_path):
    from paper_2506_04710_amd import tune
    banner("tune 20 columns")
    prob = sa.make_problem(4, 4, 16, 24, 9802)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=20, restart=4)
    rec = tune.tune(plan, "fp32", 20, reps=5, path=str(tmp_path / "t.json"))
    # three column tiles and eighteen shapes of the LDS product (one row tile:
    # every column group 2, 3, 6 fits; per frequency and in pairs over the half
    # spectrum), each with the rim and the forward tiles in one launch and in
    # two, and the persistent launch at the default tile (a small grid on 2-D
    # tiles, even b, reciprocal dense rim)
    assert rec["mfma_cols"] in (16, 32, 64) and rec["candidates"] == 43 and rec["spectrum_pass"] == 0
    from paper_2506_04710_amd import _lib
    assert plan.get_option(_lib.TP_OPT_RIM_OVERLAP) == rec["rim_overlap"]
    assert rec["multi_fused"] in (0, 1)
    assert plan.get_option(_lib.TP_OPT_PROD_LDS) == rec["prod_lds"]
    assert plan.get_option(_lib.TP_OPT_MULTI_FUSED) == rec["multi_fused"]
    assert ("persistent" in plan.path("fp32", 20)) == (rec["multi_fused"] == 1)
    plan.close()
