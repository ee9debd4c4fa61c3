"""Data movement bit for bit: on a one-element array (Nx = Ny = 1, so every
transform has length 1 and moves no value through arithmetic) with Z a signed
permutation of the Nt unknowns, every output of the operator is one input
value, possibly negated, so every path must return exactly the permuted
vector: the embedding, the crop, the rim slabs and their gathering, the
placed rim's channel map, in FP64, FP32 and mixed, for one column (fused
pass, pair stream), several columns and the matrix-core columns."""
import numpy as np
import pytest

from helpers import banner, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2506_04710_amd as tp
    tp.load()
    return tp


def _signed_permutation(Nt, seed):
    rng = np.random.default_rng(seed)
    perm = rng.permutation(Nt)
    sign = rng.choice([-1.0, 1.0], size=Nt)
    Z = np.zeros((Nt, Nt), dtype=np.complex128)
    Z[np.arange(Nt), perm] = sign
    return Z


@pytest.mark.parametrize("placed", [False, True])
@pytest.mark.parametrize("R", [1, 3, 17])
@pytest.mark.parametrize("which", ["fp64", "fp32", "mixed"])
def test_signed_permutation_bitwise(tp, which, R, placed):
    from paper_2506_04710_amd import _lib
    import torch
    banner(f"bitwise data movement {which} R={R} placed={placed}")
    b, Nr = 12, 5
    Nt = b + Nr
    Z = _signed_permutation(Nt, 11 + R)
    gen = Z[:b, :b].reshape(1, 1, b, b)
    rim_re, rim_er, rim_rr = Z[b:, :b], Z[:b, b:], Z[b:, b:]
    kw = {"rim_place": (np.array([(0, 0, r) for r in range(Nr)], dtype=np.int32), Nr)} if placed else {}
    plan = tp.Plan.create(1, 1, b, Nr, gen, rim_re, rim_rr, rim_er=rim_er, prec="mixed", max_rhs=R, restart=4,
                          **kw)
    rng = np.random.default_rng(R)
    X = rng.standard_normal((R, Nt)) + 1j * rng.standard_normal((R, Nt))
    dt = torch.complex64 if which == "fp32" else torch.complex128
    if which == "fp32":
        X = X.astype(np.complex64)
    want = (X.astype(np.complex128) @ Z.T)
    passes = [0, _lib.TP_PASS_PAIRS] if R == 1 else [0]
    for ps in passes:
        plan.set_option(_lib.TP_OPT_SPECTRUM_PASS, ps)
        y = plan.matvec(to_dev(X, dt), which=which).cpu().numpy()
        if which == "fp32":
            assert np.array_equal(y.view(np.uint32), want.astype(np.complex64).view(np.uint32)), ps
        elif which == "mixed":
            # the FP32 operator rounds the inputs to FP32 as it reads them
            w32 = (X.astype(np.complex64).astype(np.complex128) @ Z.T)
            assert np.array_equal(y.view(np.uint64), w32.view(np.uint64)), ps
        else:
            assert np.array_equal(y.view(np.uint64), want.view(np.uint64)), ps
    plan.close()
