"""Structured rim on the CPU: the oracle's placed generator and placed
preconditioner against what fixes them (the assembled Z, the plain
preconditioner of an operator without rim), the library's host-side
placement checks, and its storage against the Appendix memory counts."""
import ctypes

import numpy as np
import pytest

from synth import arrays as sa


def _ext_index(prob, place, nrc):
    """Unknown -> index of (cell, channel) in the extended operator's ordering."""
    Nx, b, N = prob.Nx, prob.b, prob.N
    bc = b + nrc
    e = np.arange(N) // b
    return np.concatenate([e * bc + np.arange(N) % b,
                           (place[:, 1] * Nx + place[:, 0]) * bc + b + place[:, 2]])


@pytest.mark.parametrize("shape", [(4, 4, 16, 24), (3, 5, 6, 40), (5, 3, 4, 16), (2, 2, 3, 12)])
def test_placed_generator_restriction_is_Z(orc, shape):
    """The two-level block-Toeplitz operator of the placed generator, assembled
    on every (cell, channel) pair, restricted to the occupied pairs, is Z bit
    for bit (sides, corners, both ends of every row and column)."""
    Nx, Ny, b, Nr = shape
    prob = sa.make_problem(Nx, Ny, b, Nr, 8100 + Nx * 10 + Ny)
    place, nrc = sa.rim_placement(prob)
    gext = orc.placed_generator(prob, place, nrc)
    ext = orc.Operator(Nx, Ny, b + nrc, 0, gext)
    Zext = orc.assemble(ext)
    idx = _ext_index(prob, place, nrc)
    Z = orc.assemble(prob)
    assert np.array_equal(Zext[np.ix_(idx, idx)].view(np.uint64), Z.view(np.uint64))
    # the element channels are the generators themselves
    assert np.array_equal(gext[:, :, :b, :b], prob.gen)


def test_placed_generator_rejects_a_wrong_placement(orc):
    prob = sa.make_problem(4, 4, 8, 24, 8200)
    place, nrc = sa.rim_placement(prob)
    bad = place.copy()
    bad[[0, 1]] = bad[[1, 0]]                       # two parts of side 1 swap cells
    with pytest.raises(ValueError):
        orc.placed_generator(prob, bad, nrc)
    bad = place.copy()
    bad[prob.Ny:2 * prob.Ny, 2] = place[:prob.Ny, 2]    # side 2 on side 1's channels
    with pytest.raises(ValueError):
        orc.placed_generator(prob, bad, nrc)
    # a whole component moved to another column changes no coupling offset pattern
    ok = place.copy()
    ok[prob.Ny:2 * prob.Ny, 0] = 1
    orc.placed_generator(prob, ok, nrc)


def test_placed_precond_full_occupancy_is_plain_precond(orc):
    """With a rim function at every cell and rim channel, the restriction is
    the whole extended operator, so the placed preconditioner is the plain
    block-circulant preconditioner of the extended operator (no rim)."""
    prob = sa.make_problem(3, 3, 4, 12, 8300)
    place, nrc = sa.rim_placement(prob)
    gext = orc.placed_generator(prob, place, nrc)
    Nx, Ny, b = 3, 3, 4
    bc = b + nrc
    ext = orc.Operator(Nx, Ny, bc, 0, gext)
    Zext = orc.assemble(ext)
    # the same operator with every rim channel of every cell as a rim function
    full = np.array([(cx, cy, c) for cy in range(Ny) for cx in range(Nx) for c in range(nrc)], dtype=np.int32)
    Nr = len(full)
    N = Nx * Ny * b
    e = np.arange(N) // b
    idx = np.concatenate([e * bc + np.arange(N) % b, (full[:, 1] * Nx + full[:, 0]) * bc + b + full[:, 2]])
    Zp = Zext[np.ix_(idx, idx)]
    op = orc.Operator(Nx, Ny, b, Nr, gext[:, :, :b, :b], Zp[N:, :N], Zp[N:, N:], Zp[:N, N:])
    rng = np.random.default_rng(5)
    X = rng.standard_normal((2, N + Nr)) + 1j * rng.standard_normal((2, N + Nr))
    for Px, Py in ((5, 5), (6, 7)):
        got = orc.placed_precond_apply(op, X, full, nrc, Px, Py)
        Xe = np.zeros((2, Nx * Ny * bc), dtype=np.complex128)
        Xe[:, idx] = X
        want = orc.precond_apply(ext, Xe, Px, Py)[:, idx]
        assert np.allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_placed_precond_without_rim_is_plain_precond(orc):
    """The placed preconditioner's element channels read and write exactly the
    plain preconditioner's slots: with the rim couplings switched off, rim
    unknowns see only their own C block."""
    prob = sa.make_problem(3, 4, 5, 14, 8400)
    place, nrc = sa.rim_placement(prob)
    op = orc.Operator(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, np.zeros_like(prob.rim_re),
                      np.diag(np.diag(prob.rim_rr)))
    rng = np.random.default_rng(6)
    X = rng.standard_normal((1, prob.Nt)) + 1j * rng.standard_normal((1, prob.Nt))
    got = orc.placed_precond_apply(op, X, place, nrc, 5, 7)
    want = orc.precond_apply(op, X, 5, 7)       # x_r / diag(C) for the rim
    assert np.allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


@pytest.fixture(scope="module")
def L():
    from paper_2506_04710_amd import _lib
    return _lib.lib()


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def test_create_placed_validates_before_device_work(L):
    from paper_2506_04710_amd import _lib
    prob = sa.make_problem(4, 4, 8, 24, 8500)
    place, nrc = sa.rim_placement(prob)
    fake = ctypes.c_void_p(0x1000)          # never dereferenced: validation fails first
    h = ctypes.c_void_p()

    def create(pl, n=nrc, rim_re=prob.rim_re, rim_er=None):
        return L.toeplitz_plan_create_placed(4, 4, 8, 24, _ptr(prob.gen), _ptr(rim_re),
                                             None if rim_er is None else _ptr(rim_er), _ptr(prob.rim_rr),
                                             None if pl is None else _ptr(pl), n, _lib.TP_FP64, 1, 8, fake,
                                             1 << 34, None, ctypes.byref(h))
    assert create(None) == _lib.TP_E_INVAL
    assert create(place, n=0) == _lib.TP_E_INVAL
    for r, col, val in ((3, 0, 4), (3, 1, -1), (5, 2, nrc)):      # cell or channel out of range
        bad = place.copy()
        bad[r, col] = val
        assert create(bad) == _lib.TP_E_INVAL
        assert b"outside" in L.toeplitz_last_error()
    bad = place.copy()
    bad[1] = bad[0]                                                 # two functions on one slot
    assert create(bad) == _lib.TP_E_INVAL and b"share" in L.toeplitz_last_error()
    bad = place.copy()
    bad[[0, 1]] = bad[[1, 0]]                                       # consistent slots, wrong couplings
    assert create(bad) == _lib.TP_E_INVAL and b"not block Toeplitz" in L.toeplitz_last_error()
    rim = prob.rim_re.copy()
    rim[2, 17] *= 1.0 + 1e-15                                       # one entry off by one ulp
    assert create(place, rim_re=rim) == _lib.TP_E_INVAL and b"not block Toeplitz" in L.toeplitz_last_error()
    er = np.ascontiguousarray(prob.rim_re.T)
    er[40, 3] += 1e-3                                               # non-reciprocal, not Toeplitz
    assert create(place, rim_er=er) == _lib.TP_E_INVAL and b"element-rim" in L.toeplitz_last_error()
    assert h.value is None


def test_placed_plan_bytes_against_the_appendix_counts(L):
    """The placed plan stores the rim in the extended spectrum: per copy
    kxh Py ((b + nrc)^2 - b^2) values instead of the dense Nr N + Nr^2.  Its
    rim share stays within a fixed factor of the Appendix count of unique rim
    entries (eqs. calcScalingB/C: O(Nx Ny)), while the dense rim (Nr N with
    Nr ~ Nx + Ny) grows one power of the side faster."""
    import oracle as orc
    from paper_2506_04710_amd import plan_bytes, plan_bytes_placed
    def grid(n):
        P = 2 * n - 1
        while True:
            m = P
            for f in (2, 3, 5, 7):
                while m % f == 0:
                    m //= f
            if m == 1:
                return P
            P += 1
    ratios_placed, ratios_dense = [], []
    for n in (8, 16, 32, 48):
        b, bm = 32, 2
        Nr = 4 * n * bm
        nrc = 4 * bm
        bc = b + nrc
        P = grid(n)
        e = [0, 0, bm, 0, bm, b, bm, 0, bm, 0]           # e1..e9 (sides bm, no corners, element b)
        mem = orc.memory_units(n, n, e)
        paper_rim = mem["B"] + mem["C"]
        for sym in (False, True):
            kxh = P // 2 + 1 if sym else P
            placed = plan_bytes_placed(n, n, b, Nr, nrc, "fp64", 1, 1, symmetric=sym)
            elem = plan_bytes(n, n, b, 0, "fp64", 1, 1, symmetric=sym)
            spec_diff = kxh * P * (bc * bc - b * b) * 16
            # beyond the extra spectrum channels: plan-time scratch and transform
            # grids widened to bc channels, mirror parts, Krylov vectors of Nt,
            # the map table
            slack = ((2 * n - 1) ** 2 + (2 * n - 1) * P) * (bc * bc - b * b) * 16 + 4 * P * P * nrc * 16 + (1 << 20)
            extra = placed - elem
            assert spec_diff <= extra <= spec_diff + slack, (n, sym, extra, spec_diff)
            if sym:
                ratios_placed.append(spec_diff / 16 / paper_rim)
                ratios_dense.append((Nr * n * n * b + Nr * Nr) / paper_rim)
    assert max(ratios_placed) / min(ratios_placed) < 1.5, ratios_placed      # same order as the Appendix
    # the dense rim grows one power of the array side faster (x6 from 8 to 48)
    assert ratios_dense[-1] / ratios_dense[0] > 5, ratios_dense
    n = ctypes.c_size_t(0)
    assert L.toeplitz_plan_bytes_placed(4, 4, 16, 24, 0, 1, 0, 1, 40, ctypes.byref(n)) == 1      # nrc 0
    assert L.toeplitz_plan_bytes_placed(4, 4, 16, 0, 4, 1, 0, 1, 40, ctypes.byref(n)) == 1       # no rim
    assert L.toeplitz_plan_bytes_placed(4, 4, 250, 24, 8, 1, 0, 1, 40, ctypes.byref(n)) == 1     # b + nrc > 256


def test_placed_symmetric_host_rule():
    """The binding's rule for the half spectrum of a placed plan (it sizes the
    device buffer): symmetric generators, reciprocal rim, symmetric C."""
    import paper_2506_04710_amd as tp
    prob = sa.make_problem(4, 4, 8, 24, 8600)
    assert tp.placed_symmetric(True, None, prob.rim_rr)
    assert not tp.placed_symmetric(False, None, prob.rim_rr)
    assert not tp.placed_symmetric(True, prob.rim_re.T, prob.rim_rr)
    rr = prob.rim_rr.copy()
    rr[3, 5] += 1e-9
    assert not tp.placed_symmetric(True, None, rr)
