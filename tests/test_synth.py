"""The synthetic rim has the margin structure of Sec. II-C: the side blocks of
B (eqs. submatrixB12, submatrixB34) and of C (C11, C21, C22, C33, C43, C44) are
one-level block Toeplitz, bit for bit; the corner blocks are not."""
import numpy as np
import pytest

from synth import arrays as sa


def _sides(prob):
    bm, bc = sa.margin_counts(prob.Nx, prob.Ny, prob.Nr)
    Nx, Ny = prob.Nx, prob.Ny
    starts = np.cumsum([0, Ny * bm, Ny * bm, Nx * bm, Nx * bm])
    return bm, bc, starts


@pytest.mark.parametrize("Nx,Ny,b,Nr", [(5, 4, 3, 36), (4, 4, 16, 24), (6, 3, 2, 40)])
def test_margin_counts_and_order(Nx, Ny, b, Nr):
    prob = sa.make_problem(Nx, Ny, b, Nr, 5)
    bm, bc, st = _sides(prob)
    assert 2 * (Nx + Ny) * bm + sum(bc) == Nr and max(bc) - min(bc) <= 1
    c = prob.centres[prob.N:]
    h = prob.d / 2
    # side 1 left of the hull, side 2 right, side 3 below, side 4 above
    assert np.all(c[st[0]:st[1], 0] < 0) and np.all(c[st[0]:st[1], 0] >= -h)
    assert np.all(c[st[1]:st[2], 0] >= Nx * prob.d)
    assert np.all(c[st[2]:st[3], 1] < 0) and np.all(c[st[3]:st[4], 1] >= Ny * prob.d)
    # parts of one side are translates: same offsets within the part, step d
    for s, axis in ((0, 1), (1, 1), (2, 0), (3, 0)):
        blk = c[st[s]:st[s + 1]].reshape(-1, bm, 3)
        if blk.shape[0] > 1:
            assert np.allclose(np.diff(blk[:, :, axis], axis=0), prob.d, atol=1e-12)
            assert np.array_equal(np.diff(blk[:, :, 1 - axis], axis=0), np.zeros_like(blk[1:, :, 0]))


@pytest.mark.parametrize("Nx,Ny,b,Nr", [(5, 4, 3, 36), (3, 6, 2, 40)])
def test_side_blocks_of_B_are_block_toeplitz(Nx, Ny, b, Nr):
    prob = sa.make_problem(Nx, Ny, b, Nr, 7)
    bm, _, st = _sides(prob)
    B = prob.rim_re.reshape(prob.Nr, Ny, Nx, b)        # [rim row, iy, ix, q]
    for s in (0, 1):          # eq. submatrixB12: block (part iy', element row iy) depends on iy' - iy
        Bs = B[st[s]:st[s + 1]].reshape(Ny, bm, Ny, Nx, b)
        for p in range(Ny - 1):
            for q in range(Ny - 1):
                assert np.array_equal(Bs[p, :, q], Bs[p + 1, :, q + 1])
    for s in (2, 3):          # eq. submatrixB34: block (part ix', element (ix, iy)) depends on ix' - ix, iy
        Bs = B[st[s]:st[s + 1]].reshape(Nx, bm, Ny, Nx, b)
        for p in range(Nx - 1):
            for q in range(Nx - 1):
                assert np.array_equal(Bs[p, :, :, q], Bs[p + 1, :, :, q + 1])
    # not constant: the Toeplitz blocks differ with the offset
    Bl = B[st[0]:st[1]].reshape(Ny, bm, Ny, Nx, b)
    assert not np.array_equal(Bl[0, :, 0], Bl[0, :, 1])


def test_side_blocks_of_C_are_block_toeplitz():
    Nx, Ny = 5, 4
    prob = sa.make_problem(Nx, Ny, 3, 40, 9)
    bm, bc, st = _sides(prob)
    C = prob.rim_rr - np.diag(np.full(prob.Nr, sa.DIAG_SHIFT))
    n = {0: Ny, 1: Ny, 2: Nx, 3: Nx}
    for a, c in ((0, 0), (1, 0), (1, 1), (2, 2), (3, 2), (3, 3)):      # C11, C21, C22, C33, C43, C44
        blk = C[st[a]:st[a + 1], st[c]:st[c + 1]].reshape(n[a], bm, n[c], bm)
        for i in range(n[a] - 1):
            for j in range(n[c] - 1):
                assert np.array_equal(blk[i, :, j], blk[i + 1, :, j + 1]), (a, c, i, j)
    # a side against another orientation is not Toeplitz (C31 in the paper is dense)
    blk = C[st[2]:st[3], st[0]:st[1]].reshape(Nx, bm, Ny, bm)
    assert not np.array_equal(blk[0, :, 0], blk[1, :, 1])
    assert np.array_equal(prob.rim_rr, prob.rim_rr.T)                   # reciprocity, bit for bit
