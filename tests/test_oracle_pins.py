"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test checks the oracle against the paper's worked examples, closed forms,
library routines or brute force, so that a dropped term, a sign or index slip or
a transposed operand in the oracle fails at least one of them.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg

from synth import arrays as sa

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")


def _random_op(orc, Nx, Ny, b, Nr, seed, reciprocal=False):
    """Operator with unstructured random (non-symmetric) blocks."""
    rng = np.random.default_rng(seed)
    N = Nx * Ny * b
    c = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    gen = c(2 * Ny - 1, 2 * Nx - 1, b, b)
    rim_er = None if reciprocal else c(N, Nr)
    return orc.Operator(Nx, Ny, b, Nr, gen, c(Nr, N), c(Nr, Nr), rim_er)


# ------------------------------------------------------------------ inputs
def test_generator_reciprocity_bitwise():
    prob = sa.make_problem(3, 4, 5, 6, 11)
    g = prob.gen
    # Z_{-m,-n}[q, p] == Z_{m,n}[p, q] for every offset, bit for bit
    flipped = np.ascontiguousarray(g[::-1, ::-1].transpose(0, 1, 3, 2))
    assert np.array_equal(flipped.view(np.uint64), g.view(np.uint64))


def test_generator_deterministic():
    a = sa.make_problem(2, 3, 4, 5, 7)
    b = sa.make_problem(2, 3, 4, 5, 7)
    assert np.array_equal(a.gen, b.gen) and np.array_equal(a.rim_re, b.rim_re)


# --------------------------------------------------------------- assembly
def test_assembly_equals_kronecker_sum(orc):
    """Z's element part equals sum_{m,n} S_y^n (x) S_x^m (x) Z_{m,n} (shift matrices)."""
    Nx, Ny, b, Nr = 3, 4, 2, 3
    op = _random_op(orc, Nx, Ny, b, Nr, 1)
    Z = orc.assemble(op)
    N = op.N
    A = np.zeros((N, N), dtype=complex)
    for n in range(-(Ny - 1), Ny):
        for m in range(-(Nx - 1), Nx):
            Sy = np.eye(Ny, k=-n)      # ones where iy - ly = n
            Sx = np.eye(Nx, k=-m)
            A += np.kron(Sy, np.kron(Sx, op.gen[n + Ny - 1, m + Nx - 1]))
    assert np.array_equal(Z[:N, :N], A)
    assert np.array_equal(Z[N:, :N], op.rim_re)
    assert np.array_equal(Z[:N, N:], op.rim_er)
    assert np.array_equal(Z[N:, N:], op.rim_rr)


def test_assembly_reciprocal_rim_is_transpose(orc):
    op = _random_op(orc, 2, 2, 3, 4, 2, reciprocal=True)
    Z = orc.assemble(op)
    assert np.array_equal(Z[:op.N, op.N:], op.rim_re.T)


def test_assembly_equals_geometry(orc):
    """Synthetic Z equals the kernel evaluated between absolute basis positions."""
    prob = sa.make_problem(3, 2, 4, 5, 3)
    Z = orc.assemble(prob)
    c, t = prob.centres, prob.tangents
    dx = c[:, 0][:, None] - c[:, 0][None, :]
    dy = c[:, 1][:, None] - c[:, 1][None, :]
    r = np.maximum(np.hypot(dx, dy), sa.R_CLAMP)
    ref = np.exp(-1j * prob.k * r) / (4 * np.pi * r) * (t @ t.T)
    ref[np.arange(prob.Nt), np.arange(prob.Nt)] += sa.DIAG_SHIFT
    assert np.max(np.abs(Z - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.array_equal(Z, Z.T)       # reciprocity (Sec. II-A): plain transpose


def test_scalar_toeplitz_matches_scipy(orc):
    """b = 1, Ny = 1, no rim: Z is the scalar Toeplitz matrix of scipy.linalg.toeplitz."""
    Nx = 7
    op = _random_op(orc, Nx, 1, 1, 0, 4)
    g = op.gen[0, :, 0, 0]                      # g[m + Nx - 1] = Z_m
    col = g[Nx - 1:]                            # Z[i, 0] = Z_i
    row = g[Nx - 1::-1]                         # Z[0, j] = Z_{-j}
    assert np.array_equal(orc.assemble(op), scipy.linalg.toeplitz(col, row))


def test_two_level_structure_scipy(orc):
    """b = 1, no rim: outer Toeplitz over y of inner Toeplitz blocks over x."""
    Nx, Ny = 3, 4
    op = _random_op(orc, Nx, Ny, 1, 0, 5)
    g = op.gen[:, :, 0, 0]
    Z = orc.assemble(op)
    inner = [scipy.linalg.toeplitz(g[n + Ny - 1, Nx - 1:], g[n + Ny - 1, Nx - 1::-1])
             for n in range(-(Ny - 1), Ny)]
    for iy in range(Ny):
        for ly in range(Ny):
            blk = Z[iy * Nx:(iy + 1) * Nx, ly * Nx:(ly + 1) * Nx]
            assert np.array_equal(blk, inner[iy - ly + Ny - 1])


# ------------------------------------------------------- paper's examples
def test_paper_part_numbering_worked_example(orc):
    gold = json.load(open(GOLDEN))["part_pairs_4x6"]
    parts = orc.paper_parts(gold["Nx"], gold["Ny"])
    for (a, b_), (c, d) in gold["equal_pairs"]:
        pa, pb, pc, pd = parts[a - 1], parts[b_ - 1], parts[c - 1], parts[d - 1]
        assert pa[0] == pc[0] and pb[0] == pd[0]           # same components
        off1 = (pb[1] - pa[1], pb[2] - pa[2])
        off2 = (pd[1] - pc[1], pd[2] - pc[2])
        assert off1 == off2                                # translation-equal pair
    # element parts: part e + 1 is the element the oracle numbers e = iy*Nx + ix
    Nx = gold["Nx"]
    for e in range(gold["Nx"] * gold["Ny"]):
        comp, col, row = parts[e]
        assert comp == 5 and row * Nx + col == e


def test_paper_part_numbering_rejects_y_fastest(orc):
    """The worked example fails if elements are numbered y fastest."""
    gold = json.load(open(GOLDEN))["part_pairs_4x6"]
    Nx, Ny = gold["Nx"], gold["Ny"]
    pos = lambda k: ((k - 1) // Ny, (k - 1) % Ny)      # y-fastest alternative
    (a, b_), (c, d) = gold["equal_pairs"][0]
    off1 = tuple(np.subtract(pos(b_), pos(a)))
    off2 = tuple(np.subtract(pos(d), pos(c)))
    assert off1 != off2


def test_part_count(orc):
    gold = json.load(open(GOLDEN))["part_count"]
    for Nx, Ny, PN in gold["cases"]:
        assert orc.part_count(Nx, Ny) == PN == len(orc.paper_parts(Nx, Ny))


def test_unique_generator_blocks(orc):
    """Distinct blocks of A up to transposition = Nx Ny + (Nx-1)(Ny-1)."""
    gold = json.load(open(GOLDEN))["unique_A_blocks"]
    for Nx, Ny, count in gold["cases"]:
        prob = sa.make_problem(Nx, Ny, 3, 0, 100 + Nx * 10 + Ny)
        Z = orc.assemble(prob)
        b = 3
        seen = set()
        E = Nx * Ny
        for i in range(E):
            for j in range(E):
                blk = Z[i * b:(i + 1) * b, j * b:(j + 1) * b]
                seen.add(min(blk.tobytes(), np.ascontiguousarray(blk.T).tobytes()))
        assert len(seen) == count == Nx * Ny + (Nx - 1) * (Ny - 1)
        assert count == orc.memory_units(Nx, Ny, [0, 0, 0, 0, 0, 1, 0, 0, 0, 0])["A"]


def test_memory_formula_reduction(orc):
    """The reduced memory count of Sec. II-C follows from the Appendix formulas."""
    rng = np.random.default_rng(0)
    for Nx, Ny in [(4, 6), (9, 9), (32, 32), (1, 7)]:
        eE, em, ec = (int(v) for v in rng.integers(1, 500, size=3))
        e = [0, ec, em, ec, em, eE, em, ec, em, ec]     # e_1..e_9 by component class
        assert orc.memory_units(Nx, Ny, e)["total"] == orc.memory_units_reduced(Nx, Ny, eE, em, ec)


def test_full_matrix_is_complex128():
    gold = json.load(open(GOLDEN))["full_matrix_bytes"]
    for edges, reported, _sig in gold["cases"]:
        assert abs(edges ** 2 * 16 - reported) / reported < 5e-3
        assert abs(edges ** 2 * 8 - reported) / reported > 0.4


# ------------------------------------------------------------- products
def test_matvec_matches_numpy(orc):
    op = _random_op(orc, 3, 2, 4, 5, 6)
    Z = orc.assemble(op)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((3, op.Nt)) + 1j * rng.standard_normal((3, op.Nt))
    ref = (Z @ X.T).T
    for Y in (orc.matvec(op, X), orc.dense_matvec(Z, X)):
        assert np.max(np.abs(Y - ref)) <= 1e-13 * np.max(np.abs(ref))
    rows = np.array([0, 5, op.Nt - 1, op.N])
    assert np.allclose(orc.matvec(op, X, rows=rows), ref[:, rows], rtol=1e-13, atol=0)


@pytest.mark.parametrize("pad", [(0, 0), (1, 0), (3, 2)])
def test_circulant_embedding_identity(orc, pad):
    Nx, Ny, b = 3, 4, 2
    op = _random_op(orc, Nx, Ny, b, 0, 7)
    Z = orc.assemble(op)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    Px, Py = 2 * Nx - 1 + pad[0], 2 * Ny - 1 + pad[1]
    y = orc.circulant_product(op, x, Px, Py)
    ref = Z @ x
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_circulant_too_small_aliases(orc):
    """Below 2N-1 the embedding wraps around: the identity must fail."""
    Nx, Ny, b = 3, 3, 1
    op = _random_op(orc, Nx, Ny, b, 0, 8)
    x = np.ones(op.N, dtype=complex)
    y = orc.circulant_product(op, x, 2 * Nx - 2, 2 * Ny - 1)
    assert np.max(np.abs(y - orc.assemble(op) @ x)) > 1e-3


def test_spectrum_single_generator_closed_form(orc):
    Nx, Ny, b = 3, 4, 2
    Px, Py = 6, 9
    for (m0, n0) in [(0, 0), (1, -2), (-2, 3)]:
        gen = np.zeros((2 * Ny - 1, 2 * Nx - 1, b, b), dtype=complex)
        blk = np.array([[1 + 2j, -0.5j], [3.0, 0.25 - 1j]])
        gen[n0 + Ny - 1, m0 + Nx - 1] = blk
        op = orc.Operator(Nx, Ny, b, 0, gen)
        kx, ky = np.meshgrid(np.arange(Px), np.arange(Py), indexing="ij")
        S = orc.spectrum(op, Px, Py, kx.ravel(), ky.ravel())
        ph = np.exp(-2j * np.pi * (kx.ravel() * m0 / Px + ky.ravel() * n0 / Py)) / (Px * Py)
        assert np.max(np.abs(S - ph[:, None, None] * blk)) <= 1e-15


def test_spectrum_matches_numpy_fft(orc):
    Nx, Ny, b = 3, 2, 2
    Px, Py = 5, 4
    op = _random_op(orc, Nx, Ny, b, 0, 9)
    grid = np.zeros((Py, Px, b, b), dtype=complex)
    for n in range(-(Ny - 1), Ny):
        for m in range(-(Nx - 1), Nx):
            grid[n % Py, m % Px] = op.gen[n + Ny - 1, m + Nx - 1]
    ref = np.fft.fft2(grid, axes=(0, 1)) / (Px * Py)          # [ky, kx]
    kx, ky = np.meshgrid(np.arange(Px), np.arange(Py), indexing="xy")
    S = orc.spectrum(op, Px, Py, kx.ravel(), ky.ravel())
    assert np.max(np.abs(S - ref.reshape(-1, b, b))) <= 1e-14 * np.max(np.abs(ref))


def test_convolution_theorem_route(orc):
    """crop(IDFT(P * G_hat . DFT(x_pad))) equals the dense element product."""
    Nx, Ny, b = 3, 4, 2
    Px, Py = 6, 8
    op = _random_op(orc, Nx, Ny, b, 0, 10)
    kx, ky = np.meshgrid(np.arange(Px), np.arange(Py), indexing="xy")
    G = orc.spectrum(op, Px, Py, kx.ravel(), ky.ravel()).reshape(Py, Px, b, b)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    xp = np.zeros((Py, Px, b), dtype=complex)
    xp[:Ny, :Nx] = x.reshape(Ny, Nx, b)
    xh = np.fft.fft2(xp, axes=(0, 1))
    yh = np.einsum("yxpq,yxq->yxp", G, xh) * (Px * Py)
    y = np.fft.ifft2(yh, axes=(0, 1))[:Ny, :Nx].reshape(-1)
    ref = orc.assemble(op) @ x
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))


# ----------------------------------------------------------------- solve
def test_lu_matches_lapack_and_backward_error(orc):
    prob = sa.make_problem(3, 3, 4, 6, 12)
    Z = orc.assemble(prob)
    V = sa.rhs_random(prob, 3)
    X = orc.lu_solve(Z, V)
    ref = np.linalg.solve(Z, V.T).T
    assert np.max(np.abs(X - ref)) <= 1e-12 * np.max(np.abs(ref))
    u = np.finfo(float).eps / 2
    for r in range(3):
        be = np.linalg.norm(Z @ X[r] - V[r]) / (np.linalg.norm(Z, 2) * np.linalg.norm(X[r]) + np.linalg.norm(V[r]))
        assert be <= 10 * prob.Nt * u


def test_lu_pivots_and_detects_singularity(orc):
    A = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 9]], dtype=complex)   # zero leading pivot
    v = np.array([[1, 2, 3]], dtype=complex)
    x = orc.lu_solve(A, v)
    assert np.allclose(A @ x[0], v[0], rtol=0, atol=1e-13)
    with pytest.raises(np.linalg.LinAlgError):
        orc.lu_solve(np.array([[1, 2], [2, 4]], dtype=complex), np.ones((1, 2)))


def test_lu_single_element_is_dense_solve(orc):
    """Nx = Ny = 1: the operator is one dense block plus the rim."""
    prob = sa.make_problem(1, 1, 6, 3, 13)
    Z = orc.assemble(prob)
    assert np.array_equal(Z[:6, :6], prob.gen[0, 0])
    V = sa.rhs_random(prob, 1)
    assert np.allclose(orc.lu_solve(Z, V)[0], scipy.linalg.solve(Z, V[0]), rtol=1e-12, atol=0)


def test_relres_of_exact_solution(orc):
    prob = sa.make_problem(2, 3, 4, 5, 14)
    Z = orc.assemble(prob)
    V = sa.rhs_random(prob, 2)
    X = orc.lu_solve(Z, V)
    assert np.all(orc.relres(prob, X, V) < 1e-13)
    assert np.all(orc.relres(prob, X * (1 + 1e-6), V) > 1e-7)


# ------------------------------------------------------------ post-steps
def test_s_matrix_closed_forms(orc):
    Z0 = 50.0
    assert np.allclose(orc.s_matrix(np.eye(4) / Z0, Z0), 0, atol=1e-14)   # matched ports
    z = 30 - 20j                                                           # one port
    assert np.isclose(orc.s_matrix(np.array([[1 / z]]), Z0)[0, 0], (z - Z0) / (z + Z0))
    rng = np.random.default_rng(4)
    Zp = rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5))
    Zp = Zp + Zp.T + 20 * np.eye(5)
    S = orc.s_matrix(np.linalg.inv(Zp), Z0)
    assert np.allclose(S, S.T, atol=1e-12)                                # reciprocity


def test_tarc(orc):
    a = np.array([1, 1j, -1, 0.5])
    assert orc.tarc(np.zeros((4, 4)), a) == 0.0
    Q, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((4, 4)) + 0j)
    assert np.isclose(orc.tarc(Q, a), 1.0)


def test_far_field_single_dipole_and_array_factor(orc):
    k, eta = 2 * np.pi, orc.ETA0
    c = np.array([[0.3, -0.2, 0.0]])
    t = np.array([[1.0, 0.0, 0.0]])
    th, ph = np.array([30.0, -45.0]), np.array([0.0, 90.0])
    Ft, Fp = orc.far_field(c, t, [2.0 + 1j], th, ph)
    for a in range(2):
        tr, pr = np.deg2rad(th[a]), np.deg2rad(ph[a])
        rh = np.array([np.sin(tr) * np.cos(pr), np.sin(tr) * np.sin(pr), np.cos(tr)])
        et = np.array([np.cos(tr) * np.cos(pr), np.cos(tr) * np.sin(pr), -np.sin(tr)])
        ref = -1j * k * eta * (2 + 1j) * et[0] * np.exp(1j * k * rh @ c[0])
        assert np.isclose(Ft[a], ref, rtol=1e-13)
    # a line of identical in-phase dipoles radiates n times one dipole at broadside
    n = 6
    cs = np.stack([np.arange(n) * 0.5, np.zeros(n), np.zeros(n)], axis=1)
    ts = np.tile([[0.0, 1.0, 0.0]], (n, 1))
    F1 = orc.far_field(cs[:1], ts[:1], [1.0], [0.0], [90.0])[0]
    Fn = orc.far_field(cs, ts, np.ones(n), [0.0], [90.0])[0]
    assert np.isclose(Fn[0], n * F1[0], rtol=1e-13)


# ------------------------------------------------------------- preconditioner
def test_circulant_matrix_cropped_is_the_operator(orc):
    """C_P applied to the zero-padded x_A and cropped is A x_A (P >= 2N - 1)."""
    prob = sa.make_problem(3, 2, 4, 0, 71)
    Px, Py = 5, 4
    C = orc.circulant_matrix(prob, Px, Py)
    x = sa.rhs_random(prob, 1)[0]
    w = np.zeros(Px * Py * prob.b, dtype=complex)
    for iy in range(prob.Ny):
        for ix in range(prob.Nx):
            g, e = ix + iy * Px, iy * prob.Nx + ix
            w[g * prob.b:(g + 1) * prob.b] = x[e * prob.b:(e + 1) * prob.b]
    u = C @ w
    y = np.concatenate([u[(ix + iy * Px) * prob.b:(ix + iy * Px + 1) * prob.b]
                        for iy in range(prob.Ny) for ix in range(prob.Nx)])
    assert np.allclose(y, orc.matvec(prob, x)[0], rtol=0, atol=1e-13 * np.abs(y).max())
    # block-circulant: shifting both points by one grid step leaves the block unchanged
    b = prob.b
    assert np.array_equal(C[0:b, b:2 * b], C[b:2 * b, 2 * b:3 * b])


def test_precond_inverts_block_diagonal_operator(orc):
    """With only Z_{0,0} nonzero and a diagonal C the preconditioner is the exact inverse."""
    rng = np.random.default_rng(9)
    Nx, Ny, b, Nr = 3, 3, 5, 4
    gen = np.zeros((2 * Ny - 1, 2 * Nx - 1, b, b), dtype=complex)
    gen[Ny - 1, Nx - 1] = rng.standard_normal((b, b)) + 1j * rng.standard_normal((b, b)) + 4 * np.eye(b)
    op = orc.Operator(Nx, Ny, b, Nr, gen, np.zeros((Nr, Nx * Ny * b)), np.diag(rng.uniform(1, 2, Nr) + 1j))
    x = rng.standard_normal((2, op.Nt)) + 1j * rng.standard_normal((2, op.Nt))
    y = orc.precond_apply(op, orc.matvec(op, x), 5, 6)
    assert np.allclose(y, x, rtol=0, atol=1e-12)


def test_precond_matches_fft_circulant_solve(orc):
    """Element part equals the circulant solve done by numpy FFT and per-frequency inverses."""
    prob = sa.make_problem(3, 2, 4, 5, 72)
    Px, Py = 6, 3
    x = sa.rhs_random(prob, 2)
    y = orc.precond_apply(prob, x, Px, Py)
    b, Nx, Ny = prob.b, prob.Nx, prob.Ny
    placed = np.zeros((Px, Py, b, b), dtype=complex)
    for n in range(-(Ny - 1), Ny):
        for m in range(-(Nx - 1), Nx):
            placed[m % Px, n % Py] = prob.gen[n + Ny - 1, m + Nx - 1]
    Ch = np.fft.fft2(placed, axes=(0, 1))
    for r in range(2):
        w = np.zeros((Px, Py, b), dtype=complex)
        w[:Nx, :Ny] = x[r, :prob.N].reshape(Ny, Nx, b).transpose(1, 0, 2)
        Wh = np.fft.fft2(w, axes=(0, 1))
        z = np.fft.ifft2(np.linalg.solve(Ch, Wh[..., None])[..., 0], axes=(0, 1))
        ref = z[:Nx, :Ny].transpose(1, 0, 2).reshape(-1)
        assert np.allclose(y[r, :prob.N], ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        assert np.allclose(y[r, prob.N:], x[r, prob.N:] / np.diag(prob.rim_rr), rtol=1e-14)
