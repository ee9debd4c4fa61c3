"""Plain FP64 CPU oracle for the array impedance operator and its solve.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_2506_04710_amd``) and neither imports the other;
both read their inputs from ``synth``.

What it computes, each by its plain definition:

* ``assemble`` / ``matvec``: the impedance matrix of eq. (matrixForm),
  Z = [[A, B^T], [B, C]], with A the two-level block-Toeplitz element part of
  eq. (submatrixAA): the block between element (ix, iy) (rows) and element
  (lx, ly) (columns) is the generator Z_{ix-lx, iy-ly}.  Dense rows, summed in
  index order (C, ``oracle.c``).
* ``lu_solve``: Gaussian elimination with partial pivoting (Golub & Van Loan,
  Alg. 3.4.1) for Z I = V (eq. MoMMatrixEq).
* ``circulant_product`` / ``spectrum``: the brute-force cyclic convolution and
  the placed-generator DFT that the FFT route computes (Sec. I: Toeplitz
  structure gives FFT-based products).
* ``circulant_matrix`` / ``precond_apply``: the dense block circulant of the
  placed generators and the block-circulant preconditioner built from it
  (solved by the same elimination as ``lu_solve``).
* ``s_matrix``: port currents -> admittance -> port impedance -> scattering
  matrix (Sec. III-B; Kurokawa's definition for a real, equal reference
  impedance), ``tarc`` (eq. TARC).
* ``far_field``: the direct sum of eq. (farfieldThetaPhiF) for point-dipole
  basis functions.
* ``paper_parts``: the part numbering of Sec. II-C (component order
  5, 2, 8, 6, 4, 3, 9, 1, 7; bottom-left first, x fastest) and the memory
  counts of the Appendix (eqs. calcScalingA/B/C).

Vectors are numpy arrays of shape (R, Nt): row r is column r of the
column-major Nt x R block.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

ETA0 = 376.730313668


def _lib():
    global _LIB
    if _LIB is None:
        # ORACLE_LIBRARY: another build of oracle.c (e.g. the sanitizer build)
        path = os.environ.get("ORACLE_LIBRARY") or os.path.join(_HERE, "_oracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        dp = ctypes.c_void_p
        lib.orc_assemble.argtypes = [ctypes.c_int] * 4 + [dp] * 5
        lib.orc_matvec_rows.argtypes = ([ctypes.c_int] * 4 + [dp] * 5 + [ctypes.c_int, dp,
                                        ctypes.c_long, dp, ctypes.c_int])
        lib.orc_dense_matvec.argtypes = [ctypes.c_long, dp, dp, ctypes.c_int, dp, ctypes.c_int]
        lib.orc_lu_solve.argtypes = [ctypes.c_long, dp, ctypes.c_int, dp, ctypes.c_int]
        lib.orc_lu_solve.restype = ctypes.c_int
        lib.orc_circulant_product.argtypes = [ctypes.c_int] * 3 + [dp, ctypes.c_int, ctypes.c_int, dp, dp]
        lib.orc_spectrum.argtypes = ([ctypes.c_int] * 3 + [dp, ctypes.c_int, ctypes.c_int, dp, dp,
                                     ctypes.c_long, dp, ctypes.c_int])
        lib.orc_max_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Operator:
    """The blocks that define Z: generators, rim blocks (rim_er None = reciprocal)."""

    def __init__(self, Nx, Ny, b, Nr, gen, rim_re=None, rim_rr=None, rim_er=None):
        self.Nx, self.Ny, self.b, self.Nr = int(Nx), int(Ny), int(b), int(Nr)
        self.gen = _c128(gen).reshape(2 * Ny - 1, 2 * Nx - 1, b, b)
        N = Nx * Ny * b
        self.rim_re = _c128(rim_re if rim_re is not None else np.zeros((Nr, N))).reshape(Nr, N)
        self.rim_rr = _c128(rim_rr if rim_rr is not None else np.zeros((Nr, Nr))).reshape(Nr, Nr)
        self.rim_er = None if rim_er is None else _c128(rim_er).reshape(N, Nr)

    @classmethod
    def from_problem(cls, prob):
        return cls(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr)

    @property
    def N(self):
        return self.Nx * self.Ny * self.b

    @property
    def Nt(self):
        return self.N + self.Nr

    def _args(self):
        return (self.Nx, self.Ny, self.b, self.Nr, _ptr(self.gen), _ptr(self.rim_re),
                _ptr(self.rim_er), _ptr(self.rim_rr))


def _op(x):
    return x if isinstance(x, Operator) else Operator.from_problem(x)


def assemble(op) -> np.ndarray:
    """Dense Nt x Nt complex128 matrix of eq. (matrixForm)."""
    op = _op(op)
    Z = np.empty((op.Nt, op.Nt), dtype=np.complex128)
    _lib().orc_assemble(*op._args(), _ptr(Z))
    return Z


def matvec(op, X, rows=None, nthreads: int = 0) -> np.ndarray:
    """Y = Z X row by row without storing Z.  ``rows`` selects output rows."""
    op = _op(op)
    X = _c128(np.atleast_2d(X))
    R = X.shape[0]
    assert X.shape[1] == op.Nt
    if rows is None:
        Y = np.empty((R, op.Nt), dtype=np.complex128)
        _lib().orc_matvec_rows(*op._args(), _ptr(X), R, None, 0, _ptr(Y), nthreads)
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        Y = np.empty((R, len(rows)), dtype=np.complex128)
        _lib().orc_matvec_rows(*op._args(), _ptr(X), R, _ptr(rows), len(rows), _ptr(Y), nthreads)
    return Y


def dense_matvec(Z, X, nthreads: int = 0) -> np.ndarray:
    Z = _c128(Z)
    X = _c128(np.atleast_2d(X))
    Y = np.empty_like(X)
    _lib().orc_dense_matvec(Z.shape[0], _ptr(Z), _ptr(X), X.shape[0], _ptr(Y), nthreads)
    return Y


def lu_solve(Z, V, nthreads: int = 0) -> np.ndarray:
    """Solve Z X = V by GEPP (Z is copied)."""
    A = _c128(Z).copy()
    B = _c128(np.atleast_2d(V)).copy()
    info = _lib().orc_lu_solve(A.shape[0], _ptr(A), B.shape[0], _ptr(B), nthreads)
    if info:
        raise np.linalg.LinAlgError(f"zero pivot at step {info - 1}")
    return B


def relres(op, X, V, nthreads: int = 0) -> np.ndarray:
    """Per-column ||V - Z X||_2 / ||V||_2 with the row-wise product."""
    V = _c128(np.atleast_2d(V))
    Y = matvec(op, X, nthreads=nthreads)
    return np.linalg.norm(V - Y, axis=1) / np.linalg.norm(V, axis=1)


def circulant_product(op, xA, Px, Py) -> np.ndarray:
    """Element part of Z x by brute-force cyclic convolution on a Px x Py grid."""
    op = _op(op)
    xA = _c128(xA).reshape(-1)
    assert xA.size == op.N
    y = np.empty(op.N, dtype=np.complex128)
    _lib().orc_circulant_product(op.Nx, op.Ny, op.b, _ptr(op.gen), Px, Py, _ptr(xA), _ptr(y))
    return y


def spectrum(op, Px, Py, kx, ky, nthreads: int = 0) -> np.ndarray:
    """Scaled DFT of the placed generators at frequencies (kx[t], ky[t]): [nk, b, b]."""
    op = _op(op)
    kx = np.ascontiguousarray(np.atleast_1d(kx), dtype=np.int32)
    ky = np.ascontiguousarray(np.atleast_1d(ky), dtype=np.int32)
    out = np.empty((len(kx), op.b, op.b), dtype=np.complex128)
    _lib().orc_spectrum(op.Nx, op.Ny, op.b, _ptr(op.gen), Px, Py, _ptr(kx), _ptr(ky), len(kx),
                        _ptr(out), nthreads)
    return out


def circulant_matrix(op, Px, Py) -> np.ndarray:
    """Dense block-circulant matrix C_P of the generators placed on the Px x Py
    torus (Z_{m,n} at grid point (m mod Px, n mod Py), zero elsewhere; the
    embedding behind the FFT route of Sec. I).  Grid point (gx, gy) has index
    gx + gy Px; the block between points i (row) and j (column) is the placed
    block at ((ix - jx) mod Px, (iy - jy) mod Py).  [Px Py b, Px Py b]."""
    op = _op(op)
    Nx, Ny, b = op.Nx, op.Ny, op.b
    assert Px >= 2 * Nx - 1 and Py >= 2 * Ny - 1
    placed = np.zeros((Px, Py, b, b), dtype=np.complex128)
    for n in range(-(Ny - 1), Ny):
        for m in range(-(Nx - 1), Nx):
            placed[m % Px, n % Py] = op.gen[n + Ny - 1, m + Nx - 1]
    P = Px * Py
    C = np.empty((P * b, P * b), dtype=np.complex128)
    for iy in range(Py):
        for ix in range(Px):
            i = ix + iy * Px
            for jy in range(Py):
                for jx in range(Px):
                    j = jx + jy * Px
                    C[i * b:(i + 1) * b, j * b:(j + 1) * b] = placed[(ix - jx) % Px, (iy - jy) % Py]
    return C


def precond_apply(op, X, Px, Py) -> np.ndarray:
    """Block-circulant preconditioner M^-1 (the paper names no preconditioner;
    this is the library's reading, an approximate inverse from the same
    embedding): the element part is crop(C_P^-1 pad(x_A)), with the
    Px x Py circulant system solved by Gaussian elimination with partial
    pivoting on the assembled C_P; the rim part is x_r / diag(C)."""
    op = _op(op)
    X = _c128(np.atleast_2d(X))
    R = X.shape[0]
    Nx, Ny, b, N = op.Nx, op.Ny, op.b, op.N
    P = Px * Py
    rhs = np.zeros((R, P * b), dtype=np.complex128)
    for iy in range(Ny):
        for ix in range(Nx):
            e = iy * Nx + ix
            g = ix + iy * Px
            rhs[:, g * b:(g + 1) * b] = X[:, e * b:(e + 1) * b]
    Zg = lu_solve(circulant_matrix(op, Px, Py), rhs)
    Y = np.empty_like(X)
    for iy in range(Ny):
        for ix in range(Nx):
            e = iy * Nx + ix
            g = ix + iy * Px
            Y[:, e * b:(e + 1) * b] = Zg[:, g * b:(g + 1) * b]
    if op.Nr:
        Y[:, N:] = X[:, N:] / np.diag(op.rim_rr)[None, :]
    return Y


def placed_generator(op, place, nrc) -> np.ndarray:
    """Generators of the structured rim (Sec. II-B margin parts, one-level
    block-Toeplitz rim blocks of eqs. submatrixB12/B34/C123/C456): unknown i
    sits at a cell (cx_i, cy_i) as channel ch_i (element basis p of element
    (ix, iy): cell (ix, iy), channel p; rim function r: cell place[r][0:2],
    channel b + place[r][2]).  The result gext [2Ny-1, 2Nx-1, b+nrc, b+nrc]
    holds, at offset (m, n) and channels (p, q), the entry Z[i, j] of every
    pair with cell_i - cell_j = (m, n), ch_i = p, ch_j = q (read off the
    assembled Z); offsets and channels no pair reaches stay zero.  Raises
    ValueError when two such pairs disagree (Z is then not the restriction
    of a block-Toeplitz operator in this placement)."""
    op = _op(op)
    Nx, Ny, b, Nr, N = op.Nx, op.Ny, op.b, op.Nr, op.N
    bc = b + nrc
    place = np.asarray(place, dtype=np.int64).reshape(Nr, 3)
    e = np.arange(N) // b
    cx = np.concatenate([e % Nx, place[:, 0]])
    cy = np.concatenate([e // Nx, place[:, 1]])
    ch = np.concatenate([np.arange(N) % b, b + place[:, 2]])
    Z = assemble(op)
    m = cx[:, None] - cx[None, :] + (Nx - 1)
    n = cy[:, None] - cy[None, :] + (Ny - 1)
    flat = ((n * (2 * Nx - 1) + m) * bc + ch[:, None]) * bc + ch[None, :]
    gext = np.zeros((2 * Ny - 1) * (2 * Nx - 1) * bc * bc, dtype=np.complex128)
    gext[flat.ravel()] = Z.ravel()
    if not np.array_equal(gext[flat.ravel()].view(np.uint64), Z.ravel().view(np.uint64)):
        raise ValueError("Z is not block Toeplitz in this placement")
    return gext.reshape(2 * Ny - 1, 2 * Nx - 1, bc, bc)


def placed_precond_apply(op, X, place, nrc, Px, Py) -> np.ndarray:
    """The block-circulant preconditioner of a structured-rim plan: with
    gext = placed_generator(op, place, nrc), crop(C_P^-1 pad(x)) where pad puts
    every unknown of x at its cell and channel on the Px x Py torus (zeros
    elsewhere), C_P is the block circulant of gext (circulant_matrix) and crop
    reads every unknown back from its cell and channel."""
    op = _op(op)
    X = _c128(np.atleast_2d(X))
    R = X.shape[0]
    Nx, Ny, b, Nr, N = op.Nx, op.Ny, op.b, op.Nr, op.N
    bc = b + nrc
    place = np.asarray(place, dtype=np.int64).reshape(Nr, 3)
    ext = Operator(Nx, Ny, bc, 0, placed_generator(op, place, nrc))
    e = np.arange(N) // b
    slot = np.concatenate([((e // Nx) * Px + e % Nx) * bc + np.arange(N) % b,
                           (place[:, 1] * Px + place[:, 0]) * bc + b + place[:, 2]])
    rhs = np.zeros((R, Px * Py * bc), dtype=np.complex128)
    rhs[:, slot] = X
    Zg = lu_solve(circulant_matrix(ext, Px, Py), rhs)
    return Zg[:, slot]


def max_threads() -> int:
    return int(_lib().orc_max_threads())


# ------------------------------------------------------------------ post-steps
def s_matrix(I_port, Z0: float = 50.0, edge_len=None) -> np.ndarray:
    """Scattering matrix from the p x p port-current block (Sec. III-B).

    Y = L I L with L = diag(1 / edge length); Z_port = Y^-1;
    S = (Z_port - Z0 I)(Z_port + Z0 I)^-1 (equal real reference impedance).
    """
    I_port = np.asarray(I_port, dtype=np.complex128)
    p = I_port.shape[0]
    L = np.diag(1.0 / np.asarray(edge_len, dtype=np.float64)) if edge_len is not None else np.eye(p)
    Y = L @ I_port @ L
    Zp = np.linalg.inv(Y)
    E = np.eye(p)
    return (Zp - Z0 * E) @ np.linalg.inv(Zp + Z0 * E)


def tarc(S, a) -> float:
    """Total active reflection coefficient (eq. TARC): ||S a|| / ||a||."""
    a = np.asarray(a, dtype=np.complex128)
    bvec = np.asarray(S) @ a
    return float(np.sqrt(np.sum(np.abs(bvec) ** 2) / np.sum(np.abs(a) ** 2)))


def far_field(centres, tangents, I, theta_deg, phi_deg, k=2 * np.pi, eta=ETA0):
    """Direct far-field sum for point-dipole basis functions.

    F_tau(rhat) = -j k eta sum_n I_n (e_tau(rhat) . t_n) exp(j k rhat . c_n), with
    e_theta = (cos th cos ph, cos th sin ph, -sin th), e_phi = (-sin ph, cos ph, 0).
    Returns (F_theta, F_phi), each of shape [len(theta)] (theta and phi paired).
    """
    th = np.deg2rad(np.asarray(theta_deg, dtype=np.float64))
    ph = np.deg2rad(np.asarray(phi_deg, dtype=np.float64))
    I = np.asarray(I, dtype=np.complex128).reshape(-1)
    Ft = np.zeros(th.shape, dtype=np.complex128)
    Fp = np.zeros(th.shape, dtype=np.complex128)
    for a in range(th.size):
        rh = np.array([np.sin(th[a]) * np.cos(ph[a]), np.sin(th[a]) * np.sin(ph[a]), np.cos(th[a])])
        et = np.array([np.cos(th[a]) * np.cos(ph[a]), np.cos(th[a]) * np.sin(ph[a]), -np.sin(th[a])])
        ep = np.array([-np.sin(ph[a]), np.cos(ph[a]), 0.0])
        phase = np.exp(1j * k * (centres @ rh))
        Ft[a] = -1j * k * eta * np.sum(I * (tangents @ et) * phase)
        Fp[a] = -1j * k * eta * np.sum(I * (tangents @ ep) * phase)
    return Ft, Fp


# ----------------------------------------------------------- paper bookkeeping
_COMPONENT_ORDER = (5, 2, 8, 6, 4, 3, 9, 1, 7)


def paper_parts(Nx: int, Ny: int):
    """Parts of an Nx x Ny array in the paper's numbering (Sec. II-C).

    Returns a list indexed by part number - 1 of (component, col, row), where the
    elements occupy cols 0..Nx-1 and rows 0..Ny-1, the left/right margin columns
    are cols -1 / Nx, the bottom/top margin rows are rows -1 / Ny.  Component
    placement follows the shared-side matrix of eq. (sharedTrianglesParttype):
    1 bottom-left, 2 left, 3 top-left, 4 bottom, 5 element, 6 top,
    7 bottom-right, 8 right, 9 top-right.  Within a component the part nearest
    the bottom-left comes first and x runs fastest.
    """
    cells = {
        5: [(c, r) for r in range(Ny) for c in range(Nx)],
        2: [(-1, r) for r in range(Ny)],
        8: [(Nx, r) for r in range(Ny)],
        6: [(c, Ny) for c in range(Nx)],
        4: [(c, -1) for c in range(Nx)],
        3: [(-1, Ny)],
        9: [(Nx, Ny)],
        1: [(-1, -1)],
        7: [(Nx, -1)],
    }
    parts = []
    for comp in _COMPONENT_ORDER:
        for (c, r) in cells[comp]:
            parts.append((comp, c, r))
    return parts


def part_count(Nx: int, Ny: int) -> int:
    """P_N of eq. (offsetMatrix)."""
    return Nx * Ny + 2 * Nx + 2 * Ny + 4


def memory_units(Nx: int, Ny: int, e) -> dict:
    """MEM_A, MEM_B, MEM_C of the Appendix (eqs. calcScalingA/B/C); e[1..9]."""
    e1, e2, e3, e4, e5, e6, e7, e8, e9 = (e[i] for i in range(1, 10))
    A = (2 * Nx * Ny - Nx - Ny + 1) * e5 ** 2
    B = ((2 * Nx * Ny - Nx) * e5 * (e2 + e8) + (2 * Nx * Ny - Ny) * e5 * (e6 + e4)
         + Nx * Ny * e5 * (e3 + e9 + e1 + e7))
    C = (Nx * Ny * (e2 + e8) * (e4 + e6) + Ny * (e2 ** 2 + e8 ** 2) + Nx * (e6 ** 2 + e4 ** 2)
         + (2 * Ny - 1) * e2 * e8 + (2 * Nx - 1) * e6 * e4
         + (Nx * (e6 + e4) + Ny * (e2 + e8)) * (e3 + e9 + e1 + e7) + e7 ** 2
         + e3 * (e3 + e9 + e1 + e7) + e9 * (e9 + e1 + e7) + e1 * (e1 + e7))
    return dict(A=A, B=B, C=C, total=A + B + C)


def memory_units_reduced(Nx: int, Ny: int, eE, em, ec):
    """The reduced closed form of Sec. II-C (eq. calcScalingApproxNew)."""
    return ((2 * Nx * Ny - Nx - Ny + 1) * eE ** 2 + (8 * Nx * Ny - 2 * Nx - 2 * Ny) * eE * em
            + 4 * Nx * Ny * eE * ec + (4 * Nx * Ny + 4 * Nx + 4 * Ny - 2) * em ** 2
            + 8 * (Nx + Ny) * em * ec + 10 * ec ** 2)
