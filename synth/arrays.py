"""Synthetic Green's-function-shaped array workloads (inputs only).

The paper fills its generator blocks with the EFIE/RWG impedance integral
(Sec. II, eq. MoMimpedanceMatrix) on meshed antenna elements.  No meshes ship
with it, so these workloads replace each basis function by a point dipole:

* wavelength 1, wavenumber k = 2*pi, element period d = 0.5;
* each element carries b basis functions at offsets u_p drawn uniformly in the
  0.5 x 0.5 cell (z = 0) with unit in-plane tangents t_p = (cos a, sin a, 0);
* Z_{m,n}[p, q] = exp(-j k r) / (4 pi r) * (t_p . t_q) between basis p of the
  element at (ix + m, iy + n) and basis q of the element at (ix, iy), with
  dx = m d + (u_p.x - u_q.x), dy = n d + (u_p.y - u_q.y), r = max(hypot, 0.01)
  (the clamp stands in for the singular self-term integration); the block at
  offset (0, 0) gets 10 + 5j added on its diagonal.  Evaluating the offsets in
  exactly this order makes Z_{-m,-n}[q, p] == Z_{m,n}[p, q] bit for bit, the
  reciprocity of Sec. II-A;
* Nr rim basis functions stand for the margin components of Sec. II-B: the
  array is an element plus eight margin components (four sides, four corners),
  each repeated by translation.  The margin is the band d/2 wide outside the
  cell hull.  Margin parts in the part order of eqs. submatrixB12/B34: side 1
  (left, Ny parts at cells (0, iy) shifted by -d/2 in x), side 2 (right, cells
  (Nx, iy)), side 3 (bottom, Nx parts at cells (ix, 0) shifted by -d/2 in y),
  side 4 (top, cells (ix, Ny)), then the four corners (bottom-left,
  bottom-right, top-left, top-right).  Each side part carries bm = Nr //
  (2 (Nx + Ny)) functions, the same offsets and tangents for every part of a
  side; the remainder goes to the corners (as evenly as possible, first corners
  first).  Every pair is evaluated as (cell difference) d + (local offset
  difference), so the side blocks of B and C are block Toeplitz bit for bit;
  the rim-rim diagonal gets 10 + 5j as well.

Global vector ordering (Sec. II-C, part ordering and eq. matrixForm): element
(ix, iy) is element number e = iy * Nx + ix (x fastest), basis p of element e is
unknown e * b + p, and rim function r is unknown N + r with N = Nx * Ny * b.

Generator layout: complex128 ``gen[n + Ny - 1, m + Nx - 1, p, q] = Z_{m,n}[p, q]``.
Rim layout: ``rim_re[r, e*b+p]`` (rim row, element column) and ``rim_rr[r, t]``;
the element-rim block is rim_re transposed (reciprocal).

All draws come from numpy's PCG64 seeded with SEED_BASE + config index, in the
order: basis offsets, basis angles, then per margin component (sides 1-4,
corners 1-4) its offsets and angles, then right-hand sides.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

SEED_BASE = 2506047100
WAVENUMBER = 2.0 * np.pi
PERIOD = 0.5
R_CLAMP = 0.01
DIAG_SHIFT = 10.0 + 5.0j

# name -> (Nx, Ny, b, Nr); the RHS recipe is chosen in make_config
CONFIGS = {
    1: dict(name="tiny-4x4-b16", Nx=4, Ny=4, b=16, Nr=24),
    2: dict(name="array-32x32-b64", Nx=32, Ny=32, b=64, Nr=256),
    3: dict(name="ports-9x9-b96", Nx=9, Ny=9, b=96, Nr=72),
    4: dict(name="scan-64x64-b48", Nx=64, Ny=64, b=48, Nr=0),
}


@dataclass
class Problem:
    Nx: int
    Ny: int
    b: int
    Nr: int
    gen: np.ndarray            # complex128 [2Ny-1, 2Nx-1, b, b]
    rim_re: np.ndarray         # complex128 [Nr, N]
    rim_rr: np.ndarray         # complex128 [Nr, Nr]
    centres: np.ndarray        # float64 [Nt, 3] basis positions (elements then rim)
    tangents: np.ndarray       # float64 [Nt, 3]
    k: float = WAVENUMBER
    d: float = PERIOD
    seed: int = 0
    rng: np.random.Generator | None = field(default=None, repr=False)

    @property
    def N(self) -> int:
        return self.Nx * self.Ny * self.b

    @property
    def Nt(self) -> int:
        return self.N + self.Nr


def _kernel(dx, dy, tdot, k):
    r = np.maximum(np.hypot(dx, dy), R_CLAMP)
    return np.exp(-1j * k * r) / (4.0 * np.pi * r) * tdot


def margin_counts(Nx: int, Ny: int, Nr: int):
    """Functions per side part (bm) and per corner (four counts) for Nr rim functions."""
    per = 2 * (Nx + Ny)
    bm = Nr // per
    rem = Nr - bm * per
    return bm, [rem // 4 + (1 if i < rem % 4 else 0) for i in range(4)]


def _margin_components(Nx, Ny, Nr, d):
    """(cells [(cx, cy)], local box origin, box size, functions per part) per
    margin component, in the rim's unknown order."""
    bm, bc = margin_counts(Nx, Ny, Nr)
    h = 0.5 * d
    return [
        ([(0, iy) for iy in range(Ny)], (-h, 0.0), (h, d), bm),        # side 1: left
        ([(Nx, iy) for iy in range(Ny)], (0.0, 0.0), (h, d), bm),      # side 2: right
        ([(ix, 0) for ix in range(Nx)], (0.0, -h), (d, h), bm),        # side 3: bottom
        ([(ix, Ny) for ix in range(Nx)], (0.0, 0.0), (d, h), bm),      # side 4: top
        ([(0, 0)], (-h, -h), (h, h), bc[0]),                           # corners
        ([(Nx, 0)], (0.0, -h), (h, h), bc[1]),
        ([(0, Ny)], (-h, 0.0), (h, h), bc[2]),
        ([(Nx, Ny)], (0.0, 0.0), (h, h), bc[3]),
    ]


def make_problem(Nx: int, Ny: int, b: int, Nr: int, seed: int | list) -> Problem:
    """Draw one array geometry and fill its generator and rim blocks."""
    if min(Nx, Ny, b) < 1 or Nr < 0:
        raise ValueError("Nx, Ny, b must be >= 1 and Nr >= 0")
    rng = np.random.default_rng(seed)
    d, k = PERIOD, WAVENUMBER
    u = rng.uniform(0.0, 0.5, size=(b, 2))          # basis offsets inside the cell
    alpha = rng.uniform(0.0, 2.0 * np.pi, size=b)    # basis tangent angles
    tx, ty = np.cos(alpha), np.sin(alpha)

    dux = u[:, 0][:, None] - u[:, 0][None, :]        # (u_p.x - u_q.x)
    duy = u[:, 1][:, None] - u[:, 1][None, :]
    tdot = tx[:, None] * tx[None, :] + ty[:, None] * ty[None, :]
    mvals = np.arange(-(Nx - 1), Nx)
    gen = np.empty((2 * Ny - 1, 2 * Nx - 1, b, b), dtype=np.complex128)
    for jn, n in enumerate(range(-(Ny - 1), Ny)):
        dx = (mvals * d)[:, None, None] + dux[None, :, :]
        dy = np.broadcast_to(n * d + duy, dx.shape)
        gen[jn] = _kernel(dx, dy, tdot[None], k)
    idx = np.arange(b)
    gen[Ny - 1, Nx - 1, idx, idx] += DIAG_SHIFT

    # absolute basis positions, element order x fastest then y, basis minor
    N = Nx * Ny * b
    iy, ix = np.divmod(np.arange(Nx * Ny), Nx)
    ex = (ix * d)[:, None] + u[None, :, 0]
    ey = (iy * d)[:, None] + u[None, :, 1]
    centres = np.zeros((N + Nr, 3))
    centres[:N, 0] = ex.reshape(-1)
    centres[:N, 1] = ey.reshape(-1)
    tangents = np.zeros((N + Nr, 3))
    tangents[:N, 0] = np.tile(tx, Nx * Ny)
    tangents[:N, 1] = np.tile(ty, Nx * Ny)

    # rim functions: integer cell, local offset and tangent per unknown
    rcell = np.zeros((Nr, 2))
    roff = np.zeros((Nr, 2))
    rtan = np.zeros((Nr, 2))
    r0 = 0
    for cells, org, size, nf in _margin_components(Nx, Ny, Nr, d):
        w = rng.uniform(0.0, 1.0, size=(nf, 2)) * np.asarray(size) + np.asarray(org)
        a = rng.uniform(0.0, 2.0 * np.pi, size=nf)
        for c in cells:
            rcell[r0:r0 + nf] = c
            roff[r0:r0 + nf] = w
            rtan[r0:r0 + nf, 0], rtan[r0:r0 + nf, 1] = np.cos(a), np.sin(a)
            r0 += nf
    assert r0 == Nr
    rim_re = np.zeros((Nr, N), dtype=np.complex128)
    rim_rr = np.zeros((Nr, Nr), dtype=np.complex128)
    if Nr:
        centres[N:, 0] = rcell[:, 0] * d + roff[:, 0]
        centres[N:, 1] = rcell[:, 1] * d + roff[:, 1]
        tangents[N:, 0], tangents[N:, 1] = rtan[:, 0], rtan[:, 1]
        ecx = np.repeat(ix, b).astype(float)
        ecy = np.repeat(iy, b).astype(float)
        eox, eoy = np.tile(u[:, 0], Nx * Ny), np.tile(u[:, 1], Nx * Ny)
        for r in range(Nr):
            dx = (rcell[r, 0] - ecx) * d + (roff[r, 0] - eox)
            dy = (rcell[r, 1] - ecy) * d + (roff[r, 1] - eoy)
            td = rtan[r, 0] * tangents[:N, 0] + rtan[r, 1] * tangents[:N, 1]
            rim_re[r] = _kernel(dx, dy, td, k)
        dx = (rcell[:, 0][:, None] - rcell[:, 0][None, :]) * d + (roff[:, 0][:, None] - roff[:, 0][None, :])
        dy = (rcell[:, 1][:, None] - rcell[:, 1][None, :]) * d + (roff[:, 1][:, None] - roff[:, 1][None, :])
        td = rtan[:, 0][:, None] * rtan[:, 0][None, :] + rtan[:, 1][:, None] * rtan[:, 1][None, :]
        rim_rr[:] = _kernel(dx, dy, td, k)
        rim_rr[np.arange(Nr), np.arange(Nr)] += DIAG_SHIFT
    return Problem(Nx, Ny, b, Nr, gen, rim_re, rim_rr, centres, tangents,
                   k=k, d=d, seed=seed if isinstance(seed, int) else -1, rng=rng)


# ---------------------------------------------------------------- right-hand sides
# Vectors are numpy arrays of shape (R, Nt): row r is column r of the
# column-major Nt x R block handed to the library.

def rhs_random(prob: Problem, R: int = 1, rng=None) -> np.ndarray:
    """Complex normal columns scaled to unit 2-norm."""
    rng = prob.rng if rng is None else rng
    v = rng.standard_normal((R, prob.Nt)) + 1j * rng.standard_normal((R, prob.Nt))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def rhs_plane_wave(prob: Problem, thetas_deg, phis_deg) -> np.ndarray:
    """x_i = exp(-j k khat . c_i) over every basis centre (elements and rim)."""
    th = np.deg2rad(np.atleast_1d(np.asarray(thetas_deg, dtype=np.float64)))
    ph = np.deg2rad(np.atleast_1d(np.asarray(phis_deg, dtype=np.float64)))
    kh = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    return np.exp(-1j * prob.k * (kh @ prob.centres.T))


def rhs_ports(prob: Problem, elements, feed: int = 0) -> np.ndarray:
    """Unit vectors at each listed element's feed basis; rim entries are zero."""
    elements = np.asarray(elements, dtype=np.int64)
    V = np.zeros((len(elements), prob.Nt), dtype=np.complex128)
    V[np.arange(len(elements)), elements * prob.b + feed] = 1.0
    return V


def make_config(idx: int, reduced: dict | None = None):
    """Problem and RHS block for one of the fixed workloads.

    ``reduced`` overrides (Nx, Ny, b, Nr) to build a smaller array with the same
    recipe (used for oracle-sized parity cases).
    """
    cfg = dict(CONFIGS[idx])
    if reduced:
        cfg.update(reduced)
    prob = make_problem(cfg["Nx"], cfg["Ny"], cfg["b"], cfg["Nr"], SEED_BASE + idx)
    if idx == 1:
        V = rhs_random(prob, 1)
    elif idx == 2:
        V = rhs_plane_wave(prob, [0.0], [0.0])
    elif idx == 3:
        V = rhs_ports(prob, np.arange(prob.Nx * prob.Ny))
    elif idx == 4:
        th = prob.rng.uniform(0.0, 60.0, size=8)
        V = rhs_plane_wave(prob, th, np.zeros(8))
    else:
        raise KeyError(idx)
    return prob, V


SERVE_SIZES = (8, 16, 24, 32, 48)
SERVE_B = (32, 64)


def serving_stream(n_requests: int = 512, rate_hz: float = 100.0, seed: int = SEED_BASE + 5,
                   sizes=SERVE_SIZES, bs=SERVE_B, max_rhs: int = 16):
    """Seeded Poisson request stream: arrival time, geometry key, port elements."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n_requests))
    reqs = []
    for i in range(n_requests):
        Nx = int(rng.choice(sizes))
        Ny = int(rng.choice(sizes))
        b = int(rng.choice(bs))
        R = int(rng.integers(1, max_rhs + 1))
        elems = np.sort(rng.choice(Nx * Ny, size=R, replace=False))
        reqs.append(dict(id=i, t=float(t[i]), Nx=Nx, Ny=Ny, b=b, R=R, elements=elems))
    return reqs


def serving_geometry(Nx: int, Ny: int, b: int, Nr: int = 0, seed: int = SEED_BASE + 5) -> Problem:
    """One cached geometry of the serving mix (seed derived from its key)."""
    return make_problem(Nx, Ny, b, Nr, [seed, Nx, Ny, b, Nr])


def rim_placement(prob: Problem):
    """Where each rim function sits as a channel of an element cell, for a
    plan that takes the rim in its one-level block-Toeplitz form: an int32
    array [Nr, 3] of (cell x, cell y, channel) and the channel count nrc.

    Every part of a margin component is a translate of the component's first
    part, so a component can be pinned to any column (row) of cells as long
    as all its parts move together: side 2 (cells (Nx, iy)) is placed at
    column Nx - 1, side 4 at row Ny - 1, the corners at the corner cells.
    Side s takes channels [s bm, (s + 1) bm); each corner its own channels
    after the sides'.  (This is metadata of the margin decomposition, not an
    evaluation of any coupling.)"""
    Nx, Ny, Nr = prob.Nx, prob.Ny, prob.Nr
    bm, bc = margin_counts(Nx, Ny, Nr)
    comps = _margin_components(Nx, Ny, Nr, prob.d)
    place = np.zeros((Nr, 3), dtype=np.int32)
    r0 = 0
    ch0 = 0
    for cells, _org, _size, nf in comps:
        for (cx, cy) in cells:
            for j in range(nf):
                place[r0] = (min(cx, Nx - 1), min(cy, Ny - 1), ch0 + j)
                r0 += 1
        ch0 += nf
    assert r0 == Nr
    return place, ch0
