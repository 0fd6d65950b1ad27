"""Seeded synthetic inputs for the algebraic-distance setup path.

This module builds the *inputs* of the path and nothing else: sparse operators
in CSR form, colourings and C/F splits.  It holds none of the method's own
arithmetic (no relaxation, no least squares, no thresholds), so the GPU path
and the CPU oracle may both be fed from it.

Operators follow the model problems of the paper's numerical section (Sec. 5.1):

* the rotated anisotropic diffusion operator  L u = a u_xx + b u_xy + c u_yy
  with a = cos^2(alpha) + eps sin^2(alpha), b = (1 - eps) sin(2 alpha),
  c = sin^2(alpha) + eps cos^2(alpha)  (Sec. 5.1, eq:scal);
* its seven-point form, whose mixed-derivative stencil uses only one diagonal
  pair (Sec. 5.1, eq. fd_seven);  the matrix is A = -h^2 L_h, which reproduces
  the printed stencil S_A for alpha = -pi/4, eps = 0.1 (diagonal 3.1);
* a nine-point form with the central mixed difference
  u_xy ~ (u_NE - u_NW - u_SE + u_SW) / (4 h^2);
* variable-coefficient 5-point (2D) and 7-point (3D) diffusion with
  log-normal face coefficients, and random-geometric-graph Laplacians with a
  diagonal shift (synthetic stand-ins for operators the paper does not fix).

Grid rows are numbered lexicographically: row = iy*N + ix in 2D and
row = (iz*N + iy)*N + ix in 3D.  Every CSR has sorted column indices and an
explicit diagonal entry.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# Seeds: test-vector seed 1106 + i and coefficient/graph seed 5990 + i for
# workload i = 1..5.
TV_SEED_BASE = 1106
COEF_SEED_BASE = 5990


@dataclasses.dataclass
class CSR:
    """A square sparse matrix in compressed-sparse-row form.

    row_ptr: int32[n+1], col: int32[nnz] (sorted per row, diagonal present),
    val: float32 or float64 [nnz].  `grid` records the structured-grid shape
    when the matrix comes from a stencil (None for graphs).
    """

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    grid: Optional[tuple] = None

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def n_edges(self) -> int:
        """Off-diagonal entries: the directed pairs (i, j), j != i."""
        return self.nnz - int(np.count_nonzero(self.col == self.row_ids()))

    def row_ids(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))

    def astype(self, dtype) -> "CSR":
        return CSR(self.n, self.row_ptr, self.col, self.val.astype(dtype), self.grid)

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n), dtype=np.float64)
        d[self.row_ids(), self.col] = self.val
        return d


# ---------------------------------------------------------------------------
# structured-grid stencils
# ---------------------------------------------------------------------------

def _stencil_2d(N: int, entries) -> CSR:
    """Assemble a constant-coefficient 2D stencil on an N x N interior grid
    with homogeneous Dirichlet boundary (out-of-grid neighbours dropped).

    entries: iterable of (dx, dy, value).  Zero values are dropped.
    """
    ents = sorted(((dy, dx, v) for dx, dy, v in entries if v != 0.0))
    n = N * N
    iy, ix = np.divmod(np.arange(n, dtype=np.int64), N)
    cols, vals, oks = [], [], []
    for dy, dx, v in ents:  # sorted by (dy, dx) == sorted by column offset
        jx, jy = ix + dx, iy + dy
        ok = (jx >= 0) & (jx < N) & (jy >= 0) & (jy < N)
        cols.append(jy * N + jx)
        vals.append(np.full(n, v))
        oks.append(ok)
    cols = np.stack(cols, 1)
    vals = np.stack(vals, 1)
    oks = np.stack(oks, 1)
    counts = oks.sum(1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(n, row_ptr.astype(np.int32), cols[oks].astype(np.int32),
               vals[oks].astype(np.float64), grid=(N, N))


def laplacian_2d_5pt(N: int) -> CSR:
    """Standard 5-point Laplacian, diagonal 4, off-diagonals -1."""
    return _stencil_2d(N, [(0, 0, 4.0), (1, 0, -1.0), (-1, 0, -1.0),
                           (0, 1, -1.0), (0, -1, -1.0)])


def anisotropy_coefficients(eps: float, alpha: float):
    """(a, b, c) of L u = a u_xx + b u_xy + c u_yy (Sec. 5.1, eq:scal)."""
    a = math.cos(alpha) ** 2 + eps * math.sin(alpha) ** 2
    b = (1.0 - eps) * math.sin(2.0 * alpha)
    c = math.sin(alpha) ** 2 + eps * math.cos(alpha) ** 2
    return a, b, c


def rotated_anisotropic_7pt(N: int, eps: float, alpha: float) -> CSR:
    """Seven-point discretisation of Sec. 5.1: the 5-point form of
    a u_xx + c u_yy plus b times the one-diagonal mixed stencil of eq.
    fd_seven, (1/(2h^2)) [[0,-1,1],[-1,2,-1],[1,-1,0]] (rows y+1, y, y-1;
    columns x-1, x, x+1).  The matrix is -h^2 times the difference operator.
    """
    a, b, c = anisotropy_coefficients(eps, alpha)
    e = {}

    def add(dx, dy, v):
        e[(dx, dy)] = e.get((dx, dy), 0.0) + v

    # -h^2 (a D_xx + c D_yy)
    add(0, 0, 2 * a + 2 * c)
    add(1, 0, -a); add(-1, 0, -a); add(0, 1, -c); add(0, -1, -c)
    # -h^2 * b * D~_xy, D~_xy = (1/2h^2)[[0,-1,1],[-1,2,-1],[1,-1,0]]
    s = -0.5 * b
    add(-1, 1, 0.0 * s); add(0, 1, -1.0 * s); add(1, 1, 1.0 * s)
    add(-1, 0, -1.0 * s); add(0, 0, 2.0 * s); add(1, 0, -1.0 * s)
    add(-1, -1, 1.0 * s); add(0, -1, -1.0 * s); add(1, -1, 0.0 * s)
    return _stencil_2d(N, [(dx, dy, v) for (dx, dy), v in e.items()])


def rotated_anisotropic_9pt(N: int, eps: float, alpha: float) -> CSR:
    """Nine-point discretisation: 5-point a u_xx + c u_yy plus the central
    mixed difference u_xy ~ (u_NE - u_NW - u_SE + u_SW)/(4 h^2); the matrix is
    -h^2 times the difference operator (same scaling as the 7-point form)."""
    a, b, c = anisotropy_coefficients(eps, alpha)
    q = -b / 4.0
    return _stencil_2d(N, [
        (0, 0, 2 * a + 2 * c),
        (1, 0, -a), (-1, 0, -a), (0, 1, -c), (0, -1, -c),
        (1, 1, q), (-1, -1, q), (-1, 1, -q), (1, -1, -q),
    ])


def lognormal_2d_5pt(N: int, sigma: float, seed) -> CSR:
    """Variable-coefficient 5-point diffusion on an N x N interior grid.

    Each cell face f carries kappa_f = exp(sigma * Z_f), Z_f ~ N(0,1) i.i.d.
    Off-diagonal a_ij = -kappa(face ij); a_ii = sum of the four faces of cell
    i, Dirichlet boundary faces included.  Draw order: x-faces [iy, fx]
    (N x (N+1)), then y-faces [fy, ix] ((N+1) x N).
    """
    rng = np.random.default_rng(seed)
    kx = np.exp(sigma * rng.standard_normal((N, N + 1)))
    ky = np.exp(sigma * rng.standard_normal((N + 1, N)))
    n = N * N
    iy, ix = np.divmod(np.arange(n, dtype=np.int64), N)
    # faces of cell (ix, iy): west kx[iy, ix], east kx[iy, ix+1],
    # south ky[iy, ix], north ky[iy+1, ix]
    west, east = kx[iy, ix], kx[iy, ix + 1]
    south, north = ky[iy, ix], ky[iy + 1, ix]
    diag = west + east + south + north
    nb = [(-N, -south, iy > 0), (-1, -west, ix > 0), (0, diag, np.ones(n, bool)),
          (1, -east, ix < N - 1), (N, -north, iy < N - 1)]
    return _assemble_offsets(n, nb, grid=(N, N))


def lognormal_3d_7pt(N: int, sigma: float, seed) -> CSR:
    """Variable-coefficient 7-point diffusion on an N^3 interior grid with
    log-normal face coefficients (as lognormal_2d_5pt, one more axis).
    Draw order: x-faces [iz, iy, fx], y-faces [iz, fy, ix], z-faces [fz, iy, ix].
    """
    rng = np.random.default_rng(seed)
    kx = np.exp(sigma * rng.standard_normal((N, N, N + 1)))
    ky = np.exp(sigma * rng.standard_normal((N, N + 1, N)))
    kz = np.exp(sigma * rng.standard_normal((N + 1, N, N)))
    n = N * N * N
    r = np.arange(n, dtype=np.int64)
    iz, rem = np.divmod(r, N * N)
    iy, ix = np.divmod(rem, N)
    w_, e_ = kx[iz, iy, ix], kx[iz, iy, ix + 1]
    s_, n_ = ky[iz, iy, ix], ky[iz, iy + 1, ix]
    d_, u_ = kz[iz, iy, ix], kz[iz + 1, iy, ix]
    diag = w_ + e_ + s_ + n_ + d_ + u_
    NN = N * N
    nb = [(-NN, -d_, iz > 0), (-N, -s_, iy > 0), (-1, -w_, ix > 0),
          (0, diag, np.ones(n, bool)),
          (1, -e_, ix < N - 1), (N, -n_, iy < N - 1), (NN, -u_, iz < N - 1)]
    return _assemble_offsets(n, nb, grid=(N, N, N))


def _assemble_offsets(n, nb, grid=None) -> CSR:
    """nb: list of (row offset, value array, validity mask), sorted by offset."""
    r = np.arange(n, dtype=np.int64)
    cols = np.stack([r + off for off, _, _ in nb], 1)
    vals = np.stack([np.broadcast_to(v, (n,)) for _, v, _ in nb], 1)
    oks = np.stack([m for _, _, m in nb], 1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(oks.sum(1), out=row_ptr[1:])
    return CSR(n, row_ptr.astype(np.int32), cols[oks].astype(np.int32),
               vals[oks].astype(np.float64), grid=grid)


# ---------------------------------------------------------------------------
# random geometric graph Laplacians
# ---------------------------------------------------------------------------

def rgg_laplacian(n: int, mean_degree: float, seed, shift: float = 1e-3,
                  wlo: float = 0.1, whi: float = 10.0) -> CSR:
    """Graph Laplacian of a random geometric graph plus a diagonal shift.

    Points are uniform in the unit square; i and j are joined when their
    distance is below r = sqrt(mean_degree / (n pi)).  Edge weights are
    uniform in [wlo, whi]; A = D - W + shift * I.  Rows are ordered by the
    row-major index of an r-sized cell, so neighbours are close in memory.
    """
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    r = math.sqrt(mean_degree / (n * math.pi))
    ncell = max(1, int(1.0 / r))
    cell = np.minimum((pts * ncell).astype(np.int64), ncell - 1)
    order = np.lexsort((pts[:, 0], cell[:, 0], cell[:, 1]))
    pts = pts[order]
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray").astype(np.int64)
    m = pairs.shape[0]
    w = wlo + (whi - wlo) * rng.random(m)
    i = np.concatenate([pairs[:, 0], pairs[:, 1], np.arange(n)])
    j = np.concatenate([pairs[:, 1], pairs[:, 0], np.arange(n)])
    deg = np.zeros(n)
    np.add.at(deg, pairs[:, 0], w)
    np.add.at(deg, pairs[:, 1], w)
    v = np.concatenate([-w, -w, deg + shift])
    key = i * n + j
    srt = np.argsort(key, kind="stable")
    i, j, v = i[srt], j[srt], v[srt]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(i, minlength=n), out=row_ptr[1:])
    return CSR(n, row_ptr.astype(np.int32), j.astype(np.int32), v)


def rgg_batch_sizes(nmat: int, seed, nmin=2_000, nmax=200_000, dmin=4.0, dmax=29.0):
    """Per-matrix (n, mean off-diagonal degree) for a batch: n log-uniform
    in [nmin, nmax], degree uniform in [dmin, dmax]."""
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), nmat))).astype(np.int64)
    ds = rng.uniform(dmin, dmax, nmat)
    return ns, ds


def _rgg_member(args):
    n, d, seed = args
    return rgg_laplacian(n, d, seed)


def rgg_batch(nmat: int, seed_base: int, nmin=2_000, nmax=200_000, workers: int = 1,
              progress=None) -> List[CSR]:
    """Matrix m uses seed (seed_base, m); `workers` > 1 builds members in
    parallel processes (same result).  Built in-process (workers <= 1),
    progress(k) is called after each member."""
    ns, ds = rgg_batch_sizes(nmat, seed_base, nmin, nmax)
    jobs = [(int(ns[m]), float(ds[m]), (seed_base, m)) for m in range(nmat)]
    if workers <= 1:
        out = []
        for j in jobs:
            out.append(_rgg_member(j))
            if progress:
                progress(len(out))
        return out
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_rgg_member, jobs, chunksize=1)


# ---------------------------------------------------------------------------
# colourings and C/F splits
# ---------------------------------------------------------------------------

def grid_parity(grid) -> np.ndarray:
    """(ix + iy [+ iz]) mod 2 for every grid point, row-major order."""
    idx = np.indices(grid[::-1]).reshape(len(grid), -1)  # (iz, iy, ix) order
    return (idx.sum(0) % 2).astype(np.int32)


def red_black(grid) -> np.ndarray:
    """Colour 0 ('red') where the index sum is even, 1 ('black') otherwise."""
    return grid_parity(grid)


def four_colour_2d(N: int) -> np.ndarray:
    """(ix mod 2) + 2 (iy mod 2): a valid colouring of any 9-point stencil."""
    iy, ix = np.divmod(np.arange(N * N), N)
    return ((ix % 2) + 2 * (iy % 2)).astype(np.int32)


def cf_red_is_coarse(grid) -> np.ndarray:
    """C/F split with C = red points: cf[i] = 1 for C, 0 for F."""
    return (grid_parity(grid) == 0).astype(np.uint8)


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    A: CSR
    K: int
    tv_seed: int
    relax: str            # "jacobi" | "gs"
    sweeps: int
    omega: float
    color: Optional[np.ndarray]
    ncolors: int
    cf: Optional[np.ndarray]
    theta: float = 0.25
    caliber: int = 4
    dtype: str = "f64"    # arithmetic type of the relax/distance steps


def workload(i: int, dtype: str = "f64", size: Optional[int] = None) -> Workload:
    """Workload i (1..5).  `size` overrides the grid side (for test-sized
    instances of the same structure); None gives the full size."""
    tv = TV_SEED_BASE + i
    cs = COEF_SEED_BASE + i
    if i == 1:
        N = size or 32
        A = laplacian_2d_5pt(N)
        return Workload("laplace2d-5pt-%d^2-K8" % N, A, 8, tv, "jacobi", 4, 2.0 / 3.0,
                        None, 0, cf_red_is_coarse((N, N)), 0.25, 4, dtype)
    if i == 2:
        N = size or 2048
        A = rotated_anisotropic_9pt(N, 1e-3, math.pi / 6)
        return Workload("aniso2d-9pt-%d^2-eps1e-3-alpha-pi/6-K16" % N, A, 16, tv, "gs", 5, 1.0,
                        red_black((N, N)), 2, cf_red_is_coarse((N, N)), 0.25, 4, dtype)
    if i == 3:
        N = size or 160
        A = lognormal_3d_7pt(N, 2.0, cs)
        A = A.astype(np.float32).astype(np.float64)  # the operator is stored in FP32
        return Workload("varcoef3d-7pt-%d^3-sigma2-K32" % N, A, 32, tv, "jacobi", 4, 0.8,
                        None, 0, cf_red_is_coarse((N, N, N)), 0.25, 4, dtype)
    if i == 5:
        N = size or 512
        A = lognormal_2d_5pt(N, 1.0, cs)
        return Workload("varcoef2d-5pt-%d^2-sigma1-K16" % N, A, 16, tv, "jacobi", 6, 2.0 / 3.0,
                        None, 0, cf_red_is_coarse((N, N)), 0.25, 4, "f64")
    raise ValueError("workload %d is a batch; use batch_workload()" % i)


def batch_workload(nmat: int = 512, nmin: int = 2_000, nmax: int = 200_000, workers: int = 1,
                   progress=None):
    """Workload 4: a batch of RGG Laplacians (n log-uniform in [nmin, nmax]),
    K = 16, 4 Jacobi sweeps with omega = 2/3, theta = 0.25."""
    return rgg_batch(nmat, COEF_SEED_BASE + 4, nmin, nmax, workers, progress)


BATCH_K, BATCH_SWEEPS, BATCH_OMEGA, BATCH_THETA = 16, 4, 2.0 / 3.0, 0.25


def concat_csr(mats: Sequence[CSR]) -> CSR:
    """Block-diagonal concatenation (column indices shifted per block)."""
    ns = [m.n for m in mats]
    roff = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    rp = [np.zeros(1, np.int64)]
    base = 0
    for m in mats:
        rp.append(m.row_ptr[1:].astype(np.int64) + base)
        base += m.nnz
    col = np.concatenate([m.col.astype(np.int64) + roff[k] for k, m in enumerate(mats)])
    val = np.concatenate([m.val for m in mats])
    return CSR(int(roff[-1]), np.concatenate(rp).astype(np.int32), col.astype(np.int32), val)
