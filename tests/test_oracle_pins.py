"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests retypes an oracle formula: each one checks the oracle
against an independent route (a closed form, a library routine solving the
same problem another way, brute force, an invariant, or a value printed in
the paper) chosen so that a dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from paper_1106_5990_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _csr_from_dense(D):
    D = np.asarray(D, dtype=np.float64)
    n = D.shape[0]
    mask = D != 0
    mask[np.arange(n), np.arange(n)] = True
    rows, cols = np.nonzero(mask)
    rp = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    return W.CSR(n, rp, cols.astype(np.int32), D[rows, cols])


def _scipy(A):
    return sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))


# ---------------------------------------------------------------- generator
def test_splitmix64_matches_published_outputs():
    want = [int(r[0]) for r in _golden_rows("splitmix64_seed1234567.txt")]
    got = [oracle.splitmix64_nth(1234567, k) for k in range(1, 6)]
    assert got == want


def test_tv_init_is_the_counter_stream_and_uniform():
    seed = 99
    X = oracle.tv_init(5, 3, seed)
    # entry (r, k) is output r*K + k + 1 of the generator, top 53 bits
    for r in range(5):
        for k in range(3):
            z = oracle.splitmix64_nth(seed, r * 3 + k + 1)
            assert X[r, k] == 2.0 * ((z >> 11) * 2.0 ** -53) - 1.0
    # offsets: rows 7..9 of a larger start are the row0=7 block
    big = oracle.tv_init(10, 4, 5)
    assert np.array_equal(big[7:], oracle.tv_init(3, 4, 5, row0=7))
    Y = oracle.tv_init(20000, 8, 1)
    assert Y.min() >= -1.0 and Y.max() < 1.0
    assert abs(Y.mean()) < 0.01 and abs(Y.var() - 1.0 / 3.0) < 0.01


# ---------------------------------------------------------------- operators
def test_seven_point_stencil_reproduces_printed_S_A():
    """Sec. 5.1: alpha = -pi/4, eps = 0.1 gives the stencil S_A."""
    want = np.array([[float(v) for v in r] for r in _golden_rows("stencil_SA.txt")])
    N = 5
    A = W.rotated_anisotropic_7pt(N, 0.1, -math.pi / 4)
    D = A.to_dense()
    c = 2 * N + 2  # interior point (2, 2)
    got = np.zeros((3, 3))
    for r, dy in enumerate((1, 0, -1)):
        for q, dx in enumerate((-1, 0, 1)):
            got[r, q] = D[c, c + dy * N + dx]
    assert np.allclose(got, want, atol=1e-14, rtol=0)
    assert A.row_ptr[c + 1] - A.row_ptr[c] == 7  # "seven nonzero values"


@pytest.mark.parametrize("maker", [W.rotated_anisotropic_9pt, W.rotated_anisotropic_7pt])
@pytest.mark.parametrize("alpha", [math.pi / 6, -math.pi / 4, math.pi / 8, 0.3])
def test_stencils_exact_on_quadratics(maker, alpha):
    """A = -h^2 L_h with L = a u_xx + b u_xy + c u_yy (eq:scal): on unit grid
    coordinates the difference operator is exact for x^2, y^2 and xy."""
    eps = 1e-3
    N = 9
    a, b, c = W.anisotropy_coefficients(eps, alpha)
    A = _scipy(maker(N, eps, alpha))
    iy, ix = np.divmod(np.arange(N * N), N)
    inner = (ix > 0) & (ix < N - 1) & (iy > 0) & (iy < N - 1)
    for u, want in [(ix ** 2, -2 * a), (iy ** 2, -2 * c), (ix * iy, -b)]:
        got = (A @ u.astype(float))[inner]
        assert np.allclose(got, want, atol=1e-12)


@pytest.mark.parametrize("alpha", [0.0, math.pi / 6, -math.pi / 4, 1.0])
def test_anisotropy_coefficients_are_a_rotation(alpha):
    """K = R diag(1, eps) R^T (eq:a): trace a + c = 1 + eps and
    4ac - b^2 = 4 eps (b is twice the off-diagonal of K)."""
    eps = 0.05
    a, b, c = W.anisotropy_coefficients(eps, alpha)
    assert abs(a + c - (1 + eps)) < 1e-15
    assert abs(4 * a * c - b * b - 4 * eps) < 1e-14
    R = np.array([[math.cos(alpha), -math.sin(alpha)], [math.sin(alpha), math.cos(alpha)]])
    K = R @ np.diag([1, eps]) @ R.T
    assert np.allclose([K[0, 0], 2 * K[0, 1], K[1, 1]], [a, b, c], atol=1e-15)


def test_workload_shapes():
    w1 = W.workload(1)
    assert (w1.A.n, w1.A.nnz) == (1024, 4992)
    A = W.rotated_anisotropic_9pt(16, 1e-3, math.pi / 6)
    assert A.nnz == 9 * 256 - 3 * 4 * 16 + 4  # 9 per row minus boundary losses
    A3 = W.lognormal_3d_7pt(6, 2.0, 1)
    assert A3.nnz == 7 * 216 - 6 * 36
    for A in (w1.A, A, A3, W.lognormal_2d_5pt(7, 1.0, 3), W.rgg_laplacian(300, 8.0, 4)):
        D = A.to_dense()
        assert np.allclose(D, D.T, rtol=0, atol=0)
        np.linalg.cholesky(D)  # SPD
        for i in range(A.n):  # sorted columns, explicit diagonal
            cols = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
            assert np.all(np.diff(cols) > 0) and i in cols


def test_rgg_laplacian_structure():
    A = W.rgg_laplacian(500, 10.0, 7)
    D = A.to_dense()
    off = D - np.diag(np.diag(D))
    assert np.all(off <= 0)
    w = -off[off < 0]
    assert w.min() >= 0.1 and w.max() <= 10.0
    assert np.allclose(np.diag(D), -off.sum(1) + 1e-3, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- relaxation
@pytest.mark.parametrize("k,l", [(1, 1), (3, 5), (7, 2)])
def test_jacobi_damps_fourier_modes_by_closed_form(k, l):
    """Damped Jacobi on the 5-point Dirichlet Laplacian multiplies the mode
    sin(k pi x) sin(l pi y) by 1 - omega (1 - (cos k pi h + cos l pi h)/2)."""
    N, omega, sweeps = 15, 2.0 / 3.0, 3
    h = 1.0 / (N + 1)
    A = W.laplacian_2d_5pt(N)
    iy, ix = np.divmod(np.arange(N * N), N)
    v = np.sin(k * math.pi * (ix + 1) * h) * np.sin(l * math.pi * (iy + 1) * h)
    X0 = np.stack([v, 2 * v], 1)
    X, _ = oracle.jacobi(A, X0, omega, sweeps)
    g = 1 - omega * (1 - (math.cos(k * math.pi * h) + math.cos(l * math.pi * h)) / 2)
    assert np.allclose(X, X0 * g ** sweeps, atol=1e-14, rtol=0)


def _sequential_gs(A, x, order):
    """Textbook Gauss-Seidel sweep for A x = 0 in the given row order:
    with P A P^T = L + U (L lower incl. diagonal), x_new = -L^{-1} U x_old."""
    S = _scipy(A)[order][:, order]
    L = sp.tril(S, 0, format="csr")
    U = sp.triu(S, 1, format="csr")
    y = x[order]
    xn = spla.spsolve_triangular(L, -(U @ y), lower=True)
    out = np.empty_like(x)
    out[order] = xn
    return out


@pytest.mark.parametrize("case", ["rb-5pt", "four-colour-9pt"])
def test_colour_gs_equals_sequential_gs_for_valid_colourings(case):
    N = 12
    if case == "rb-5pt":
        A = W.laplacian_2d_5pt(N)
        color, nc = W.red_black((N, N)), 2
    else:
        A = W.rotated_anisotropic_9pt(N, 1e-2, math.pi / 6)
        color, nc = W.four_colour_2d(N), 4
    X0 = oracle.tv_init(A.n, 3, 17)
    X, held = oracle.color_gs(A, X0, color, nc, 2)
    assert held == 0
    order = np.argsort(color, kind="stable")
    want = X0.copy()
    for _ in range(2):
        want = _sequential_gs(A, want, order)
    assert np.allclose(X, want, atol=1e-13, rtol=0)


def test_single_colour_gs_is_undamped_jacobi():
    A = W.rotated_anisotropic_9pt(10, 1e-3, math.pi / 6)
    X0 = oracle.tv_init(A.n, 4, 3)
    Xg, _ = oracle.color_gs(A, X0, np.zeros(A.n, np.int32), 1, 3)
    Xj, _ = oracle.jacobi(A, X0, 1.0, 3)
    assert np.allclose(Xg, Xj, atol=1e-14, rtol=0)


def test_colour_gs_rows_matches_full_sweep():
    N = 10
    A = W.rotated_anisotropic_9pt(N, 1e-3, math.pi / 6)
    color = W.red_black((N, N))
    X0 = oracle.tv_init(A.n, 4, 8)
    X1, _ = oracle.color_gs(A, X0, color, 2, 1)
    rows = np.array([0, 5, 13, 57, 99])
    assert np.array_equal(oracle.color_gs_rows(A, color, 2, X0, X1, rows), X1[rows])
    Xj, _ = oracle.jacobi(A, X0, 0.7, 1)
    assert np.array_equal(oracle.jacobi_rows(A, X0, 0.7, rows), Xj[rows])


def test_zero_diagonal_and_bad_colour_rows_are_held():
    A = W.laplacian_2d_5pt(4)
    A.val = A.val.copy()
    i = 5
    A.val[A.row_ptr[i]:A.row_ptr[i + 1]][A.col[A.row_ptr[i]:A.row_ptr[i + 1]] == i] = 0.0
    X0 = oracle.tv_init(16, 2, 1)
    X, z = oracle.jacobi(A, X0, 0.5, 2)
    assert z == 1 and np.array_equal(X[i], X0[i])
    color = W.red_black((4, 4)).copy()
    color[3] = 7
    X, held = oracle.color_gs(A, X0, color, 2, 2)
    assert held == 2 and np.array_equal(X[i], X0[i]) and np.array_equal(X[3], X0[3])


# ---------------------------------------------------------------- algebraic distance
def test_algdist_hand_example():
    g = {r[0]: [float(v) for v in r[1:]] for r in _golden_rows("algdist_hand_example.txt")}
    A = _csr_from_dense([[2.0, -1.0], [-1.0, 2.0]])
    X = np.array([g["x_i"], g["x_j"]])
    mu, p, _ = oracle.algdist(A, X, want_p=True)
    # row 0 entries: (0,0), (0,1)
    assert p[1] == g["p"][0] and mu[1] == g["mu"][0]


def _random_case(n=9, K=5, seed=0, density=0.4):
    rng = np.random.default_rng(seed)
    D = np.where(rng.random((n, n)) < density, rng.standard_normal((n, n)), 0.0)
    D = D + D.T + np.diag(4.0 + rng.random(n))
    return _csr_from_dense(D), rng.standard_normal((n, K)), 0.5 + rng.random(K)


@pytest.mark.parametrize("target", [oracle.TARGET_PLAIN, oracle.TARGET_RESIDUAL])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_algdist_matches_lstsq(target, seed):
    A, X, w = _random_case(seed=seed)
    mu, p, _ = oracle.algdist(A, X, w, target, want_p=True)
    D = A.to_dense()
    sw = np.sqrt(w)
    e = 0
    for i in range(A.n):
        t = X[i] if target == oracle.TARGET_PLAIN else X[i] - (D[i] @ X) / D[i, i]
        for j in A.col[A.row_ptr[i]:A.row_ptr[i + 1]]:
            sol, res, rank, _ = np.linalg.lstsq((sw * X[j])[:, None], sw * t, rcond=None)
            want = float(np.sum((sw * t - sol[0] * sw * X[j]) ** 2))
            assert abs(p[e] - sol[0]) <= 1e-12 * max(1, abs(sol[0]))
            assert abs(mu[e] - want) <= 1e-12 * max(want, 1e-300) + 1e-15 * np.sum(w * t * t)
            e += 1


def test_residual_target_is_a_local_jacobi_step():
    """Sec. 3.1 eq:modls with r = A v: v_i - r_i/a_ii = -sum_{j!=i} a_ij v_j / a_ii,
    so the residual-target distance equals the plain distance of the
    Jacobi-updated (omega = 1) value at i."""
    A, X, w = _random_case(seed=4)
    D = A.to_dense()
    mu_r = oracle.algdist(A, X, w, oracle.TARGET_RESIDUAL)
    off = D - np.diag(np.diag(D))
    T = -(off @ X) / np.diag(D)[:, None]
    e = 0
    for i in range(A.n):
        for j in A.col[A.row_ptr[i]:A.row_ptr[i + 1]]:
            xj = X[j]
            p = np.sum(w * T[i] * xj) / np.sum(w * xj * xj)
            want = np.sum(w * (T[i] - p * xj) ** 2)
            assert abs(mu_r[e] - want) <= 1e-11 * want + 1e-14
            e += 1


def test_algdist_brute_force_minimum():
    rng = np.random.default_rng(5)
    for _ in range(20):
        K = int(rng.integers(1, 5))
        X = rng.standard_normal((2, K))
        w = 0.1 + rng.random(K)
        A = _csr_from_dense([[1.0, 0.5], [0.5, 1.0]])
        mu = oracle.algdist(A, X, w)[1]
        f = lambda q: float(np.sum(w * (X[0] - q * X[1]) ** 2))
        grid = np.linspace(-20, 20, 40001)
        vals = np.array([f(q) for q in grid])
        q0 = grid[np.argmin(vals)]
        lo, hi = q0 - 1e-3, q0 + 1e-3
        g = (math.sqrt(5) - 1) / 2
        for _ in range(80):
            a1, b1 = hi - g * (hi - lo), lo + g * (hi - lo)
            if f(a1) < f(b1):
                hi = b1
            else:
                lo = a1
        best = f(0.5 * (lo + hi))
        assert mu >= 0 and mu <= best * (1 + 1e-9) + 1e-15 and best - mu <= 1e-9 * max(best, 1e-12)


def test_algdist_zero_for_power_of_two_multiples_and_diagonal():
    rng = np.random.default_rng(6)
    X = rng.standard_normal((3, 8))
    X[1] = 4.0 * X[0]
    X[2] = -0.125 * X[0]
    A = _csr_from_dense(np.ones((3, 3)) + 3 * np.eye(3))
    mu = oracle.algdist(A, X, 0.3 + rng.random(8)).reshape(3, 3)
    assert np.all(mu == 0.0)
    Y = rng.standard_normal((3, 8))
    Y[1] = 3.7 * Y[0]
    mu = oracle.algdist(A, Y).reshape(3, 3)
    assert mu[0, 1] <= 1e-28 * np.sum(Y[0] ** 2) and np.all(np.diag(mu) == 0.0)


def test_algdist_scaling_and_nonnegativity():
    A, X, w = _random_case(seed=7)
    mu = oracle.algdist(A, X, w)
    assert np.all(mu >= 0)
    mu2 = oracle.algdist(A, 4.0 * X, w)
    assert np.array_equal(mu2, 16.0 * mu)
    mu3 = oracle.algdist(A, X, 8.0 * w)
    assert np.array_equal(mu3, 8.0 * mu)


def test_algdist_zero_column_gives_p_zero():
    A = _csr_from_dense([[2.0, -1.0], [-1.0, 2.0]])
    X = np.array([[1.0, -2.0, 3.0], [0.0, 0.0, 0.0]])
    mu, p, _ = oracle.algdist(A, X, want_p=True)
    assert p[1] == 0.0 and mu[1] == 14.0


# ---------------------------------------------------------------- strength graph
def _strength_case(seed=0):
    N = 12
    A = W.rotated_anisotropic_9pt(N, 1e-3, math.pi / 6)
    X, _ = oracle.color_gs(A, oracle.tv_init(A.n, 8, seed), W.red_black((N, N)), 2, 3)
    return A, X


def test_strength_every_row_keeps_its_strongest_edge():
    A, X = _strength_case()
    mu = oracle.algdist(A, X)
    strong, ns = oracle.strength(A, mu, 0.25)
    rid = A.row_ids()
    for i in range(A.n):
        s, e = A.row_ptr[i], A.row_ptr[i + 1]
        off = A.col[s:e] != i
        m = mu[s:e][off]
        assert ns[i] >= 1 and ns[i] == strong[s:e].sum()
        assert strong[s:e][off][np.argmin(m)] == 1
        assert np.all(strong[s:e][~off] == 0)
    # brute force of eq:strength_graph with r = 1/mu
    r = 1.0 / mu
    for e_ in range(len(mu)):
        i = rid[e_]
        s, e = A.row_ptr[i], A.row_ptr[i + 1]
        if A.col[e_] == i:
            continue
        rmax = max(r[k] for k in range(s, e) if A.col[k] != i)
        assert strong[e_] == (r[e_] > 0.25 * rmax)


def test_strength_zero_distance_edges_are_the_strong_ones():
    mu = np.array([0.0, 0.0, 3.0, 0.0, 1.0])  # row 0: diag, j1 mu=0, j2, j3 mu=0, j4
    A = _csr_from_dense(np.ones((5, 5)) + 4 * np.eye(5))
    mu_full = np.ones(25)
    mu_full[:5] = mu
    strong, ns = oracle.strength(A, mu_full, 0.5)
    assert list(strong[:5]) == [0, 1, 0, 1, 0] and ns[0] == 2


def test_strength_inequality_is_strict():
    """eq:strength_graph keeps r_ij > theta max_k r_ik strictly: an edge whose
    strength is exactly theta times the row maximum is weak."""
    A = _csr_from_dense(np.ones((3, 3)) + 2 * np.eye(3))
    mu = np.ones(9)
    mu[0:3] = [0.0, 2.0, 1.0]  # row 0: r = 1/2 and 1; theta * max = 1/2
    strong, ns = oracle.strength(A, mu, 0.5)
    assert list(strong[:3]) == [0, 0, 1] and ns[0] == 1


def test_strength_invariances():
    A, X = _strength_case(1)
    base = oracle.strength(A, oracle.algdist(A, X), 0.25)[0]
    # global scaling of x or w
    assert np.array_equal(base, oracle.strength(A, oracle.algdist(A, 2.0 * X), 0.25)[0])
    assert np.array_equal(base, oracle.strength(A, oracle.algdist(A, X, np.full(8, 3.0)), 0.25)[0])
    # A -> D A D with x0 -> D^-1 x0 for Jacobi (power-of-two D: exact)
    N = 10
    A = W.rotated_anisotropic_9pt(N, 1e-3, math.pi / 6)
    X0 = oracle.tv_init(A.n, 8, 2)
    d = 2.0 ** np.random.default_rng(0).integers(-3, 4, A.n)
    B = W.CSR(A.n, A.row_ptr, A.col, A.val * d[A.row_ids()] * d[A.col])
    Xa, _ = oracle.jacobi(A, X0, 0.7, 3)
    Xb, _ = oracle.jacobi(B, X0 / d[:, None], 0.7, 3)
    sa = oracle.strength(A, oracle.algdist(A, Xa), 0.25)[0]
    sb = oracle.strength(B, oracle.algdist(B, Xb), 0.25)[0]
    assert np.array_equal(sa, sb)


def test_strength_permutation_equivariance():
    A, X = _strength_case(2)
    n = A.n
    perm = np.random.default_rng(3).permutation(n)  # new index of old row i is inv
    inv = np.argsort(perm)
    D = A.to_dense()[perm][:, perm]
    B = _csr_from_dense(D)
    mu_a = oracle.algdist(A, X)
    mu_b = oracle.algdist(B, X[perm])
    sa, _ = oracle.strength(A, mu_a, 0.25)
    sb, _ = oracle.strength(B, mu_b, 0.25)
    Sa = sp.csr_matrix((sa.astype(float) + 1, A.col, A.row_ptr), shape=(n, n)).toarray()
    Sb = sp.csr_matrix((sb.astype(float) + 1, B.col, B.row_ptr), shape=(n, n)).toarray()
    assert np.array_equal(Sa[perm][:, perm], Sb)


def test_strength_fmask_restricts_to_F():
    A, X = _strength_case(4)
    mu = oracle.algdist(A, X)
    f = (np.arange(A.n) % 3 != 0).astype(np.uint8)
    strong, ns = oracle.strength(A, mu, 0.25, f)
    rid = A.row_ids()
    assert np.all(strong[(f[rid] == 0) | (f[A.col] == 0)] == 0)
    assert np.all(ns[f == 0] == 0)


@pytest.mark.parametrize("sign", [1, -1])
def test_strength_follows_the_anisotropy(sign):
    """Sec. 5.1: strong connections align with the direction xi.  With the
    paper's test-vector protocol (40 Gauss-Seidel sweeps, Sec. 5.2) on the
    rotated operator (alpha = +-pi/6, eps = 1e-3), the median distance of the
    eight neighbour directions is ordered by |eta . delta| (eta = (-sin a,
    cos a)): the xi-aligned diagonal first, the opposite diagonal last."""
    N = 48
    alpha = sign * math.pi / 6
    A = W.rotated_anisotropic_9pt(N, 1e-3, alpha)
    X, _ = oracle.color_gs(A, oracle.tv_init(A.n, 8, 11), W.red_black((N, N)), 2, 40)
    mu = oracle.algdist(A, X)
    strong, _ = oracle.strength(A, mu, 0.25)
    rid = A.row_ids()
    off = A.col.astype(np.int64) - rid
    iy, ix = np.divmod(np.arange(A.n), N)
    inner = ((ix > 1) & (ix < N - 2) & (iy > 1) & (iy < N - 2))[rid]
    diag_a, diag_b = (N + 1, N - 1) if sign > 0 else (N - 1, N + 1)  # aligned / opposite
    med = {o: np.median(mu[inner & (np.abs(off) == o)]) for o in (1, N, diag_a, diag_b)}
    eta = np.array([-math.sin(alpha), math.cos(alpha)])
    proj = {1: abs(eta[0]), N: abs(eta[1]),
            diag_a: abs(eta @ ([1, 1] if sign > 0 else [-1, 1])),
            diag_b: abs(eta @ ([-1, 1] if sign > 0 else [1, 1]))}
    assert sorted(med, key=med.get) == sorted(proj, key=proj.get)
    # the opposite diagonal is almost never strong
    frac = strong[inner & (np.abs(off) == diag_b)].mean()
    assert frac < 0.02


# ---------------------------------------------------------------- LS interpolation
def _ls_case(seed, K=6, n=14):
    rng = np.random.default_rng(seed)
    D = np.where(rng.random((n, n)) < 0.5, -rng.random((n, n)), 0.0)
    D = D + D.T + np.diag(8.0 + rng.random(n))
    A = _csr_from_dense(D)
    X = rng.standard_normal((n, K))
    w = 0.5 + rng.random(K)
    cf = (rng.random(n) < 0.5).astype(np.uint8)
    mu = oracle.algdist(A, X, w)
    return A, X, w, cf, mu


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("target", [oracle.TARGET_PLAIN, oracle.TARGET_RESIDUAL])
def test_ls_interp_matches_lstsq_on_selected_set(seed, target):
    A, X, w, cf, mu = _ls_case(seed)
    cal = 3
    Pc, Pv, ls, st = oracle.ls_interp(A, X, w, cf, mu, cal, target)
    D = A.to_dense()
    sw = np.sqrt(w)
    for i in range(A.n):
        if cf[i]:
            assert Pc[i, 0] == i and Pv[i, 0] == 1.0 and ls[i] == 0 and st[i] == 0
            continue
        s, e = A.row_ptr[i], A.row_ptr[i + 1]
        cand = [(mu[k], A.col[k]) for k in range(s, e) if A.col[k] != i and cf[A.col[k]]]
        sel = [c for _, c in sorted(cand)[:cal]]
        t = X[i] if target == oracle.TARGET_PLAIN else X[i] - D[i] @ X / D[i, i]
        if not sel:
            assert st[i] == 1 and np.all(Pc[i] == -1) and abs(ls[i] - np.sum(w * t * t)) <= 1e-12 * ls[i]
            continue
        M = (sw[:, None] * X[sel].T)
        sol = np.linalg.lstsq(M, sw * t, rcond=None)[0]
        want = np.sum((sw * t - M @ sol) ** 2)
        assert list(Pc[i, :len(sel)]) == sel and st[i] == 0
        assert np.allclose(Pv[i, :len(sel)], sol, atol=1e-11, rtol=1e-11)
        assert abs(ls[i] - want) <= 1e-10 * want + 1e-13


def test_ls_interp_exact_recovery_and_duplicate_drop():
    rng = np.random.default_rng(9)
    K = 6
    # row 0 is F with C-neighbours 1..4
    D = -np.ones((5, 5)) + 10 * np.eye(5)
    A = _csr_from_dense(D)
    X = rng.standard_normal((5, K))
    q = np.array([0.5, -1.25, 2.0])
    X[0] = q @ X[1:4]
    cf = np.array([0, 1, 1, 1, 0], np.uint8)
    mu = np.zeros(A.nnz)
    mu[1:4] = [0.1, 0.2, 0.3]
    Pc, Pv, ls, st = oracle.ls_interp(A, X, None, cf, mu, 3)
    assert list(Pc[0]) == [1, 2, 3] and np.allclose(Pv[0], q, atol=1e-12) and ls[0] < 1e-24
    # duplicate column: neighbour 3 equals neighbour 1 -> dropped, status 2
    X[3] = X[1]
    X[0] = 0.75 * X[1] + 0.5 * X[2]
    Pc, Pv, ls, st = oracle.ls_interp(A, X, None, cf, mu, 3)
    assert st[0] == 2 and list(Pc[0]) == [1, 2, -1]
    assert np.allclose(Pv[0, :2], [0.75, 0.5], atol=1e-12) and ls[0] < 1e-24


def test_ls_interp_monotone_in_the_set():
    """Sec. 4.3: W' subset of W'' implies LS_W' >= LS_W''.  The selected sets
    for caliber c are nested in c (same mu order)."""
    A, X, w, cf, mu = _ls_case(11, K=8, n=20)
    prev = None
    for cal in range(1, 6):
        ls = oracle.ls_interp(A, X, w, cf, mu, cal)[2]
        if prev is not None:
            assert np.all(ls <= prev * (1 + 1e-12) + 1e-15)
        prev = ls


def test_ls_interp_two_column_brute_force():
    rng = np.random.default_rng(12)
    for _ in range(10):
        K = 4
        X = rng.standard_normal((3, K))
        w = 0.2 + rng.random(K)
        A = _csr_from_dense(-np.ones((3, 3)) + 5 * np.eye(3))
        cf = np.array([0, 1, 1], np.uint8)
        mu = oracle.algdist(A, X, w)
        Pc, Pv, ls, st = oracle.ls_interp(A, X, w, cf, mu, 2)
        f = lambda a, b: np.sum(w * (X[0] - a * X[Pc[0, 0]] - b * X[Pc[0, 1]]) ** 2)
        g = np.linspace(-1, 1, 201)
        best = min(f(Pv[0, 0] + da, Pv[0, 1] + db) for da in g for db in g)
        assert ls[0] <= best + 1e-12
        assert abs(f(*Pv[0]) - ls[0]) <= 1e-12 * (1 + ls[0])


def test_ls_interp_unique_when_vectors_span():
    """Sec. 3.1 remark: with K >= caliber and spanning restricted vectors the
    LS solution is unique, so two orderings of the same set agree."""
    rng = np.random.default_rng(13)
    K = 4
    X = rng.standard_normal((5, K))
    A = _csr_from_dense(-np.ones((5, 5)) + 9 * np.eye(5))
    cf = np.array([0, 1, 1, 1, 1], np.uint8)
    mu1 = np.zeros(25); mu1[1:5] = [1, 2, 3, 4]
    mu2 = np.zeros(25); mu2[1:5] = [4, 3, 2, 1]
    a = oracle.ls_interp(A, X, None, cf, mu1, 4)
    b = oracle.ls_interp(A, X, None, cf, mu2, 4)
    pa = dict(zip(a[0][0], a[1][0]))
    pb = dict(zip(b[0][0], b[1][0]))
    assert set(pa) == set(pb) == {1, 2, 3, 4}
    assert all(abs(pa[j] - pb[j]) < 1e-10 for j in pa)
    assert a[2][0] < 1e-20  # K = caliber = 4: exact fit


# ---------------------------------------------------------------- adjoint
def _adjoint_case():
    """Log-normal 5-point operator made non-symmetric (a_ij != a_ji), so that
    A and its transpose play visibly different parts in the chain rule."""
    N = 6
    A = W.lognormal_2d_5pt(N, 1.0, 5)
    rid = A.row_ids()
    skew = 1.0 + 0.4 * np.random.default_rng(8).random(A.nnz)
    A = W.CSR(A.n, A.row_ptr, A.col, np.where(A.col != rid, A.val * skew, A.val))
    X0 = oracle.tv_init(A.n, 4, 21)
    cf = W.cf_red_is_coarse((N, N))
    w = np.array([1.0, 0.5, 2.0, 1.5])
    return A, X0, cf, w


def test_adjoint_matches_central_differences():
    A, X0, cf, w = _adjoint_case()
    sweeps, omega, cal = 4, 0.7, 4
    L, g, gw = oracle.ls_loss_grad(A, X0, sweeps, omega, w, cf, cal)
    assert abs(L - oracle.ls_loss(A, X0, sweeps, omega, w, cf, cal)) <= 1e-14 * L
    h = 1e-6
    fd = (oracle.ls_loss(A, X0, sweeps, omega + h, w, cf, cal)
          - oracle.ls_loss(A, X0, sweeps, omega - h, w, cf, cal)) / (2 * h)
    assert abs(gw - fd) <= 1e-6 * abs(fd) + 1e-9
    rng = np.random.default_rng(0)
    for e in list(rng.choice(A.nnz, 25, replace=False)) + [0, A.row_ptr[7] + 2]:
        hv = h * max(1.0, abs(A.val[e]))
        vp, vm = A.val.copy(), A.val.copy()
        vp[e] += hv
        vm[e] -= hv
        fd = (oracle.ls_loss(A, X0, sweeps, omega, w, cf, cal, val=vp)
              - oracle.ls_loss(A, X0, sweeps, omega, w, cf, cal, val=vm)) / (2 * hv)
        assert abs(g[e] - fd) <= 1e-5 * abs(fd) + 1e-8 * np.abs(g).max(), e


def test_adjoint_taylor_remainder_is_second_order():
    A, X0, cf, w = _adjoint_case()
    sweeps, omega, cal = 3, 0.8, 4
    L, g, gw = oracle.ls_loss_grad(A, X0, sweeps, omega, w, cf, cal)
    d = np.random.default_rng(1).standard_normal(A.nnz)
    dw = 0.3
    rem = []
    for h in (1e-2, 5e-3, 2.5e-3):
        Lh = oracle.ls_loss(A, X0, sweeps, omega + h * dw, w, cf, cal, val=A.val + h * d)
        rem.append(abs(Lh - L - h * (g @ d + gw * dw)))
    assert rem[1] / rem[0] < 0.3 and rem[2] / rem[1] < 0.3  # ~ 1/4 per halving
