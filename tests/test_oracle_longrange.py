"""Pins of the oracle's long-range connectivity and interpolatory-set search
(Sec. 4.1 eq. graph, the closing remark of Sec. 4.2, Sec. 4.3 eq:nbhd and
the set-size penalty) against independent routes: sparse matrix powers,
closed-form neighbourhood sizes, numpy least squares over itertools
enumerations, hand-built cases whose functional values are known exactly,
the monotonicity of Sec. 4.3, and the paper's claim that long-range
distances let strength and interpolation follow an anisotropy the stencil
itself does not contain (Sec. 5.3, Figs. 2-3)."""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_1106_5990_amd import workloads as W


def _csr_from_dense(D):
    D = np.asarray(D, dtype=np.float64)
    n = D.shape[0]
    mask = D != 0
    mask[np.arange(n), np.arange(n)] = True
    rows, cols = np.nonzero(mask)
    rp = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    return W.CSR(n, rp, cols.astype(np.int32), D[rows, cols])


def _random_asymmetric(n, seed, density=0.15):
    rng = np.random.default_rng(seed)
    D = np.where(rng.random((n, n)) < density, -rng.random((n, n)), 0.0)
    D += np.diag(4.0 + rng.random(n))
    return _csr_from_dense(D)


# ---------------------------------------------------------------- pattern of A^d
@pytest.mark.parametrize("case", ["lap5", "aniso9", "rgg", "asym", "lap3d"])
@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_power_pattern_matches_sparse_matrix_powers(case, d):
    """Row i of A^d's pattern = the nonzeros of (|A|)^d (nonnegative
    entries: no cancellation), columns sorted."""
    A = {"lap5": lambda: W.laplacian_2d_5pt(9),
         "aniso9": lambda: W.rotated_anisotropic_9pt(8, 1e-3, math.pi / 6),
         "rgg": lambda: W.rgg_laplacian(150, 6.0, 3),
         "asym": lambda: _random_asymmetric(40, 5),
         "lap3d": lambda: W.lognormal_3d_7pt(5, 1.0, 2)}[case]()
    G = oracle.power_pattern(A, d)
    B = sp.csr_matrix((np.abs(A.val), A.col, A.row_ptr), shape=(A.n, A.n))
    P = B.copy()
    for _ in range(d - 1):
        P = P @ B
    P = sp.csr_matrix(P)
    P.sort_indices()
    P.eliminate_zeros()
    assert np.array_equal(G.row_ptr, P.indptr)
    assert np.array_equal(G.col, P.indices)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_power_pattern_closed_form_neighbourhoods(d):
    """Interior rows: 5-point -> the diamond |dx| + |dy| <= d, 2d^2 + 2d + 1
    points; 9-point -> the (2d + 1)^2 box; 7-point 3D -> the octahedron
    (2d + 1)(2d^2 + 2d + 3) / 3 points."""
    N = 2 * d + 5
    c = (N // 2) * N + N // 2
    G5 = oracle.power_pattern(W.laplacian_2d_5pt(N), d)
    assert G5.row_ptr[c + 1] - G5.row_ptr[c] == 2 * d * d + 2 * d + 1
    G9 = oracle.power_pattern(W.rotated_anisotropic_9pt(N, 0.1, 0.3), d)
    cols = G9.col[G9.row_ptr[c]:G9.row_ptr[c + 1]]
    dy, dx = np.divmod(cols - c + (d * N + d), N)
    assert len(cols) == (2 * d + 1) ** 2 and dx.max() - dx.min() == 2 * d
    N3 = 2 * d + 3
    c3 = ((N3 // 2) * N3 + N3 // 2) * N3 + N3 // 2
    G3 = oracle.power_pattern(W.lognormal_3d_7pt(N3, 1.0, 1), d)
    assert G3.row_ptr[c3 + 1] - G3.row_ptr[c3] == (2 * d + 1) * (2 * d * d + 2 * d + 3) // 3


# ---------------------------------------------------------------- distances on G_d
def _residual_target(A, X):
    S = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
    return X - (S @ X) / S.diagonal()[:, None]


@pytest.mark.parametrize("target", [oracle.TARGET_PLAIN, oracle.TARGET_RESIDUAL])
@pytest.mark.parametrize("seed", [0, 1])
def test_graph_distances_match_lstsq(target, seed):
    """mu_ij on A^2's pattern = the weighted one-column least-squares
    residual of the row's target (from A) on x_j (numpy lstsq)."""
    rng = np.random.default_rng(seed)
    A = _random_asymmetric(12, seed + 7, 0.2)
    K = 5
    X = rng.standard_normal((A.n, K))
    w = 0.5 + rng.random(K)
    G = oracle.power_pattern(A, 2)
    mu, p = oracle.algdist_graph(A, G, X, w, target, want_p=True)
    T = X if target == oracle.TARGET_PLAIN else _residual_target(A, X)
    sw = np.sqrt(w)
    for e, (i, j) in enumerate(zip(G.row_ids(), G.col)):
        sol, res, *_ = np.linalg.lstsq((sw * X[j])[:, None], sw * T[i], rcond=None)
        r = sw * T[i] - sol[0] * sw * X[j]
        assert mu[e] == pytest.approx(float(r @ r), rel=1e-10, abs=1e-13)
        assert p[e] == pytest.approx(sol[0], rel=1e-10, abs=1e-13)
        assert mu[e] >= 0.0


def test_graph_distances_on_the_first_power_are_the_distances():
    """G = A^1 gives the distances of the stencil itself (oracle.algdist)."""
    A = W.rotated_anisotropic_9pt(10, 1e-3, math.pi / 6)
    X = oracle.tv_init(A.n, 8, 3)
    G = oracle.power_pattern(A, 1)
    for t in (oracle.TARGET_PLAIN, oracle.TARGET_RESIDUAL):
        assert np.array_equal(oracle.algdist_graph(A, G, X, None, t), oracle.algdist(A, X, None, t))


def _knight_case(N=40):
    """The rotated 9-point operator with tan(alpha) = 1/2: smooth error is
    constant along xi = (2, 1)/sqrt(5), a direction no stencil neighbour
    lies on, but the offset (2, 1) of A^2's pattern does.  Test vectors by
    the paper's protocol (40 Gauss-Seidel sweeps, Sec. 5.2)."""
    alpha = math.atan(0.5)
    A = W.rotated_anisotropic_9pt(N, 1e-3, alpha)
    X, _ = oracle.color_gs(A, oracle.tv_init(A.n, 8, 11), W.red_black((N, N)), 2, 40)
    iy, ix = np.divmod(np.arange(A.n), N)
    inner = (ix > 2) & (ix < N - 3) & (iy > 2) & (iy < N - 3)
    return A, X, inner


def test_long_range_distances_find_the_knight_move_anisotropy():
    """On G_2 the offset +-(2, 1), which lies on xi, has the least median
    distance of all 24 offsets, and is the row's least distance in most
    interior rows (Sec. 5.3: larger d lets the strength graph follow
    anisotropies not aligned with the stencil)."""
    N = 40
    A, X, inner = _knight_case(N)
    G = oracle.power_pattern(A, 2)
    mu = oracle.algdist_graph(A, G, X)
    rid = G.row_ids()
    off = G.col.astype(np.int64) - rid
    sel = inner[rid] & (off != 0)
    med = {o: np.median(mu[sel & (off == o)]) for o in np.unique(off[sel])}
    assert sorted(med, key=med.get)[:2] == sorted([N + 2, -(N + 2)], key=med.get)
    wins = 0
    rows = np.nonzero(inner)[0]
    for i in rows:
        s, e = G.row_ptr[i], G.row_ptr[i + 1]
        m = np.where(off[s:e] == 0, np.inf, mu[s:e])
        wins += abs(off[s + int(np.argmin(m))]) == N + 2
    assert wins >= 0.7 * len(rows)


# ---------------------------------------------------------------- interpolatory-set search
def _search_case(seed, n=14, K=6, density=0.3):
    rng = np.random.default_rng(seed)
    D = np.where(rng.random((n, n)) < density, -rng.random((n, n)), 0.0)
    D = D + D.T + np.diag(8.0 + rng.random(n))
    A = _csr_from_dense(D)
    X = rng.standard_normal((A.n, K))
    w = 0.5 + rng.random(K)
    cf = (rng.random(n) < 0.5).astype(np.uint8)
    return A, X, w, cf


def _lstsq_val(T, X, w, cols):
    sw = np.sqrt(w)
    M = (sw[:, None] * X[list(cols)].T)
    sol, *_ = np.linalg.lstsq(M, sw * T, rcond=None)
    r = sw * T - M @ sol
    return float(r @ r), sol


@pytest.mark.parametrize("target", [oracle.TARGET_PLAIN, oracle.TARGET_RESIDUAL])
@pytest.mark.parametrize("seed", range(3))
def test_search_best_per_size_matches_brute_force(target, seed):
    """For every F row and size m, best_m / S equals the least numpy lstsq
    residual over all m-subsets of the row's C-candidates in A^2's pattern
    (itertools), the chosen set attains its size's best, and its weights are
    lstsq's."""
    A, X, w, cf = _search_case(seed)
    G = oracle.power_pattern(A, 2)
    cal = 3
    Pc, Pv, ls, st, best, nc = oracle.ls_search(A, G, X, w, cf, cal, 1.5, target)
    T = X if target == oracle.TARGET_PLAIN else _residual_target(A, X)
    for i in range(A.n):
        if cf[i]:
            assert Pc[i, 0] == i and Pv[i, 0] == 1.0 and ls[i] == 0.0
            continue
        cand = [j for j in G.col[G.row_ptr[i]:G.row_ptr[i + 1]] if j != i and cf[j]]
        assert nc[i] == len(cand)
        S = float(w @ (T[i] * T[i]))
        assert best[i, 0] == pytest.approx(S, rel=1e-12)
        for m in range(1, cal + 1):
            vals = [_lstsq_val(T[i], X, w, W_)[0] for W_ in itertools.combinations(cand, m)]
            if not vals:
                assert best[i, m] == -1.0
                continue
            assert best[i, m] == pytest.approx(min(vals) / S, rel=1e-9, abs=1e-14)
        chosen = [c for c in Pc[i] if c >= 0]
        if not cand:
            assert st[i] == 1 and not chosen
            continue
        val, sol = _lstsq_val(T[i], X, w, chosen)
        assert val / S == pytest.approx(best[i, len(chosen)], rel=1e-9, abs=1e-14)
        assert ls[i] == pytest.approx(val, rel=1e-9, abs=1e-14)
        assert np.allclose(Pv[i, :len(chosen)], sol, rtol=1e-9, atol=1e-12)
        assert list(chosen) == sorted(chosen)


def _hand_case(b2, c2, noise=True, K=5):
    """F row 0 with C-neighbours 1, 2 (and 3): target t = (a, b, c, 0, 0)
    with a^2 = 0.9, b^2 = b2, c^2 = c2 (S = 0.9 + b2 + c2), x_1 = e_1,
    x_2 = e_2, x_3 = e_4 (orthogonal to t).  Then LS({1}) = b2 + c2,
    LS({2}) = 0.9 + c2, LS({1,2}) = c2 and adding 3 changes nothing."""
    n = 4 if noise else 3
    D = np.eye(n) * 4.0
    D[0, 1:] = D[1:, 0] = -1.0
    A = _csr_from_dense(D)
    X = np.zeros((n, K))
    X[0, :3] = [math.sqrt(0.9), math.sqrt(b2), math.sqrt(c2)]
    X[1, 0] = 1.0
    X[2, 1] = 1.0
    if noise:
        X[3, 3] = 1.0
    cf = np.array([0] + [1] * (n - 1), dtype=np.uint8)
    return A, X, cf


@pytest.mark.parametrize("scale", [1.0, 3.0])
@pytest.mark.parametrize("b2, c2, gamma, size", [
    (0.08, 0.02, 1.5, 2),   # 0.02 < 0.1^1.5 = 0.0316: the pair is preferred
    (0.05, 0.05, 1.5, 1),   # 0.05 > 0.0316: one point is kept
    (0.05, 0.05, 1.0, 2),   # gamma = 1: any reduction is accepted
    (0.095, 0.005, 2.0, 2),  # 0.005 < 0.1^2 = 0.01
    (0.08, 0.02, 2.0, 1),   # 0.02 > 0.01: kept
])
def test_search_penalty_rule_on_hand_built_values(b2, c2, gamma, size, scale):
    """The rule acts on values relative to the empty set's S (the target
    scaled by 3 gives the same choices)."""
    A, X, cf = _hand_case(b2, c2)
    X[0] *= scale
    S = (0.9 + b2 + c2) * scale ** 2
    G = oracle.power_pattern(A, 1)
    Pc, Pv, ls, st, best, nc = oracle.ls_search(A, G, X, None, cf, 3, gamma, rows=[0])
    assert best[0, 0] == pytest.approx(S, rel=1e-12)
    assert best[0, 1] == pytest.approx((b2 + c2) * scale ** 2 / S, rel=1e-12)
    assert best[0, 2] == pytest.approx(c2 * scale ** 2 / S, rel=1e-12)
    assert best[0, 3] == pytest.approx(c2 * scale ** 2 / S, rel=1e-12)  # orthogonal point: no help
    chosen = [c for c in Pc[0] if c >= 0]
    assert chosen == ([1] if size == 1 else [1, 2])
    want = ((b2 + c2) if size == 1 else c2) * scale ** 2
    assert ls[0] == pytest.approx(want, rel=1e-12, abs=1e-15)


def test_search_penalty_compares_with_the_incumbent():
    """Three orthogonal candidates, t = (a, b, c, d) on them and a fourth
    axis: best_1 = 0.1 ({1}), best_2 = 0.05 ({1, 2}), best_3 = 0.005.
    Against the incumbent {1}: 0.05 > 0.1^1.5 and 0.005 > 0.1^3 = 0.001, so
    {1} stays (a scan that compared size 3 with size 2 would take it:
    0.005 < 0.05^1.5)."""
    K = 5
    D = np.eye(4) * 4.0
    D[0, 1:] = D[1:, 0] = -1.0
    A = _csr_from_dense(D)
    X = np.zeros((4, K))
    X[0, :4] = np.sqrt([0.9, 0.05, 0.045, 0.005])
    X[1, 0] = X[2, 1] = X[3, 2] = 1.0
    cf = np.array([0, 1, 1, 1], dtype=np.uint8)
    G = oracle.power_pattern(A, 1)
    Pc, Pv, ls, st, best, nc = oracle.ls_search(A, G, X, None, cf, 3, 1.5, rows=[0])
    assert np.allclose(best[0, 1:], [0.1, 0.05, 0.005], rtol=1e-12)
    assert list(Pc[0]) == [1, -1, -1]


def test_search_is_exhaustive_not_greedy():
    """t = x_1 + x_2 exactly, while x_3 is the single best point: a greedy
    forward selection starting from x_3 cannot reach zero, the search over
    all pairs finds {1, 2} with a zero functional."""
    K = 4
    D = np.eye(4) * 4.0
    D[0, 1:] = D[1:, 0] = -1.0
    A = _csr_from_dense(D)
    X = np.zeros((4, K))
    X[1, 0] = 1.0
    X[2, 1] = 1.0
    X[3] = [0.9 / math.sqrt(2), 0.9 / math.sqrt(2), 0.436, 0.0]
    X[0] = X[1] + X[2]
    cf = np.array([0, 1, 1, 1], dtype=np.uint8)
    G = oracle.power_pattern(A, 1)
    Pc, Pv, ls, st, best, nc = oracle.ls_search(A, G, X, None, cf, 2, 1.5, rows=[0])
    single = {j: _lstsq_val(X[0], X, np.ones(K), [j])[0] for j in (1, 2, 3)}
    assert min(single, key=single.get) == 3
    assert list(Pc[0]) == [1, 2] and abs(ls[0]) < 1e-28
    assert np.allclose(Pv[0], [1.0, 1.0], atol=1e-14)


@pytest.mark.parametrize("seed", range(3))
def test_search_best_is_monotone_in_the_size(seed):
    """Sec. 4.3: W' within W'' gives LS_W' >= LS_W''; so the best value can
    only fall as the size grows (no dependent sets in random data)."""
    A, X, w, cf = _search_case(seed + 10, n=16, K=8, density=0.35)
    G = oracle.power_pattern(A, 2)
    *_, best, nc = oracle.ls_search(A, G, X, w, cf, 4, 1.5)
    for i in np.nonzero(cf == 0)[0]:
        b = [v for v in best[i, 1:] if v >= 0]
        assert all(b[q + 1] <= b[q] * (1 + 1e-12) for q in range(len(b) - 1))


def test_search_exact_recovery_and_dependent_sets():
    """x_i = 0.3 x_a - 1.2 x_b for two C-neighbours: that pair with those
    weights and a vanishing functional; a duplicated candidate column makes
    every set holding both copies dependent, and they are skipped."""
    A, X, w, cf = _search_case(4, n=14, K=6, density=0.4)
    G = oracle.power_pattern(A, 2)
    i = int(np.nonzero(cf == 0)[0][0])
    cand = [j for j in G.col[G.row_ptr[i]:G.row_ptr[i + 1]] if j != i and cf[j]]
    assert len(cand) >= 3
    a, b, c = cand[:3]
    X = X.copy()
    X[i] = 0.3 * X[a] - 1.2 * X[b]
    X[c] = X[a]  # a duplicate of a
    Pc, Pv, ls, st, best, nc = oracle.ls_search(A, G, X, w, cf, 3, 1.5, rows=[i])
    assert list(Pc[0][:2]) == sorted([a, b]) and Pc[0][2] == -1
    want = {a: 0.3, b: -1.2}
    assert np.allclose(Pv[0][:2], [want[Pc[0][0]], want[Pc[0][1]]], atol=1e-12)
    assert ls[0] < 1e-24 * float(w @ (X[i] * X[i]))


@pytest.mark.parametrize("rel2,dep", [(1e-10, 1), (3e-9, 1), (3e-8, 0), (1e-6, 0)])
def test_fit_sets_dependence_rule(rel2, dep):
    """The search's dependence rule in closed form: x_c = x_a + delta u with
    u orthogonal to x_a and |u| = |x_a| leaves x_c a part orthogonal to x_a
    whose squared norm is delta^2 / (1 + delta^2) of |x_c|^2; the set
    {a, c} is dependent exactly when that is <= 1e-8 (in either order)."""
    A, X, w, cf = _search_case(6, n=12, K=8, density=0.4)
    X = X.copy()
    a, c, i = 0, 1, 2
    u = X[3] - (X[3] @ X[a]) / (X[a] @ X[a]) * X[a]
    u *= np.linalg.norm(X[a]) / np.linalg.norm(u)
    d2 = rel2 / (1.0 - rel2)  # delta^2 with delta^2 / (1 + delta^2) = rel2
    X[c] = X[a] + np.sqrt(d2) * u
    for pair in ([a, c], [c, a]):
        sets = np.array([pair + [-1, -1]], dtype=np.int32)
        pv, lv, rd = oracle.ls_fit_sets(A, X, None, sets, [i])
        assert rd[0] == dep, (pair, rel2)
        if not dep:
            sol, *_ = np.linalg.lstsq(X[pair].T, X[i], rcond=None)
            assert np.allclose(pv[0][:2], sol, rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("seed", range(2))
def test_fit_sets_matches_lstsq(seed):
    A, X, w, cf = _search_case(seed + 20)
    rng = np.random.default_rng(seed)
    rows = np.arange(A.n, dtype=np.int32)
    sets = -np.ones((A.n, 3), dtype=np.int32)
    for i in range(A.n):
        m = int(rng.integers(0, 4))
        sets[i, :m] = np.sort(rng.choice(A.n, m, replace=False))
    Pv, ls, rd = oracle.ls_fit_sets(A, X, w, sets, rows)
    for i in range(A.n):
        cols = [c for c in sets[i] if c >= 0]
        assert rd[i] == 0
        if not cols:
            assert ls[i] == pytest.approx(float(w @ (X[i] * X[i])), rel=1e-12)
            continue
        val, sol = _lstsq_val(X[i], X, w, cols)
        assert ls[i] == pytest.approx(val, rel=1e-9, abs=1e-14)
        assert np.allclose(Pv[i, :len(cols)], sol, rtol=1e-9, atol=1e-12)


def test_search_interpolation_follows_the_knight_move_anisotropy():
    """C = red points, search depth 2, caliber 2 to 4, gamma = 1.5: most
    interior F points interpolate from their two C-neighbours at +-(2, 1),
    on the direction of the anisotropy (Sec. 5.3: with A^2 the LS
    interpolation follows an anisotropy the stencil does not see)."""
    N = 40
    A, X, inner = _knight_case(N)
    G = oracle.power_pattern(A, 2)
    cf = W.cf_red_is_coarse((N, N))
    rows = np.nonzero(inner & (cf == 0))[0].astype(np.int32)
    for cal in (2, 4):
        Pc, Pv, ls, st, best, nc = oracle.ls_search(A, G, X, None, cf, cal, 1.5, rows=rows)
        hit = sum(sorted(int(c) - int(i) for c in Pc[r] if c >= 0) == [-(N + 2), N + 2]
                  for r, i in enumerate(rows))
        assert hit >= 0.8 * len(rows)
