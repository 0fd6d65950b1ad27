"""Pins of the oracle's compatible-relaxation coarsening (Sec. 3.2 eq:frelax,
eq:meas1; Sec. 4.2 Algorithm 1 and the candidate measure): the F-relaxation
against the colour-phase splitting written as a dense matrix and iterated
with numpy, the spectral radius of red-black Gauss-Seidel on the 1D Laplacian
(cos^2(pi h)), the exact zero rate of F-relaxation when every F point
couples only to C points, a hand case of the candidate rule, the greedy
independent set characterised by its defining properties, and the
coarsening loop's invariants."""
import math

import numpy as np
import pytest

import oracle
from paper_1106_5990_amd import workloads as W


def dense(A):
    M = np.zeros((A.n, A.n))
    for i in range(A.n):
        for e in range(A.row_ptr[i], A.row_ptr[i + 1]):
            M[i, A.col[e]] += A.val[e]
    return M


def lap1d(n):
    rp = [0]
    ci, va = [], []
    for i in range(n):
        for j, v in ((i - 1, -1.0), (i, 2.0), (i + 1, -1.0)):
            if 0 <= j < n:
                ci.append(j)
                va.append(v)
        rp.append(len(ci))
    return W.CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va))


def splitting_iterate(A, color, cf, nu):
    """u^nu of F-relaxation as a stationary iteration u <- u - M_ff^{-1} A_ff u,
    M holding the diagonal and the couplings to earlier colours (the
    colour-phase rule's splitting), on the F rows and columns only."""
    D = dense(A)
    F = np.nonzero(cf == 0)[0]
    Aff = D[np.ix_(F, F)]
    cF = color[F]
    M = np.where(cF[None, :] < cF[:, None], Aff, 0.0) + np.diag(np.diag(Aff))
    u = np.ones(len(F))
    for _ in range(nu):
        u = u - np.linalg.solve(M, Aff @ u)
    full = np.zeros(A.n)
    full[F] = u
    return full


@pytest.mark.parametrize("case", ["aniso9", "lap5", "lognormal"])
def test_f_relaxation_is_the_splitting_iteration(case):
    rng = np.random.default_rng(7)
    if case == "aniso9":
        N = 13
        A = W.rotated_anisotropic_9pt(N, 1e-2, math.pi / 5)
    elif case == "lap5":
        N = 14
        A = W.laplacian_2d_5pt(N)
    else:
        N = 12
        A = W.lognormal_2d_5pt(N, 1.0, 3)
    color = W.red_black((N, N))
    cf = (rng.random(A.n) < 0.3).astype(np.uint8)
    nu = 5
    rho, u = oracle.cr_rate(A, color, 2, cf, nu)
    want = splitting_iterate(A, color, cf, nu)
    assert np.max(np.abs(u - want)) <= 1e-12 * max(1.0, np.max(np.abs(want)))
    assert np.all(u[cf == 1] == 0.0)
    nf = int((cf == 0).sum())
    assert rho == pytest.approx((np.linalg.norm(want) / math.sqrt(nf)) ** (1.0 / nu), rel=1e-12)


def test_rate_of_red_black_gauss_seidel_on_the_1d_laplacian():
    """With C empty, rho_f estimates the spectral radius of red-black
    Gauss-Seidel on the 1D Dirichlet Laplacian, cos^2(pi/(n+1)); from the
    constant start the estimate converges to it as nu grows."""
    n = 31
    A = lap1d(n)
    color = (np.arange(n) % 2).astype(np.int32)
    cf = np.zeros(n, np.uint8)
    rho_true = math.cos(math.pi / (n + 1)) ** 2
    r400, _ = oracle.cr_rate(A, color, 2, cf, 400)
    r800, _ = oracle.cr_rate(A, color, 2, cf, 800)
    assert abs(r800 - rho_true) < abs(r400 - rho_true) + 1e-15
    assert r800 == pytest.approx(rho_true, abs=2e-3)


def test_f_points_coupled_only_to_c_points_converge_in_one_sweep():
    """5-point Laplacian, C = the red points: every F (black) point's
    neighbours are C points, A_ff is diagonal, one F-relaxation sweep maps
    u_f to zero and rho_f = 0."""
    N = 16
    A = W.laplacian_2d_5pt(N)
    color = W.red_black((N, N))
    cf = (color == 0).astype(np.uint8)
    rho, u = oracle.cr_rate(A, color, 2, cf, 5)
    assert rho == 0.0 and np.all(u == 0.0)
    cf2, rhos, nc = oracle.cr_coarsen(A, color, 2, np.ones(A.nnz), 0.25, cf0=cf)
    assert len(rhos) == 1 and rhos[0] == 0.0 and nc[0] == int(cf.sum())
    assert np.array_equal(cf2, cf)
    # everything coarse: F is empty and the rate is 0
    cfa = np.ones(A.n, np.uint8)
    assert oracle.cr_rate(A, color, 2, cfa, 5)[0] == 0.0


def test_candidate_rule_hand_case():
    cf = np.array([0, 0, 0, 1, 0], np.uint8)
    u = np.array([0.5, -1.0, 0.2, 7.0, -0.4])  # the C entry is not part of the max
    z = oracle.cr_candidates(cf, u, 0.4)
    assert z.tolist() == [1, 1, 0, 0, 0]
    # sigma equal to tol is not a candidate; all-zero u gives none
    assert oracle.cr_candidates(cf, u, 0.5).tolist() == [0, 1, 0, 0, 0]
    assert oracle.cr_candidates(cf, np.zeros(5), 0.1).tolist() == [0] * 5


def _priority(A, strong, seed):
    lam = np.bincount(A.col[strong.astype(bool)], minlength=A.n)
    h = [oracle.splitmix64_nth(seed, i + 1) for i in range(A.n)]
    return [(int(lam[i]), int(h[i]), i) for i in range(A.n)]


def _neighbours(A, strong):
    nb = [set() for _ in range(A.n)]
    for i in range(A.n):
        for e in range(A.row_ptr[i], A.row_ptr[i + 1]):
            j = int(A.col[e])
            if strong[e] and j != i:
                nb[i].add(j)
                nb[j].add(i)
    return nb


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_independent_set_is_the_greedy_one(seed):
    """On random strong graphs (not symmetric) and candidate sets: the set is
    independent and maximal among the candidates, and every candidate left
    out has a chosen neighbour of higher priority -- the property that
    singles out the greedy set in decreasing priority."""
    rng = np.random.default_rng(seed)
    A = W.rgg_laplacian(300, 8.0, (seed, 0))
    strong = (rng.random(A.nnz) < 0.5).astype(np.uint8)
    strong[A.col == A.row_ids()] = 0
    z = (rng.random(A.n) < 0.7).astype(np.uint8)
    sel = oracle.independent_set(A, strong, z, seed)
    pr = _priority(A, strong, seed)
    nb = _neighbours(A, strong)
    assert np.all(sel <= z) and sel.sum() > 0
    for i in range(A.n):
        if sel[i]:
            assert not any(sel[j] for j in nb[i] if z[j]), i
        elif z[i]:
            blockers = [j for j in nb[i] if sel[j]]
            assert blockers, i  # maximal
            assert any(pr[j] > pr[i] for j in blockers), i  # greedy order
    # the rule is a function of the graph: a relabelled seed changes only ties
    sel2 = oracle.independent_set(A, strong, z, seed)
    assert np.array_equal(sel, sel2)


def test_independent_set_on_a_path_prefers_heavy_vertices():
    """Hand case: path 0-1-2-3-4 with strong entries pointing at 1 and 3
    (lambda = 2 each) and none at 0, 2, 4: the set is {1, 3}."""
    n = 5
    rp, ci, st = [0], [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                ci.append(j)
                st.append(1 if j in (1, 3) and j != i else 0)
        rp.append(len(ci))
    A = W.CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.ones(len(ci)))
    sel = oracle.independent_set(A, np.array(st, np.uint8), np.ones(n, np.uint8), 11)
    assert sel.tolist() == [0, 1, 0, 1, 0]


@pytest.mark.parametrize("wl", [1, 2])
def test_coarsening_loop_invariants(wl):
    """Algorithm 1 on a test-sized workload: C only grows, each growth step
    adds an independent set of that step's candidates on that step's
    strength graph, and the loop stops with rho_f <= delta (or no
    candidates, or the stage limit)."""
    w = W.workload(wl, size=24)
    A = w.A
    color = w.color if w.color is not None else W.red_black((24, 24))
    X = oracle.tv_init(A.n, w.K, 5)
    X, _ = oracle.color_gs(A, X, color, 2, 5)
    mu = oracle.algdist(A, X)
    cf, rho, nc = oracle.cr_coarsen(A, color, 2, mu, 0.25, nu=5, delta=0.7, max_stages=20,
                                    seed=9)
    assert len(rho) >= 2 and rho[0] > 0.7
    assert rho[-1] <= 0.7 or len(rho) == 21
    assert np.all(np.diff(nc) > 0) and nc[-1] == cf.sum()
    # replay the stages by hand from the oracle's building blocks
    c = np.zeros(A.n, np.uint8)
    for s in range(len(rho) - 1):
        r, u = oracle.cr_rate(A, color, 2, c, 5)
        assert r == rho[s]
        z = oracle.cr_candidates(c, u, 1.0 - r)
        strong, _ = oracle.strength(A, mu, 0.25, fmask=(c == 0).astype(np.uint8))
        sel = oracle.independent_set(A, strong, z, 9 + s)
        nb = _neighbours(A, strong)
        for i in np.nonzero(sel)[0]:
            assert not any(sel[j] for j in nb[i])
        c = c | sel
        assert c.sum() == nc[s + 1]
    assert np.array_equal(c, cf)


def test_coarsening_on_a_pattern_equal_to_a_gives_the_plain_call():
    w = W.workload(2, size=20)
    A = w.A
    X, _ = oracle.color_gs(A, oracle.tv_init(A.n, 8, 2), w.color, 2, 5)
    mu = oracle.algdist(A, X)
    got = oracle.cr_coarsen(A, w.color, 2, mu, 0.25, seed=4,
                            G=oracle.Pattern(A.n, A.row_ptr, A.col))
    want = oracle.cr_coarsen(A, w.color, 2, mu, 0.25, seed=4)
    for g, r in zip(got, want):
        assert np.array_equal(g, r)


def test_coarsening_loop_on_the_graph_of_a_squared():
    """Algorithm 1 with M^2 (Sec. 4.2): the strength graph and the
    independent set on the graph of A^2 with distances on it, CR relaxing
    with A.  Replayed by hand from the building blocks: each growth step
    adds an independent set of the candidates in the symmetric closure of
    that step's strength graph on A^2, whose edges reach two steps in A."""
    w = W.workload(2, size=24)
    A = w.A
    X, _ = oracle.color_gs(A, oracle.tv_init(A.n, 8, 5), w.color, 2, 5)
    G = oracle.power_pattern(A, 2)
    mu = oracle.algdist_graph(A, G, X)
    cf, rho, nc = oracle.cr_coarsen(A, w.color, 2, mu, 0.25, seed=9, G=G)
    assert len(rho) >= 2 and rho[0] > 0.7
    assert rho[-1] <= 0.7 or len(rho) == 21
    Gc = W.CSR(A.n, G.row_ptr, G.col, np.zeros(len(G.col)))
    c = np.zeros(A.n, np.uint8)
    for s in range(len(rho) - 1):
        r, u = oracle.cr_rate(A, w.color, 2, c, 5)
        assert r == rho[s]
        z = oracle.cr_candidates(c, u, 1.0 - r)
        strong, _ = oracle.strength(Gc, mu, 0.25, fmask=(c == 0).astype(np.uint8))
        sel = oracle.independent_set(Gc, strong, z, 9 + s)
        nb = _neighbours(Gc, strong)
        for i in np.nonzero(sel)[0]:
            assert not any(sel[j] for j in nb[i])
        c = c | sel
        assert c.sum() == nc[s + 1]
    assert np.array_equal(c, cf)
    # M^2 has strong edges two steps away in A (the first stage's graph)
    strong, _ = oracle.strength(Gc, mu, 0.25, fmask=np.ones(A.n, np.uint8))
    rid = Gc.row_ids()
    in_a = set(zip(A.row_ids().tolist(), A.col.tolist()))
    far = [(int(i), int(j)) for i, j, st in zip(rid, Gc.col, strong) if st and (i, j) not in in_a]
    assert len(far) > 0
