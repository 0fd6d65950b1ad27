"""The long-range calls on the GPU against the oracle: the pattern of A^d
(bit-exact), distances and the strength graph on it (the per-step bars of
the short-range distances), and the search over interpolatory sets
(identical sets and statuses wherever the oracle's decision is not within
rounding of a tie; where it is, the GPU's set is checked to be a valid
choice; weights and functional to the LS bars)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1106_5990_amd import workloads as W
from gpu_common import check_mu, dev_csr, lib, say, to_np

pytestmark = pytest.mark.gpu


def _csr_from_dense(D):
    D = np.asarray(D, dtype=np.float64)
    n = D.shape[0]
    mask = D != 0
    mask[np.arange(n), np.arange(n)] = True
    rows, cols = np.nonzero(mask)
    rp = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    return W.CSR(n, rp, cols.astype(np.int32), D[rows, cols])


def _asym(n, seed, density):
    rng = np.random.default_rng(seed)
    D = np.where(rng.random((n, n)) < density, -rng.random((n, n)), 0.0)
    return _csr_from_dense(D + np.diag(4.0 + rng.random(n)))


def _matrices():
    return {"lap5": W.laplacian_2d_5pt(33), "aniso9": W.rotated_anisotropic_9pt(30, 1e-3, 0.4),
            "rgg": W.rgg_laplacian(2000, 8.0, 11), "asym": _asym(300, 4, 0.01),
            # rows of A^2 from 16 to 97 entries: both sides of the per-lane list
            "rgg20": W.rgg_laplacian(1500, 20.0, 12),
            "lap3d": W.lognormal_3d_7pt(12, 1.0, 3), "one": W.laplacian_2d_5pt(1)}


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_power_graph_is_the_oracle_pattern(d):
    ad = lib()
    for name, A in _matrices().items():
        say("pattern of A^%d, %s (n = %d)" % (d, name, A.n))
        Ad = dev_csr(A, torch.float64)
        G = ad.power_graph(Ad, d)
        R = oracle.power_pattern(A, d)
        assert np.array_equal(to_np(G.row_ptr), R.row_ptr), name
        assert np.array_equal(to_np(G.col), R.col), name
    assert ad.status(clear=True) == 0


def test_power_graph_limits():
    """Rows of A^d past 1024 entries are refused; an empty matrix gives an
    empty pattern; d < 1 is an argument error."""
    ad = lib()
    A = _asym(2000, 8, 0.05)  # about 100 entries per row: A^2 rows pass 1024
    assert oracle.power_pattern(A, 2).row_ptr[1] > 1024
    Ad = dev_csr(A, torch.float64)
    with pytest.raises(ad.AlgdistError, match="AD_EUNSUPPORTED"):
        ad.power_graph(Ad, 2)
    with pytest.raises(ad.AlgdistError, match="AD_EINVAL"):
        ad.power_graph(Ad, 0)
    E = ad.Csr(torch.zeros(1, dtype=torch.int32, device="cuda"),
               torch.zeros(0, dtype=torch.int32, device="cuda"),
               torch.zeros(0, dtype=torch.float64, device="cuda"))
    G = ad.power_graph(E, 2)
    assert G.nnz == 0 and to_np(G.row_ptr).tolist() == [0]
    assert ad.status(clear=True) == 0


@pytest.mark.parametrize("d,mat", [(2, "aniso9"), (2, "rgg20"), (3, "aniso9")])
def test_power_graph_cols_with_foreign_row_pointers(d, mat):
    """power_graph_cols with row pointers that do not match A^d (rows one
    entry short or long, alternately): the pattern flag is raised, each row
    holds the first min(room, |row|) columns of the true row, and nothing
    lands outside the rows (a guard region after the last row stays)."""
    ad = lib()
    A = _matrices()[mat]
    Ad = dev_csr(A, torch.float64)
    R = oracle.power_pattern(A, d)
    cnt = np.diff(R.row_ptr).astype(np.int64)
    room = np.maximum(cnt + np.where(np.arange(A.n) % 2 == 0, -1, 1), 0)
    rpd = np.concatenate([[0], np.cumsum(room)]).astype(np.int32)
    guard = 4096
    col = torch.full((int(rpd[-1]) + guard,), -7, dtype=torch.int32, device="cuda")
    ad.status(clear=True)
    rc = ad._lib.power_graph_cols(ad.handle(0), Ad.ref(), d, ad._ptr(torch.as_tensor(rpd, device="cuda")),
                                  ad._ptr(col), ad._stream())
    assert rc == 0
    got = to_np(col)
    assert ad.status(clear=True) & ad.STAT_PATTERN
    assert np.all(got[int(rpd[-1]):] == -7)
    for i in range(A.n):
        w = min(room[i], cnt[i])
        assert np.array_equal(got[rpd[i]:rpd[i] + w], R.col[R.row_ptr[i]:R.row_ptr[i] + w]), i


def _graph_csr(G, n):
    rp, col = to_np(G.row_ptr), to_np(G.col)
    return W.CSR(n, rp, col, np.zeros(len(col)))


def _saa_graph(Gc, T, w=None):
    w = np.ones(T.shape[1]) if w is None else np.asarray(w)
    return ((T * T * w).sum(1))[Gc.row_ids()]


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("target", ["plain", "residual"])
@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("lpr", [0, 4])
def test_distances_on_the_pattern_of_a_power(dt, target, weighted, lpr):
    """mu on A^2's pattern (and A^3's) against the oracle given the same
    panel: FP64 1e-10, FP32 1e-4 relative (with the S_aa floors); the
    strength graph on that pattern bit-exact given mu."""
    ad = lib()
    N, K = 37, 16
    A = W.rotated_anisotropic_9pt(N, 1e-3, math.atan(0.5))
    if dt == torch.float32:
        A = W.CSR(A.n, A.row_ptr, A.col, A.val.astype(np.float32).astype(np.float64))
    Ad = dev_csr(A, dt)
    color = torch.as_tensor(W.red_black((N, N)), device="cuda")
    X = ad.setup_testvectors(Ad, K, seed=9, relax="gs", sweeps=3, color=color, ncolors=2)
    x = to_np(X).astype(np.float64)
    w = (0.5 + np.random.default_rng(2).random(K)) if weighted else None
    wt = None if w is None else torch.as_tensor(w, device="cuda")
    ad.set_launch("algdist", dt, K, lanes_per_row=lpr)
    try:
        for d in (2, 3):
            say("distances on A^%d: %s %s weighted=%s lpr=%d" % (d, dt, target, weighted, lpr))
            G = ad.power_graph(Ad, d)
            Gc = _graph_csr(G, A.n)
            mu, strong, ns = ad.algebraic_distance_graph(Ad, G, X, w=wt, target=target, fuse=True,
                                                         theta=0.25)
            tg = oracle.TARGET_PLAIN if target == "plain" else oracle.TARGET_RESIDUAL
            ref = oracle.algdist_graph(A, oracle.Pattern(A.n, Gc.row_ptr, Gc.col), x, w, tg)
            if target == "plain":
                T = x
            else:
                import scipy.sparse as sp
                S_ = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
                T = x - (S_ @ x) / S_.diagonal()[:, None]
            mu_h = to_np(mu).astype(np.float64)
            check_mu(mu_h, ref, _saa_graph(Gc, T, w), dt, "A^%d" % d)
            s_ref, ns_ref = oracle.strength(Gc, mu_h, 0.25)
            assert np.array_equal(to_np(strong), s_ref) and np.array_equal(to_np(ns), ns_ref)
    finally:
        ad.set_launch("algdist", dt, K, lanes_per_row=0)
    assert ad.status(clear=True) == 0


def _scan_sizes(best_rel, gamma, tol=1e-6):
    """The penalty scan on given relative best values; returns (size,
    near) where near says some comparison was within tol of its threshold."""
    inc_m, inc_v, near = 0, None, False
    for m in range(1, len(best_rel)):
        v = best_rel[m]
        if v < 0:
            continue
        if inc_m == 0:
            inc_m, inc_v = m, v
            continue
        thr = inc_v ** (gamma * (m - inc_m))
        if thr > 0 and abs(v / thr - 1.0) < tol:
            near = True
        if v < thr:
            inc_m, inc_v = m, v
    return inc_m, near


def check_search(A, G, x, w, cf, cal, gamma, target, got, dt, rows=None, Gp=None):
    """GPU search results `got` against the oracle (see the module doc), on
    every row or on the given rows."""
    if Gp is None:
        Gp = oracle.Pattern(A.n, to_np(G.row_ptr), to_np(G.col))
    tg = oracle.TARGET_PLAIN if target == "plain" else oracle.TARGET_RESIDUAL
    Rc, Rv, Rl, Rs, best, nc = oracle.ls_search(A, Gp, x, w, cf, cal, gamma, tg, rows=rows)
    Pc, Pv, ls, st = (to_np(t) for t in got)
    ids = np.arange(A.n) if rows is None else np.asarray(rows)
    Pc, Pv, ls, st, cfr = Pc[ids], Pv[ids], ls[ids], st[ids], cf[ids]
    assert np.array_equal(st, Rs), "status differ at %s" % ids[np.nonzero(st != Rs)[0][:5]]
    same = np.all(Pc == Rc, axis=1)
    diff_rows = np.nonzero(~same)[0]
    say("  rows %d, F rows %d, sets differ in %d rows; candidates %d..%d"
        % (len(ids), int((cfr == 0).sum()), len(diff_rows), nc.min(), nc.max()))
    S = best[:, 0]
    for q in diff_rows:
        i = ids[q]
        assert cfr[q] == 0
        mine = [c for c in Pc[q] if c >= 0]
        m_g = len(mine)
        assert m_g >= 1
        pv, lv, rd = oracle.ls_fit_sets(A, x, w, np.array([list(Pc[q])]), [i], tg)
        assert rd[0] == 0
        rel = lv[0] / S[q] if S[q] > 0 else 0.0
        # a (near-)best set of its size ...
        assert rel <= best[q, m_g] * (1 + 1e-7) + 1e-13, (i, rel, best[q, m_g])
        # ... and a size the penalty scan reaches within rounding
        m_o, near = _scan_sizes(list(best[q]), gamma)
        assert m_g == m_o or near, (i, m_g, m_o)
    assert len(diff_rows) <= max(2, 0.002 * len(ids))
    ok = same & (cfr == 0)
    perr = np.abs(Pv - Rv)[ok] / np.maximum(1.0, np.abs(Rv[ok]))
    assert np.all(perr <= 1e-6), perr.max()
    lerr = np.abs(ls - Rl)[ok]
    assert np.all(lerr <= 1e-6 * np.abs(Rl[ok]) + 1e-12 * S[ok]), lerr.max()
    c = cfr != 0
    assert np.all(Pc[c, 0] == ids[c]) and np.all(Pv[c, 0] == 1.0)
    return nc


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("target", ["plain", "residual"])
@pytest.mark.parametrize("d, cal", [(1, 4), (2, 2), (2, 3), (2, 4), (3, 2)])
def test_search_matches_the_oracle(dt, target, d, cal):
    ad = lib()
    N, K = 23, 16
    A = W.rotated_anisotropic_9pt(N, 1e-3, math.pi / 6)
    if dt == torch.float32:
        A = W.CSR(A.n, A.row_ptr, A.col, A.val.astype(np.float32).astype(np.float64))
    Ad = dev_csr(A, dt)
    color = torch.as_tensor(W.red_black((N, N)), device="cuda")
    X = ad.setup_testvectors(Ad, K, seed=4, relax="gs", sweeps=4, color=color, ncolors=2)
    x = to_np(X).astype(np.float64)
    cf = W.cf_red_is_coarse((N, N))
    G = ad.power_graph(Ad, d)
    say("search: %s %s d=%d caliber=%d" % (dt, target, d, cal))
    got = ad.ls_interp_search(Ad, G, X, torch.as_tensor(cf, device="cuda"), cal, 1.5,
                              target=target)
    check_search(A, G, x, None, cf, cal, 1.5, target, got, dt)
    assert ad.status(clear=True) == 0


@pytest.mark.parametrize("target", ["residual", "plain"])
def test_search_near_exact_fits(target):
    """The setup of the two-grid tables on the 7-point operator with eps
    1e-4, alpha pi/4 on 64^2: 8 test vectors of 40 Gauss-Seidel sweeps, CR
    on the strength graph M^2, the search over the C points of A^4.  Near
    the corners the vectors are nearly of low rank: sets of 4 fit the
    target to about 1e-20 of its squared norm, and sets of nearly dependent
    rows fit it through cancelling weights.  The search still agrees with
    the oracle, its weights stay moderate, and the Galerkin operator is
    positive definite (the two-grid cycle runs)."""
    ad = lib()
    N = 64
    A = W.rotated_anisotropic_7pt(N, 1e-4, math.pi / 4)
    Ad = dev_csr(A, torch.float64)
    color = torch.as_tensor(W.four_colour_2d(N), device="cuda")
    X = ad.setup_testvectors(Ad, 8, seed=3, relax="gs", sweeps=40, color=color, ncolors=4)
    G2 = ad.power_graph(Ad, 2)
    mu2 = ad.algebraic_distance_graph(Ad, G2, X)
    cf, _, _ = ad.cr_coarsening(Ad, color, 4, mu2, 0.5, seed=1, G=G2)
    G4 = ad.power_graph(Ad, 4)
    say("search on A^4 after CR on M^2, eps 1e-4, alpha pi/4, 64^2, %s target" % target)
    got = ad.ls_interp_search(Ad, G4, X, cf, 4, 1.5, target=target)
    check_search(A, G4, to_np(X), None, to_np(cf), 4, 1.5, target, got, torch.float64)
    Pc, Pv, _, _ = got
    assert float(Pv.abs().max()) < 1e3
    Ac = ad.galerkin(Ad, Pc, Pv, cf)
    E0 = torch.rand((A.n, 2), dtype=torch.float64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(5)) * 2 - 1
    rho, _ = ad.two_grid_rate(Ad, color, 4, Pc, Pv, cf, Ac, E0, iters=10)
    assert all(0.0 <= float(r) < 1.0 for r in rho)
    assert ad.status(clear=True) == 0


@pytest.mark.parametrize("gamma", [1.0, 1.5, 3.0])
def test_search_weights_gamma_and_graph_rows(gamma):
    """Weighted functional, other gammas, a random graph with a random C/F
    split and rows of uneven candidate counts."""
    ad = lib()
    A = W.rgg_laplacian(900, 6.0, 21)
    K = 8
    Ad = dev_csr(A, torch.float64)
    X = ad.setup_testvectors(Ad, K, seed=3, relax="jacobi", sweeps=3, omega=0.7)
    x = to_np(X)
    rng = np.random.default_rng(7)
    cf = (rng.random(A.n) < 0.4).astype(np.uint8)
    w = 0.5 + rng.random(K)
    G = ad.power_graph(Ad, 2)
    got = ad.ls_interp_search(Ad, G, X, torch.as_tensor(cf, device="cuda"), 3, gamma,
                              w=torch.as_tensor(w, device="cuda"))
    check_search(A, G, x, w, cf, 3, gamma, "plain", got, torch.float64)
    assert ad.status(clear=True) == 0


@pytest.mark.parametrize("dt,target,d,cal", [(torch.float64, "plain", 4, 2),
                                             (torch.float32, "residual", 4, 3),
                                             (torch.float64, "residual", 5, 2),
                                             (torch.float32, "plain", 6, 2)])
def test_search_rows_past_the_first_pass(dt, target, d, cal):
    """Rows with 33 to 64 candidates are searched by the second pass: an
    interior F row of the 9-point operator has 2d(d + 1) C-points in the
    pattern of A^d (40, 60 and 84 for d = 4, 5, 6); rows near the boundary
    have fewer and stay in the first pass, and A^6's interior rows, past
    64, are left empty with status 4."""
    ad = lib()
    N, K = 17, 16
    A = W.rotated_anisotropic_9pt(N, 1e-3, math.pi / 6)
    if dt == torch.float32:
        A = W.CSR(A.n, A.row_ptr, A.col, A.val.astype(np.float32).astype(np.float64))
    Ad = dev_csr(A, dt)
    color = torch.as_tensor(W.red_black((N, N)), device="cuda")
    X = ad.setup_testvectors(Ad, K, seed=6, relax="gs", sweeps=4, color=color, ncolors=2)
    x = to_np(X).astype(np.float64)
    cf = W.cf_red_is_coarse((N, N))
    G = ad.power_graph(Ad, d)
    say("search past the first pass: %s %s d=%d caliber=%d" % (dt, target, d, cal))
    got = ad.ls_interp_search(Ad, G, X, torch.as_tensor(cf, device="cuda"), cal, 1.5,
                              target=target)
    rp, col = to_np(G.row_ptr), to_np(G.col)
    rid = np.repeat(np.arange(A.n), np.diff(rp))
    nc = np.bincount(rid, weights=(cf[col] != 0) & (col != rid), minlength=A.n).astype(int)
    F = cf == 0
    assert np.any((nc[F] > 32) & (nc[F] <= 64)) and np.any((nc[F] <= 32) & (nc[F] > 0))
    assert nc[F].max() == {4: 40, 5: 60, 6: 84}[d]
    # rows past the cap: empty, status 4, functional of the empty set
    over = np.nonzero(F & (nc > 64))[0]
    Pc, _, ls, st = (to_np(t) for t in got)
    assert np.all(st[over] == 4) and np.all(Pc[over] == -1)
    T = x if target == "plain" else None
    if T is not None:
        assert np.allclose(ls[over], (T[over] * T[over]).sum(1), rtol=1e-12, atol=0)
    assert bool(ad.status(clear=True) & ad.STAT_SEARCH_CAP) == (len(over) > 0)
    rows = np.nonzero(~(F & (nc > 64)))[0].astype(np.int32)
    check_search(A, G, x, None, cf, cal, 1.5, target, got, dt, rows=rows)


def test_search_full_size_sampled():
    """The bench's long-range configuration: the 2048^2 anisotropic 9-point
    operator in FP32, test vectors from 5 colour-phase sweeps, the pattern
    of A^2 (every row against the oracle's), caliber 4, gamma 1.5; 2048
    sampled rows of the search against the oracle."""
    ad = lib()
    ad.status(clear=True)
    wl = W.workload(2, "f32")
    A = wl.A
    Ad = dev_csr(A, torch.float32)
    color = torch.as_tensor(wl.color, device="cuda")
    X = ad.setup_testvectors(Ad, wl.K, seed=wl.tv_seed, relax="gs", sweeps=wl.sweeps,
                             color=color, ncolors=wl.ncolors)
    G = ad.power_graph(Ad, 2)
    say("search full size: n %d, pattern entries %d" % (A.n, G.nnz))
    R = oracle.power_pattern(A, 2)
    assert np.array_equal(to_np(G.row_ptr), R.row_ptr) and np.array_equal(to_np(G.col), R.col)
    got = ad.ls_interp_search(Ad, G, X, torch.as_tensor(wl.cf, device="cuda"), 4, 1.5)
    rng = np.random.default_rng(5)
    rows = np.unique(np.concatenate([rng.choice(A.n, 2048, replace=False), [0, 1, A.n - 1]]))
    rows = rows.astype(np.int32)
    Gp = oracle.Pattern(A.n, to_np(G.row_ptr), to_np(G.col))
    check_search(A, G, to_np(X).astype(np.float64), None, wl.cf, 4, 1.5, "plain", got,
                 torch.float32, rows=rows, Gp=Gp)
    assert np.all(to_np(got[3]) == 0)
    assert ad.status(clear=True) == 0


def test_search_follows_the_knight_move_anisotropy():
    """tan(alpha) = 1/2 on a 64^2 grid, test vectors by 40 colour-phase GS
    sweeps on the GPU, C = red, search depth 2: most interior F points pick
    their two C-neighbours at +-(2, 1), and the rows match the oracle."""
    ad = lib()
    N, K = 64, 8
    A = W.rotated_anisotropic_9pt(N, 1e-3, math.atan(0.5))
    Ad = dev_csr(A, torch.float64)
    color = torch.as_tensor(W.red_black((N, N)), device="cuda")
    X = ad.setup_testvectors(Ad, K, seed=11, relax="gs", sweeps=40, color=color, ncolors=2)
    cf = W.cf_red_is_coarse((N, N))
    G = ad.power_graph(Ad, 2)
    got = ad.ls_interp_search(Ad, G, X, torch.as_tensor(cf, device="cuda"), 2, 1.5)
    check_search(A, G, to_np(X), None, cf, 2, 1.5, "plain", got, torch.float64)
    Pc = to_np(got[0])
    iy, ix = np.divmod(np.arange(A.n), N)
    inner = (ix > 2) & (ix < N - 3) & (iy > 2) & (iy < N - 3) & (cf == 0)
    rows = np.nonzero(inner)[0]
    hit = sum(sorted(int(c) - int(i) for c in Pc[i] if c >= 0) == [-(N + 2), N + 2] for i in rows)
    say("  knight-move sets: %d of %d interior F rows" % (hit, len(rows)))
    assert hit >= 0.8 * len(rows)
    assert ad.status(clear=True) == 0


def test_search_candidate_cap_and_errors():
    """An F row with more than 64 candidates gets status 4, an empty row and
    the sticky bit; caliber 5 and caliber > K are refused."""
    ad = lib()
    N, K = 21, 8
    A = W.rotated_anisotropic_9pt(N, 1e-3, 0.3)
    Ad = dev_csr(A, torch.float64)
    X = ad.setup_testvectors(Ad, K, seed=1, relax="jacobi", sweeps=1, omega=0.7)
    cf = np.ones(A.n, dtype=np.uint8)
    c = (N // 2) * N + N // 2
    cf[c] = 0
    G = ad.power_graph(Ad, 4)  # 81 entries, 80 of them C
    Pc, Pv, ls, st = ad.ls_interp_search(Ad, G, X, torch.as_tensor(cf, device="cuda"), 2)
    assert to_np(st)[c] == 4 and np.all(to_np(Pc)[c] == -1)
    x = to_np(X)
    assert to_np(ls)[c] == pytest.approx(float((x[c] * x[c]).sum()), rel=1e-12)
    assert ad.status(clear=True) & ad.STAT_SEARCH_CAP
    cft = torch.as_tensor(cf, device="cuda")
    with pytest.raises(ad.AlgdistError, match="AD_ECALIBER"):
        ad.ls_interp_search(Ad, G, X, cft, 5)
    X2 = ad.setup_testvectors(Ad, 2, seed=1)
    with pytest.raises(ad.AlgdistError, match="AD_ECALIBER"):
        ad.ls_interp_search(Ad, G, X2, cft, 3)
    assert ad.status(clear=True) == 0
