"""GPU parity of every step against the CPU oracle, at sizes the oracle
finishes in seconds that still span many tiles and a ragged tail, plus the
edge cases (empty input, diagonal-only rows, zero diagonals, bad colours,
duplicate interpolation columns, rows without C-neighbours, every K).
All calls go through the C ABI (paper_1106_5990_amd.algdist)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1106_5990_amd import workloads as W
from gpu_common import (check_ls, check_mu, dev_csr, lib, residual_target, row_abs_bound,
                        saa_per_edge, say, to_np)

pytestmark = pytest.mark.gpu

DT = {"f32": torch.float32, "f64": torch.float64}


def host_vals(A, dt):
    """The operator values as the GPU path of type dt sees them, in FP64."""
    return A.val.astype(np.float32).astype(np.float64) if dt == torch.float32 else A.val


def as_oracle(A, dt):
    return W.CSR(A.n, A.row_ptr, A.col, host_vals(A, dt))


def aniso(N, alpha=math.pi / 6, eps=1e-3):
    return W.rotated_anisotropic_9pt(N, eps, alpha)


# ------------------------------------------------------------------ start
@pytest.mark.parametrize("n,K", [(1000, 8), (1001, 2), (37, 64), (513, 16)])
def test_tv_init_bitwise(n, K):
    say("tv_init n=%d K=%d" % (n, K))
    ad = lib()
    A = W.laplacian_2d_5pt(1)  # any matrix: the start depends only on (i, k, seed)
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.arange(1, n + 1)
    A = W.CSR(n, rp, np.arange(n, dtype=np.int32), np.ones(n))
    want = oracle.tv_init(n, K, 1234)
    for dt in (torch.float64, torch.float32):
        X = ad.setup_testvectors(dev_csr(A, dt), K, seed=1234, sweeps=0)
        got = to_np(X)
        if dt == torch.float64:
            assert np.array_equal(got, want)
        else:
            assert np.array_equal(got, want.astype(np.float32))


# ------------------------------------------------------------------ relaxation
@pytest.mark.parametrize("K", [2, 8, 16, 32, 64])
def test_jacobi_fp64_matches_oracle(K):
    say("jacobi f64 K=%d" % K)
    ad = lib()
    A = aniso(45)  # 2025 rows: ragged against every tile size
    X = ad.setup_testvectors(dev_csr(A, torch.float64), K, seed=7, relax="jacobi", sweeps=4,
                             omega=0.8)
    want, _ = oracle.jacobi(A, oracle.tv_init(A.n, K, 7), 0.8, 4)
    got = to_np(X)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("K", [4, 16, 32])
def test_jacobi_fp32_one_sweep_bound(K):
    say("jacobi f32 K=%d" % K)
    ad = lib()
    A = W.lognormal_3d_7pt(13, 2.0, 3)  # 2197 rows, coefficient jumps
    A32 = as_oracle(A, torch.float32)
    Ad = dev_csr(A, torch.float32)
    X1 = ad.setup_testvectors(Ad, K, seed=5, relax="jacobi", sweeps=1, omega=0.8)
    X2 = ad.setup_testvectors(Ad, K, X0=X1, relax="jacobi", sweeps=1, omega=0.8)
    x1 = to_np(X1).astype(np.float64)
    want = oracle.jacobi_rows(A32, x1, 0.8, np.arange(A.n))
    bound = row_abs_bound(A32, x1, x1, 0.8)
    err = np.abs(to_np(X2) - want)
    say("  max err/bound %.3g" % np.max(err / bound))
    assert np.all(err <= bound)
    # the first sweep from the hashed start as well
    x0 = oracle.tv_init(A.n, K, 5).astype(np.float32).astype(np.float64)
    want1 = oracle.jacobi_rows(A32, x0, 0.8, np.arange(A.n))
    assert np.all(np.abs(x1 - want1) <= row_abs_bound(A32, x0, x0, 0.8))


@pytest.mark.parametrize("ncol,K", [(2, 16), (4, 8), (3, 32)])
def test_colour_gs_fp64_matches_oracle(ncol, K):
    say("gs f64 ncolors=%d K=%d" % (ncol, K))
    ad = lib()
    N = 47
    A = aniso(N)
    if ncol == 2:
        color = W.red_black((N, N))
    elif ncol == 4:
        color = W.four_colour_2d(N)
    else:
        color = (np.arange(N * N) % 3).astype(np.int32)
    X = ad.setup_testvectors(dev_csr(A, torch.float64), K, seed=9, relax="gs", sweeps=5,
                             color=torch.as_tensor(color, device="cuda"), ncolors=ncol)
    want, held = oracle.color_gs(A, oracle.tv_init(A.n, K, 9), color, ncol, 5)
    assert held == 0
    got = to_np(X)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    assert ad.status(clear=True) == 0


@pytest.mark.parametrize("ncol,used,N", [(64, 64, 101), (5, 2, 73), (7, 7, 9)])
def test_colour_gs_random_colouring_partition(ncol, used, N):
    """Random colours (up to the maximum of 64, some classes absent, a few
    invalid) over several partition blocks with a ragged tail: the colour
    phases against the oracle."""
    say("gs f64 random colours ncolors=%d used=%d n=%d" % (ncol, used, N * N))
    ad = lib()
    K = 8
    A = aniso(N)
    rng = np.random.default_rng(ncol * 1000 + used)
    pal = np.sort(rng.choice(ncol, used, replace=False)).astype(np.int32)
    color = pal[rng.integers(0, used, A.n)].astype(np.int32)
    bad = rng.choice(A.n, max(1, A.n // 500), replace=False)
    color[bad] = np.where(np.arange(bad.size) % 2 == 0, -3, ncol + 1)
    ad.status(clear=True)
    X = ad.setup_testvectors(dev_csr(A, torch.float64), K, seed=31, relax="gs", sweeps=2,
                             color=torch.as_tensor(color, device="cuda"), ncolors=ncol)
    want, held = oracle.color_gs(A, oracle.tv_init(A.n, K, 31), color, ncol, 2)
    assert held == bad.size
    got = to_np(X)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    assert ad.status(clear=True) & ad.STAT_BAD_COLOR  # the invalid colours are reported


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_relaxation_with_unaligned_csr_arrays(dt):
    """Column and value arrays that are not 16-byte aligned take the
    entry-by-entry staging copy: Jacobi sweeps (single matrix and batch)
    bitwise equal to the aligned arrays' result."""
    say("unaligned CSR arrays %s" % dt)
    ad = lib()
    dtype = DT[dt]
    A = aniso(37)
    Ad = dev_csr(A, dtype)
    col = torch.empty(A.nnz + 1, dtype=torch.int32, device="cuda")
    val = torch.empty(A.nnz + 1, dtype=dtype, device="cuda")
    col[1:] = Ad.col
    val[1:] = Ad.val
    Au = ad.Csr(Ad.row_ptr, col[1:], val[1:])
    assert Au.col.data_ptr() % 16 != 0 and Au.val.data_ptr() % 16 != 0
    for K in (16, 8):
        Xa = ad.setup_testvectors(Ad, K, seed=4, relax="jacobi", sweeps=3, omega=0.7)
        Xu = ad.setup_testvectors(Au, K, seed=4, relax="jacobi", sweeps=3, omega=0.7)
        assert torch.equal(Xa, Xu), K
    ga = ad.relax_algdist_batched([Ad, Ad], 16, seed=4, sweeps=3, omega=0.7, theta=0.25)
    gu = ad.relax_algdist_batched([Ad, Au], 16, seed=4, sweeps=3, omega=0.7, theta=0.25)
    for a, b in zip(ga, gu):
        assert torch.equal(a, b)
    assert ad.status(clear=True) == 0


def test_colour_gs_fp32_one_sweep_bound():
    say("gs f32 one sweep")
    ad = lib()
    N, K = 61, 16
    A = aniso(N)
    A32 = as_oracle(A, torch.float32)
    Ad = dev_csr(A, torch.float32)
    color = W.red_black((N, N))
    ct = torch.as_tensor(color, device="cuda")
    X3 = ad.setup_testvectors(Ad, K, seed=3, relax="gs", sweeps=3, color=ct, ncolors=2)
    X4 = ad.setup_testvectors(Ad, K, X0=X3, relax="gs", sweeps=1, color=ct, ncolors=2)
    x3, x4 = to_np(X3).astype(np.float64), to_np(X4).astype(np.float64)
    rows = np.arange(A.n)
    want = oracle.color_gs_rows(A32, color, 2, x3, x4, rows)
    # z_j: new values for red neighbours of black rows, old otherwise
    Z = np.where((color == 0)[:, None], x4, x3)
    bound = np.maximum(row_abs_bound(A32, Z, x3, 1.0), row_abs_bound(A32, x3, x3, 1.0))
    err = np.abs(x4 - want)
    say("  max err/bound %.3g" % np.max(err / bound))
    assert np.all(err <= bound)


def test_held_rows_zero_diagonal_and_bad_colour():
    say("held rows")
    ad = lib()
    N, K = 20, 8
    A = aniso(N)
    val = A.val.copy()
    i0 = 77
    val[A.row_ptr[i0]:A.row_ptr[i0 + 1]][A.col[A.row_ptr[i0]:A.row_ptr[i0 + 1]] == i0] = 0.0
    A = W.CSR(A.n, A.row_ptr, A.col, val)
    color = W.red_black((N, N)).copy()
    color[5] = 9
    color[300] = -1
    X0 = oracle.tv_init(A.n, K, 2)
    ad.status(clear=True)
    X = ad.setup_testvectors(dev_csr(A, torch.float64), K, seed=2, relax="gs", sweeps=3,
                             color=torch.as_tensor(color, device="cuda"), ncolors=2)
    want, held = oracle.color_gs(A, X0, color, 2, 3)
    assert held == 3
    got = to_np(X)
    for r in (i0, 5, 300):
        assert np.array_equal(got[r], X0[r])
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    bits = ad.status(clear=True)
    assert bits & ad.STAT_ZERO_DIAG and bits & ad.STAT_BAD_COLOR
    Xj = ad.setup_testvectors(dev_csr(A, torch.float64), K, seed=2, relax="jacobi", sweeps=2,
                              omega=0.7)
    wantj, z = oracle.jacobi(A, X0, 0.7, 2)
    assert z == 1 and np.max(np.abs(to_np(Xj) - wantj)) <= 1e-12 * np.max(np.abs(wantj))
    assert ad.status(clear=True) == ad.STAT_ZERO_DIAG


@pytest.mark.parametrize("every,sweeps", [(2, 6), (1, 3), (4, 5), (3, 0)])
def test_checkpoints_hold_the_iterates(every, sweeps):
    say("ckpt every=%d sweeps=%d" % (every, sweeps))
    ad = lib()
    A = W.lognormal_2d_5pt(33, 1.0, 1)
    Ad = dev_csr(A, torch.float64)
    K = 16
    nck = max(1, -(-sweeps // every))
    ck = torch.empty((nck, A.n, K), dtype=torch.float64, device="cuda")
    X = ad.setup_testvectors(Ad, K, seed=4, relax="jacobi", sweeps=sweeps, omega=0.6, ckpt=ck,
                             ckpt_every=every)
    for q in range(nck):
        s = q * every
        ref = ad.setup_testvectors(Ad, K, seed=4, relax="jacobi", sweeps=s, omega=0.6)
        assert torch.equal(ck[q], ref), "checkpoint %d" % q
    ref = ad.setup_testvectors(Ad, K, seed=4, relax="jacobi", sweeps=sweeps, omega=0.6)
    assert torch.equal(X, ref)


def test_user_start_and_empty_matrix():
    say("user start / empty")
    ad = lib()
    A = W.laplacian_2d_5pt(9)
    K = 4
    X0 = torch.as_tensor(oracle.tv_init(A.n, K, 77) * 3.0, device="cuda")
    X = ad.setup_testvectors(dev_csr(A, torch.float64), K, X0=X0, relax="jacobi", sweeps=2,
                             omega=0.5)
    want, _ = oracle.jacobi(A, to_np(X0), 0.5, 2)
    assert np.max(np.abs(to_np(X) - want)) <= 1e-13
    E = W.CSR(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    Ed = dev_csr(E, torch.float64)
    X = ad.setup_testvectors(Ed, K, seed=1, sweeps=3)
    assert X.shape == (0, K)
    mu = ad.algebraic_distance(Ed, X)
    assert mu.numel() == 0
    s, ns = ad.strength_graph(Ed, mu, 0.25)
    Pc, Pv, ls, st, tot = ad.ls_interp(Ed, X, torch.zeros(0, dtype=torch.uint8, device="cuda"), mu,
                                       2, want_sum=True)
    assert float(tot) == 0.0


# ------------------------------------------------------------------ distances
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("target", ["plain", "residual"])
@pytest.mark.parametrize("K,weighted", [(8, False), (16, True), (32, False), (2, True), (64, True)])
def test_algdist_matches_oracle(dt, target, K, weighted):
    say("algdist %s %s K=%d w=%s" % (dt, target, K, weighted))
    ad = lib()
    dtype = DT[dt]
    N = 41
    A = aniso(N)
    Ao = as_oracle(A, dtype)
    Ad = dev_csr(A, dtype)
    color = torch.as_tensor(W.red_black((N, N)), device="cuda")
    X = ad.setup_testvectors(Ad, K, seed=11, relax="gs", sweeps=4, color=color, ncolors=2)
    w = (0.5 + np.random.default_rng(K).random(K)) if weighted else None
    wt = None if w is None else torch.as_tensor(w, device="cuda")
    mu, p = ad.algebraic_distance(Ad, X, w=wt, target=target, want_p=True)
    x = to_np(X).astype(np.float64)
    tg = oracle.TARGET_PLAIN if target == "plain" else oracle.TARGET_RESIDUAL
    mu_ref, p_ref, bad = oracle.algdist(Ao, x, w, tg, want_p=True)
    assert bad == 0
    T = x if target == "plain" else residual_target(Ao, x)
    check_mu(to_np(mu).astype(np.float64), mu_ref, saa_per_edge(Ao, T, w), dtype)
    # p is the minimiser; compare where the problem is well posed
    pg = to_np(p)
    assert np.all(np.abs(pg - p_ref) <= (1e-3 if dt == "f32" else 1e-10) * np.maximum(1, np.abs(p_ref)))
    # diagonal distances of the plain target are exactly zero
    if target == "plain":
        diag = A.col == A.row_ids()
        assert np.all(to_np(mu)[diag] == 0)
    assert ad.status(clear=True) == 0


def coo_csr(n, i, j, v, diag):
    """CSR from off-diagonal pairs (both orientations given) plus a diagonal."""
    i = np.concatenate([i, np.arange(n)])
    j = np.concatenate([j, np.arange(n)])
    v = np.concatenate([v, diag])
    o = np.lexsort((j, i))
    i, j, v = i[o], j[o], v[o]
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(i, minlength=n), out=rp[1:])
    return W.CSR(n, rp.astype(np.int32), j.astype(np.int32), v)


def irregular(n, seed):
    """Random geometric graph plus one hub row joined to a fifth of the nodes
    (a row spanning several 64-entry chunks) and a few isolated nodes (rows
    with only the diagonal)."""
    B = W.rgg_laplacian(n, 25.0, seed)
    rid = B.row_ids()
    off = B.col != rid
    i, j, v = rid[off], B.col[off], B.val[off]
    rng = np.random.default_rng(seed)
    hub = n // 3
    nb = rng.choice(np.setdiff1d(np.arange(n), [hub]), n // 5, replace=False)
    keep = (i != hub) & (j != hub)
    iso = rng.choice(n, 5, replace=False)
    keep &= ~np.isin(i, iso) & ~np.isin(j, iso)
    w = -(0.1 + rng.random(len(nb)))
    i = np.concatenate([i[keep], np.full(len(nb), hub), nb])
    j = np.concatenate([j[keep], nb, np.full(len(nb), hub)])
    v = np.concatenate([v[keep], w, w])
    deg = np.zeros(n)
    np.add.at(deg, i, -v)
    return coo_csr(n, i, j, v, deg + 1e-3)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("weighted", [False, True])
def test_edge_parallel_distances_irregular_rows(dt, weighted):
    """The edge-parallel kernel (default shape, plain target) and the
    row-group kernel against the oracle on rows of very uneven length: mu,
    p, the fused strength row with and without an F mask."""
    say("edge-parallel distances %s weighted=%s" % (dt, weighted))
    ad = lib()
    dtype = DT[dt]
    K = 16
    A = irregular(3000, 17)
    Ao = as_oracle(A, dtype)
    Ad = dev_csr(A, dtype)
    X = ad.setup_testvectors(Ad, K, seed=5, relax="jacobi", sweeps=3, omega=0.7)
    x = to_np(X).astype(np.float64)
    w = (0.5 + np.random.default_rng(3).random(K)) if weighted else None
    wt = None if w is None else torch.as_tensor(w, device="cuda")
    fm = (np.random.default_rng(4).random(A.n) < 0.6).astype(np.uint8)
    fmt = torch.as_tensor(fm, device="cuda")
    mu_ref, p_ref, bad = oracle.algdist(Ao, x, w, oracle.TARGET_PLAIN, want_p=True)
    saa = saa_per_edge(Ao, x, w)
    try:
        for lpr in (0, 2):
            ad.set_launch("algdist", dtype, K, lpr, 1, True)
            mu, p = ad.algebraic_distance(Ad, X, w=wt, want_p=True)
            check_mu(to_np(mu).astype(np.float64), mu_ref, saa, dtype, "lpr %d" % lpr)
            pg = to_np(p)
            assert np.all(np.abs(pg - p_ref) <= (1e-3 if dt == "f32" else 1e-10)
                          * np.maximum(1, np.abs(p_ref))), lpr
            for fmask, fmh in ((None, None), (fmt, fm)):
                mu2, s, ns = ad.algebraic_distance(Ad, X, w=wt, fuse=True, theta=0.3, fmask=fmask)
                assert torch.equal(mu2, mu), lpr
                sr, nsr = oracle.strength(A, to_np(mu).astype(np.float64), 0.3, fmh)
                assert np.array_equal(to_np(s), sr) and np.array_equal(to_np(ns), nsr), lpr
    finally:
        ad.set_launch("algdist", dtype, K, 0, 1, True)
    assert ad.status(clear=True) == 0


@pytest.mark.parametrize("n", [1, 63, 64, 65, 257])
def test_edge_parallel_distances_small_and_ragged(n):
    say("edge-parallel distances n=%d" % n)
    ad = lib()
    K = 8
    i = np.arange(n - 1)
    A = coo_csr(n, np.concatenate([i, i + 1]), np.concatenate([i + 1, i]),
                -np.ones(2 * (n - 1)), np.full(n, 2.5))
    for dtype in (torch.float32, torch.float64):
        Ad = dev_csr(A, dtype)
        X = ad.setup_testvectors(Ad, K, seed=n, relax="jacobi", sweeps=2, omega=0.6)
        x = to_np(X).astype(np.float64)
        mu, s, ns = ad.algebraic_distance(Ad, X, fuse=True, theta=0.25)
        check_mu(to_np(mu).astype(np.float64), oracle.algdist(as_oracle(A, dtype), x),
                 saa_per_edge(A, x), dtype)
        sr, nsr = oracle.strength(A, to_np(mu).astype(np.float64), 0.25)
        assert np.array_equal(to_np(s), sr) and np.array_equal(to_np(ns), nsr)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_algdist_exact_zero_for_proportional_vectors(dt):
    say("algdist exact zeros %s" % dt)
    ad = lib()
    dtype = DT[dt]
    n, K = 300, 16
    A = W.laplacian_2d_5pt(1)
    rng = np.random.default_rng(1)
    # tridiagonal chain: x_{i+1} = 2^m x_i
    rp = np.zeros(n + 1, np.int32)
    cols = []
    for i in range(n):
        cols.extend([j for j in (i - 1, i, i + 1) if 0 <= j < n])
        rp[i + 1] = len(cols)
    A = W.CSR(n, rp, np.array(cols, np.int32), np.where(
        np.array(cols) == np.repeat(np.arange(n), np.diff(rp)), 4.0, -1.0))
    base = rng.standard_normal(K)
    X = np.stack([base * 2.0 ** (int(i % 7) - 3) for i in range(n)])
    Xt = torch.as_tensor(X, dtype=dtype, device="cuda")
    mu = to_np(ad.algebraic_distance(dev_csr(A, dtype), Xt))
    assert np.all(mu == 0.0)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("use_fmask", [False, True])
def test_fused_and_standalone_strength_bit_exact(dt, use_fmask):
    say("strength %s fmask=%s" % (dt, use_fmask))
    ad = lib()
    dtype = DT[dt]
    N, K = 53, 16
    A = aniso(N)
    Ad = dev_csr(A, dtype)
    color = torch.as_tensor(W.red_black((N, N)), device="cuda")
    X = ad.setup_testvectors(Ad, K, seed=13, relax="gs", sweeps=5, color=color, ncolors=2)
    fm = (np.random.default_rng(2).random(A.n) < 0.7).astype(np.uint8) if use_fmask else None
    fmt = None if fm is None else torch.as_tensor(fm, device="cuda")
    mu, strong, ns = ad.algebraic_distance(Ad, X, fuse=True, theta=0.25, fmask=fmt)
    mu_h = to_np(mu).astype(np.float64)
    s_ref, ns_ref = oracle.strength(A, mu_h, 0.25, fm)
    assert np.array_equal(to_np(strong), s_ref)
    assert np.array_equal(to_np(ns), ns_ref)
    s2, ns2 = ad.strength_graph(Ad, mu, 0.25, fmask=fmt)
    assert np.array_equal(to_np(s2), s_ref) and np.array_equal(to_np(ns2), ns_ref)
    # theta sweep on the standalone kernel
    for th in (0.05, 0.5, 0.9):
        s3, n3 = ad.strength_graph(Ad, mu, th, fmask=fmt)
        r3, rn3 = oracle.strength(A, mu_h, th, fm)
        assert np.array_equal(to_np(s3), r3) and np.array_equal(to_np(n3), rn3)


def test_strength_zero_distance_rows():
    say("strength zero-distance rows")
    ad = lib()
    A = aniso(12)
    rng = np.random.default_rng(5)
    mu = rng.random(A.nnz) + 0.1
    mu[rng.random(A.nnz) < 0.2] = 0.0
    for dt in (torch.float64, torch.float32):
        mt = torch.as_tensor(mu, dtype=dt, device="cuda")
        s, ns = ad.strength_graph(dev_csr(A, dt), mt, 0.25)
        r, rn = oracle.strength(A, to_np(mt).astype(np.float64), 0.25)
        assert np.array_equal(to_np(s), r) and np.array_equal(to_np(ns), rn)


# ------------------------------------------------------------------ LS interpolation
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("target", ["plain", "residual"])
@pytest.mark.parametrize("K,cal", [(8, 4), (16, 4), (8, 8), (32, 3), (4, 2), (64, 6), (2, 1)])
def test_ls_interp_matches_oracle(dt, target, K, cal):
    say("ls_interp %s %s K=%d cal=%d" % (dt, target, K, cal))
    ad = lib()
    dtype = DT[dt]
    N = 43
    A = aniso(N)
    Ao = as_oracle(A, dtype)
    Ad = dev_csr(A, dtype)
    color = torch.as_tensor(W.red_black((N, N)), device="cuda")
    X = ad.setup_testvectors(Ad, K, seed=17, relax="gs", sweeps=3, color=color, ncolors=2)
    w = 0.5 + np.random.default_rng(cal).random(K)
    wt = torch.as_tensor(w, device="cuda")
    mu = ad.algebraic_distance(Ad, X, w=wt)
    # C points: a random 40% (rows with 0..8 C-neighbours, some with none)
    cf = (np.random.default_rng(3).random(A.n) < 0.4).astype(np.uint8)
    cft = torch.as_tensor(cf, device="cuda")
    Pc, Pv, ls, st, tot = ad.ls_interp(Ad, X, cft, mu, cal, w=wt, target=target, want_sum=True)
    x = to_np(X).astype(np.float64)
    tg = oracle.TARGET_PLAIN if target == "plain" else oracle.TARGET_RESIDUAL
    ref = oracle.ls_interp(Ao, x, w, cf, to_np(mu).astype(np.float64), cal, tg)
    T = x if target == "plain" else residual_target(Ao, x)
    wtt = (T * T * w).sum(1)
    check_ls((to_np(Pc), to_np(Pv), to_np(ls), to_np(st)), ref, dtype, wtt)
    assert np.any(ref[3] == 1)  # some F rows have no C-neighbour
    # the F-row sum
    lsn = to_np(ls)
    assert abs(float(tot) - lsn[cf == 0].sum()) <= 1e-12 * lsn.sum()


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_ls_interp_duplicate_columns_and_zero_diagonal(dt):
    say("ls_interp degenerate %s" % dt)
    ad = lib()
    dtype = DT[dt]
    N, K, cal = 24, 8, 4
    A = W.laplacian_2d_5pt(N)
    val = A.val.copy()
    cf = W.cf_red_is_coarse((N, N))
    X = oracle.tv_init(A.n, K, 19)
    # F row 1 (ix=1, iy=0): C-neighbours 0, 2, 25; make 2 a copy of 0 and 25 zero
    X[2] = X[0]
    X[25] = 0.0
    # F row 26 gets a zero diagonal (residual target falls back, status 3)
    r = 26
    val[A.row_ptr[r]:A.row_ptr[r + 1]][A.col[A.row_ptr[r]:A.row_ptr[r + 1]] == r] = 0.0
    A = W.CSR(A.n, A.row_ptr, A.col, val)
    Ao = as_oracle(A, dtype)
    Ad = dev_csr(A, dtype)
    Xt = torch.as_tensor(X, dtype=dtype, device="cuda")
    mu = ad.algebraic_distance(Ad, Xt)
    cft = torch.as_tensor(cf, device="cuda")
    x = to_np(Xt).astype(np.float64)
    for target, tg in (("plain", 0), ("residual", 1)):
        ad.status(clear=True)
        got = ad.ls_interp(Ad, Xt, cft, mu, cal, target=target)
        ref = oracle.ls_interp(Ao, x, None, cf, to_np(mu).astype(np.float64), cal, tg)
        T = x if tg == 0 else residual_target(Ao, x)
        check_ls(tuple(to_np(t) for t in got), ref, dtype, (T * T).sum(1))
        st = to_np(got[3])
        assert st[1] == 2
        if tg == 1:
            assert st[26] == 3 and ad.status(clear=True) & ad.STAT_ZERO_DIAG


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("target", ["plain", "residual"])
@pytest.mark.parametrize("K,cal,weighted", [(16, 4, False), (8, 8, True), (32, 3, True)])
def test_fused_distance_ls_equals_separate_calls(dt, target, K, cal, weighted):
    """distance_ls against algebraic_distance + ls_interp with the same lanes
    per row: mu, mask, counts and every LS row bitwise; ls_sum to 1e-12; and
    against the oracle."""
    say("distance_ls %s %s K=%d cal=%d w=%s" % (dt, target, K, cal, weighted))
    ad = lib()
    dtype = DT[dt]
    N = 45
    A = aniso(N)
    Ao = as_oracle(A, dtype)
    Ad = dev_csr(A, dtype)
    color = torch.as_tensor(W.red_black((N, N)), device="cuda")
    X = ad.setup_testvectors(Ad, K, seed=23, relax="gs", sweeps=3, color=color, ncolors=2)
    x = to_np(X).astype(np.float64)
    w = (0.5 + np.random.default_rng(K).random(K)) if weighted else None
    wt = None if w is None else torch.as_tensor(w, device="cuda")
    cf = (np.random.default_rng(5).random(A.n) < 0.4).astype(np.uint8)
    cft = torch.as_tensor(cf, device="cuda")
    fm = (np.random.default_rng(6).random(A.n) < 0.8).astype(np.uint8)
    fmt = torch.as_tensor(fm, device="cuda")
    tg = oracle.TARGET_PLAIN if target == "plain" else oracle.TARGET_RESIDUAL
    T = x if target == "plain" else residual_target(Ao, x)
    wv = np.ones(K) if w is None else w
    try:
        for lpr in [0] + valid_lprs(dtype, K):
            for kern in ("distance_ls", "ls_interp"):
                ad.set_launch(kern, dtype, K, lpr, 1, True)
            # the separate distance call in the row-group form of the same shape
            ad.set_launch("algdist", dtype, K, lpr if lpr else ls_default_lpr(dtype, K), 1, True)
            for fmask in (None, fmt):
                got = ad.distance_ls(Ad, X, cft, cal, w=wt, target=target, theta=0.25,
                                     fmask=fmask, want_sum=True)
                mu, s, ns = ad.algebraic_distance(Ad, X, w=wt, target=target, fuse=True, theta=0.25,
                                                  fmask=fmask)
                Pc, Pv, ls, st, tot = ad.ls_interp(Ad, X, cft, mu, cal, w=wt, target=target,
                                                   want_sum=True)
                assert torch.equal(got[0], mu) and torch.equal(got[1], s) and torch.equal(got[2], ns), lpr
                for a, b in zip(got[3:7], (Pc, Pv, ls, st)):
                    assert torch.equal(a, b), lpr
                assert abs(float(got[7]) - float(tot)) <= 1e-12 * abs(float(tot)), lpr
            mh = to_np(got[0]).astype(np.float64)
            ref = oracle.ls_interp(Ao, x, w, cf, mh, cal, tg)
            check_ls(tuple(to_np(t) for t in got[3:7]), ref, dtype, (T * T * wv).sum(1))
            check_mu(mh, oracle.algdist(Ao, x, w, tg), saa_per_edge(Ao, T, w), dtype)
    finally:
        for kern in ("distance_ls", "ls_interp", "algdist"):
            ad.set_launch(kern, dtype, K, 0, 1, True)
    assert ad.status(clear=True) == 0


def ls_default_lpr(dt, K):
    """The LS rows' default lanes per row: 16 bytes of panel per lane."""
    size = 4 if dt == torch.float32 else 8
    for L in valid_lprs(dt, K):
        if (K // L) * size <= 16:
            return L
    return valid_lprs(dt, K)[-1]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_fused_distance_ls_degenerate_rows(dt):
    """Duplicate and zero C-neighbour columns (status 2), a zero diagonal on
    the residual target (status 3), rows without C-neighbours (status 1),
    diagonal-only rows, through the fused call."""
    say("distance_ls degenerate %s" % dt)
    ad = lib()
    dtype = DT[dt]
    N, K, cal = 24, 8, 4
    A = W.laplacian_2d_5pt(N)
    val = A.val.copy()
    cf = W.cf_red_is_coarse((N, N))
    X = oracle.tv_init(A.n, K, 19)
    X[2] = X[0]
    X[25] = 0.0
    r = 26
    val[A.row_ptr[r]:A.row_ptr[r + 1]][A.col[A.row_ptr[r]:A.row_ptr[r + 1]] == r] = 0.0
    A = W.CSR(A.n, A.row_ptr, A.col, val)
    Ao = as_oracle(A, dtype)
    Ad = dev_csr(A, dtype)
    Xt = torch.as_tensor(X, dtype=dtype, device="cuda")
    cft = torch.as_tensor(cf, device="cuda")
    x = to_np(Xt).astype(np.float64)
    for target, tg in (("plain", 0), ("residual", 1)):
        ad.status(clear=True)
        got = ad.distance_ls(Ad, Xt, cft, cal, target=target)
        mh = to_np(got[0]).astype(np.float64)
        ref = oracle.ls_interp(Ao, x, None, cf, mh, cal, tg)
        T = x if tg == 0 else residual_target(Ao, x)
        check_ls(tuple(to_np(t) for t in got[3:7]), ref, dtype, (T * T).sum(1))
        st = to_np(got[6])
        assert st[1] == 2
        if tg == 1:
            assert st[26] == 3 and ad.status(clear=True) & ad.STAT_ZERO_DIAG
    # all rows F: every row has status 1 and ls_val = sum w t^2
    cf0 = torch.zeros(A.n, dtype=torch.uint8, device="cuda")
    got = ad.distance_ls(Ad, Xt, cf0, cal, want_sum=True)
    assert np.all(to_np(got[6]) == 1)
    assert np.allclose(to_np(got[5]), (x * x).sum(1), rtol=1e-12)
    # empty matrix
    E = W.CSR(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    got = ad.distance_ls(dev_csr(E, dtype), torch.empty((0, K), dtype=dtype, device="cuda"),
                         torch.empty(0, dtype=torch.uint8, device="cuda"), cal, want_sum=True)
    assert float(got[7]) == 0.0


def test_diagonal_only_rows():
    say("diagonal-only rows")
    ad = lib()
    n, K = 130, 8
    rp = np.arange(n + 1, dtype=np.int32)
    A = W.CSR(n, rp, np.arange(n, dtype=np.int32), np.full(n, 2.0))
    Ad = dev_csr(A, torch.float64)
    X = ad.setup_testvectors(Ad, K, seed=1, relax="jacobi", sweeps=2, omega=0.5)
    want, _ = oracle.jacobi(A, oracle.tv_init(n, K, 1), 0.5, 2)
    assert np.array_equal(to_np(X), want)  # exact: x - 0.5 * 2x / 2 per sweep
    mu, s, ns = ad.algebraic_distance(Ad, X, fuse=True, theta=0.25)
    assert np.all(to_np(mu) == 0) and np.all(to_np(s) == 0) and np.all(to_np(ns) == 0)
    cf = torch.zeros(n, dtype=torch.uint8, device="cuda")
    Pc, Pv, ls, st = ad.ls_interp(Ad, X, cf, mu, 2)
    assert np.all(to_np(st) == 1) and np.all(to_np(Pc) == -1)
    xn = to_np(X)
    assert np.allclose(to_np(ls), (xn * xn).sum(1), rtol=1e-14)


# ------------------------------------------------------------------ determinism / errors
def test_run_to_run_bitwise_identical():
    say("determinism")
    ad = lib()
    N, K = 64, 16
    A = aniso(N)
    Ad = dev_csr(A, torch.float32)
    color = torch.as_tensor(W.red_black((N, N)), device="cuda")
    cf = torch.as_tensor(W.cf_red_is_coarse((N, N)), device="cuda")
    outs = []
    for _ in range(2):
        X = ad.setup_testvectors(Ad, K, seed=1, relax="gs", sweeps=5, color=color, ncolors=2)
        mu, s, ns = ad.algebraic_distance(Ad, X, fuse=True, theta=0.25)
        res = ad.ls_interp(Ad, X, cf, mu, 4, want_sum=True)
        outs.append([X, mu, s, ns] + list(res))
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_step_graph_replay_matches_eager():
    """The whole step (start, colour-phase sweeps, fused distances + strength +
    LS rows with the F-row sum) captured once and replayed: every replay,
    with eager steps on other start vectors between the replays, equals the
    eager result bitwise."""
    say("graph replay of the whole step")
    ad = lib()
    N, K = 97, 16
    A = aniso(N)
    Ad = dev_csr(A, torch.float32)
    color = torch.as_tensor(W.red_black((N, N)), device="cuda")
    cf = torch.as_tensor(W.cf_red_is_coarse((N, N)), device="cuda")
    X = torch.empty((A.n, K), dtype=torch.float32, device="cuda")
    ad.setup_testvectors(Ad, K, seed=1, relax="gs", sweeps=5, color=color, ncolors=2, out=X)
    out = ad.distance_ls(Ad, X, cf, 4, theta=0.25, want_sum=True)

    def step(seed):
        ad.setup_testvectors(Ad, K, seed=seed, relax="gs", sweeps=5, color=color, ncolors=2,
                             out=X)
        ad.distance_ls(Ad, X, cf, 4, theta=0.25, mu=out[0], strong=out[1], nstrong=out[2],
                       P_col=out[3], P_val=out[4], ls_val=out[5], row_status=out[6],
                       ls_sum=out[7], want_sum=True)

    bufs = [X] + list(out)
    step(1)
    torch.cuda.synchronize()
    ref = [b.clone() for b in bufs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step(1)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step(1)
    for r in range(3):
        step(7 + r)
        torch.cuda.synchronize()
        assert not torch.equal(X, ref[0])
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(bufs, ref):
            assert torch.equal(a, b), "replay %d" % r
    assert ad.status(clear=True) == 0


def test_host_argument_errors():
    say("argument errors")
    ad = lib()
    A = aniso(8)
    Ad = dev_csr(A, torch.float64)
    with pytest.raises(ad.AlgdistError, match="AD_EINVAL"):
        ad.setup_testvectors(Ad, 3, seed=1)
    X = ad.setup_testvectors(Ad, 4, seed=1)
    mu = ad.algebraic_distance(Ad, X)
    cf = torch.ones(A.n, dtype=torch.uint8, device="cuda")
    with pytest.raises(ad.AlgdistError, match="AD_ECALIBER"):
        ad.ls_interp(Ad, X, cf, mu, 5)
    with pytest.raises(ad.AlgdistError, match="AD_EINVAL"):
        ad.strength_graph(Ad, mu, 1.5)
    big = torch.empty(A.n * 4 + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(ad.AlgdistError, match="aligned"):
        ad.algebraic_distance(Ad, big[1:].view(A.n, 4))
    with pytest.raises(ad.AlgdistError, match="AD_EINVAL"):
        ad.setup_testvectors(Ad, 4, relax="gs", sweeps=1, color=None, ncolors=2)


def test_csr_validate_flags():
    say("csr_validate")
    ad = lib()
    A = aniso(10)
    ad.status(clear=True)
    ad.csr_validate(dev_csr(A, torch.float64))
    assert ad.status(clear=True) == 0
    col = A.col.copy()
    s = A.row_ptr[33]
    col[s], col[s + 1] = col[s + 1], col[s]  # unsorted row
    B = W.CSR(A.n, A.row_ptr, col, A.val)
    ad.csr_validate(dev_csr(B, torch.float64))
    assert ad.status(clear=True) & ad.STAT_CSR_COLS
    col = A.col.copy()
    r = 40
    row = slice(A.row_ptr[r], A.row_ptr[r + 1])
    col[row] = np.where(col[row] == r, r + 50, col[row])  # no diagonal, unsorted too
    ad.csr_validate(dev_csr(W.CSR(A.n, A.row_ptr, col, A.val), torch.float64))
    assert ad.status(clear=True) & ad.STAT_CSR_NODIAG


# ------------------------------------------------------------------ launch shapes
def valid_lprs(dt, K):
    """Lanes-per-row values the kernels accept (mirror of the library's rule)."""
    size = 4 if dt == torch.float32 else 8
    vmax = 64 // size
    out = []
    L = 1
    while L <= 64:
        V = K // L
        if K % L == 0 and V <= vmax and V * size >= 8 and (V >= vmax // 4 or V == K):
            out.append(L)
        L *= 2
    return out


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("K", [4, 16, 32])
def test_every_launch_shape_gives_the_same_results(dt, K):
    ad = lib()
    dtype = DT[dt]
    say("launch shapes %s K=%d lprs=%s" % (dt, K, valid_lprs(dtype, K)))
    N = 39
    A = aniso(N)
    Ad = dev_csr(A, dtype)
    color = torch.as_tensor(W.red_black((N, N)), device="cuda")
    cf = torch.as_tensor(W.cf_red_is_coarse((N, N)), device="cuda")
    ref = None
    try:
        for lpr in [0] + valid_lprs(dtype, K):
            for it in (1, 3):
                for xcd in (1, 0, 4):
                    for kern in ("jacobi", "gs_phase", "algdist"):
                        ad.set_launch(kern, dtype, K, lpr, it, xcd)
                    ad.set_launch("ls_interp", dtype, K, 0, 1, xcd)
                    Xg = ad.setup_testvectors(Ad, K, seed=3, relax="gs", sweeps=3, color=color, ncolors=2)
                    Xj = ad.setup_testvectors(Ad, K, seed=3, relax="jacobi", sweeps=3, omega=0.7)
                    mu, s, ns = ad.algebraic_distance(Ad, Xg, fuse=True, theta=0.25)
                    P = ad.ls_interp(Ad, Xg, cf, mu, 4)
                    if ref is None:
                        ref = (Xg, Xj)
                        x = to_np(Xg).astype(np.float64)
                        mu_ref = oracle.algdist(as_oracle(A, dtype), x)
                        saa = saa_per_edge(A, x)
                    assert torch.equal(Xg, ref[0]) and torch.equal(Xj, ref[1]), (lpr, it, xcd)
                    check_mu(to_np(mu).astype(np.float64), mu_ref, saa, dtype, "lpr=%d it=%d" % (lpr, it))
                    mh = to_np(mu).astype(np.float64)
                    sr, nsr = oracle.strength(A, mh, 0.25)
                    assert np.array_equal(to_np(s), sr) and np.array_equal(to_np(ns), nsr)
                    R = oracle.ls_interp(as_oracle(A, dtype), x, None, W.cf_red_is_coarse((N, N)), mh, 4)
                    check_ls(tuple(to_np(t) for t in P), R, dtype, (x * x).sum(1))
    finally:
        for kern in ("jacobi", "gs_phase", "algdist", "ls_interp"):
            ad.set_launch(kern, dtype, K, 0, 1, True)


def test_autotune_installs_and_caches(tmp_path):
    ad = lib()
    say("autotune")
    N, K = 96, 16
    A = aniso(N)
    dtype = torch.float32
    Ad = dev_csr(A, dtype)
    color = torch.as_tensor(W.red_black((N, N)), device="cuda")
    cfh = W.cf_red_is_coarse((N, N))
    cf = torch.as_tensor(cfh, device="cuda")
    cache = str(tmp_path / "tune.json")
    try:
        ad.autotune(Ad, K, relax="gs", color=color, ncolors=2, cf=cf, caliber=4, cache_json=cache)
        lines = open(cache).read().splitlines()
        kinds = sorted(l.split('"')[3] for l in lines)
        assert kinds == ["algdist", "distance_ls", "gs_phase", "ls_interp"], lines
        ad.autotune(Ad, K, relax="gs", color=color, ncolors=2, cf=cf, caliber=4, cache_json=cache)
        assert open(cache).read().splitlines() == lines  # served from the cache
        X = ad.setup_testvectors(Ad, K, seed=2, relax="gs", sweeps=3, color=color, ncolors=2)
        mu, s, ns = ad.algebraic_distance(Ad, X, fuse=True, theta=0.25)
        x = to_np(X).astype(np.float64)
        check_mu(to_np(mu).astype(np.float64), oracle.algdist(as_oracle(A, dtype), x),
                 saa_per_edge(A, x), dtype, "tuned")
        sr, nsr = oracle.strength(A, to_np(mu).astype(np.float64), 0.25)
        assert np.array_equal(to_np(s), sr)
        P = ad.ls_interp(Ad, X, cf, mu, 4)
        R = oracle.ls_interp(as_oracle(A, dtype), x, None, cfh, to_np(mu).astype(np.float64), 4)
        check_ls(tuple(to_np(t) for t in P), R, dtype, (x * x).sum(1))
    finally:
        for kern in ("gs_phase", "algdist", "ls_interp"):
            ad.set_launch(kern, dtype, K, 0, 1, True)
