"""The Galerkin operator P^T A P and the two-grid method (Sec. 5.2) on the
GPU against the oracle: A_c bit for bit (same products, same accumulation
order, no contraction) for interpolation from the setup (CR coarsening, LS
rows, and the long-range set search), FP32 operators, the 1D closed form,
P = I, ignored bad columns, the size limits; the two-grid A-norm history
and rate against the oracle, and its exactness with the ideal
interpolation."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1106_5990_amd import workloads as W
from gpu_common import dev_csr, lib, say, to_np

pytestmark = pytest.mark.gpu


def gpu(t):
    return torch.as_tensor(np.ascontiguousarray(t), device="cuda")


def setup(kind, N, seed=1, longrange=False):
    if kind == "aniso9":
        A = W.rotated_anisotropic_9pt(N, 1e-3, math.pi / 6)
    elif kind == "fd7":
        A = W.rotated_anisotropic_7pt(N, 1e-2, -math.pi / 4)
    else:
        A = W.lognormal_2d_5pt(N, 1.0, seed)
    color = W.red_black((N, N))
    X = oracle.tv_init(A.n, 8, seed)
    X, _ = oracle.color_gs(A, X, color, 2, 20)
    mu = oracle.algdist(A, X)
    cf, _, _ = oracle.cr_coarsen(A, color, 2, mu, 0.25, seed=seed)
    if longrange:
        G = oracle.power_pattern(A, 2)
        Pc, Pv, _, _, _, _ = oracle.ls_search(A, G, X, None, cf, 4)
    else:
        Pc, Pv, _, _ = oracle.ls_interp(A, X, None, cf, mu, 4)
    return A, color, cf, Pc, Pv


def compare(A, Pc, Pv, cf, dt=torch.float64):
    ad = lib()
    Ac_ref = oracle.galerkin(A, Pc, Pv, cf)
    Ac = ad.galerkin(dev_csr(A, dt), gpu(Pc), gpu(Pv), gpu(cf))
    assert Ac.n == Ac_ref.n
    assert np.array_equal(to_np(Ac.row_ptr), Ac_ref.row_ptr)
    assert np.array_equal(to_np(Ac.col), Ac_ref.col)
    assert np.array_equal(to_np(Ac.val), Ac_ref.val)
    return Ac, Ac_ref


@pytest.mark.parametrize("kind,N,longrange", [("aniso9", 24, False), ("aniso9", 61, False),
                                              ("lognormal", 40, False), ("fd7", 33, False),
                                              ("aniso9", 30, True)])
def test_galerkin_bitwise(kind, N, longrange):
    say("galerkin %s N=%d longrange=%s" % (kind, N, longrange))
    A, color, cf, Pc, Pv = setup(kind, N, longrange=longrange)
    Ac, _ = compare(A, Pc, Pv, cf)
    say("  nc %d nnz_c %d (gamma_o %.3f)" % (Ac.n, Ac.nnz, (A.nnz + Ac.nnz) / A.nnz))
    assert lib().status(clear=True) == 0


def test_galerkin_wide_rows_take_the_sort_kernel():
    """Interpolation from random C points of a random geometric graph gives
    coarse rows of more than 32 distinct columns (left by the lane kernel
    to the sort kernel) beside narrower ones; A_c bit for bit either way."""
    say("galerkin: wide coarse rows")
    G = W.rgg_laplacian(600, 8.0, (3, 3), shift=0.5)
    rng = np.random.default_rng(7)
    cf = (rng.random(G.n) < 0.3).astype(np.uint8)
    C = np.nonzero(cf)[0]
    Pc = -np.ones((G.n, 3), np.int32)
    Pv = np.zeros((G.n, 3))
    for i in range(G.n):
        if cf[i]:
            Pc[i, 0], Pv[i, 0] = i, 1.0
        else:
            k = 1 + i % 3
            Pc[i, :k] = np.sort(rng.choice(C, k, replace=False))
            Pv[i, :k] = rng.random(k) - 0.3
    Ac, ref = compare(G, Pc, Pv, cf)
    ln = np.diff(ref.row_ptr)
    say("  nc %d, row lengths %d..%d, %d rows past 32" % (ref.n, ln.min(), ln.max(), (ln > 32).sum()))
    assert np.any(ln > 32) and np.any(ln <= 32)
    assert lib().status(clear=True) == 0


def test_galerkin_full_size():
    """The 2048^2 anisotropic 9-point operator (FP32) with the CR coarse
    grid and LS rows of its test vectors, as the bench forms it: A_c bit
    for bit the oracle's over all 1.17 M coarse rows."""
    say("galerkin full size")
    ad = lib()
    wl = W.workload(2, "f32")
    A32 = W.CSR(wl.A.n, wl.A.row_ptr, wl.A.col, wl.A.val.astype(np.float32).astype(np.float64))
    Ad = dev_csr(A32, torch.float32)
    color = torch.as_tensor(wl.color, device="cuda")
    X = ad.setup_testvectors(Ad, wl.K, seed=wl.tv_seed, relax="gs", sweeps=wl.sweeps,
                             color=color, ncolors=wl.ncolors)
    mu = ad.algebraic_distance(Ad, X)
    cf, _, _ = ad.cr_coarsening(Ad, color, 2, mu, wl.theta, seed=1)
    Pc, Pv, _, _ = ad.ls_interp(Ad, X, cf, mu, wl.caliber)
    Ac = ad.galerkin(Ad, Pc, Pv, cf)
    ref = oracle.galerkin(A32, to_np(Pc), to_np(Pv), to_np(cf))
    say("  nc %d nnz_c %d" % (ref.n, ref.nnz))
    assert Ac.n == ref.n
    assert np.array_equal(to_np(Ac.row_ptr), ref.row_ptr)
    assert np.array_equal(to_np(Ac.col), ref.col)
    assert np.array_equal(to_np(Ac.val), ref.val)
    assert ad.status(clear=True) == 0


def test_galerkin_fp32_operator():
    A, color, cf, Pc, Pv = setup("aniso9", 32)
    A32 = W.CSR(A.n, A.row_ptr, A.col, A.val.astype(np.float32).astype(np.float64))
    ad = lib()
    Ac = ad.galerkin(dev_csr(A, torch.float32), gpu(Pc), gpu(Pv), gpu(cf))
    ref = oracle.galerkin(A32, Pc, Pv, cf)
    assert np.array_equal(to_np(Ac.val), ref.val) and np.array_equal(to_np(Ac.col), ref.col)


def lap1d(n):
    rp, ci, va = [0], [], []
    for i in range(n):
        for j, v in ((i - 1, -1.0), (i, 2.0), (i + 1, -1.0)):
            if 0 <= j < n:
                ci.append(j)
                va.append(v)
        rp.append(len(ci))
    return W.CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va))


def linear_1d(n):
    cf = (np.arange(n) % 2 == 1).astype(np.uint8)
    Pc = -np.ones((n, 2), np.int32)
    Pv = np.zeros((n, 2))
    for i in range(n):
        if cf[i]:
            Pc[i, 0], Pv[i, 0] = i, 1.0
        else:
            q = 0
            for j in (i - 1, i + 1):
                if 0 <= j < n:
                    Pc[i, q], Pv[i, q] = j, 0.5
                    q += 1
    return cf, Pc, Pv


def test_closed_forms_identity_and_bad_columns():
    ad = lib()
    n = 63
    A = lap1d(n)
    cf, Pc, Pv = linear_1d(n)
    Ac, _ = compare(A, Pc, Pv, cf)
    vals = to_np(Ac.val)
    rp = to_np(Ac.row_ptr)
    col = to_np(Ac.col)
    for I in range(Ac.n):
        for e in range(rp[I], rp[I + 1]):
            assert vals[e] == (1.0 if col[e] == I else -0.5)
    # P = I: A_c = A
    B = W.lognormal_2d_5pt(20, 1.0, 4)
    cfI = np.ones(B.n, np.uint8)
    AcI, _ = compare(B, np.arange(B.n, dtype=np.int32)[:, None], np.ones((B.n, 1)), cfI)
    assert np.array_equal(to_np(AcI.val), B.val)
    # a column naming an F point (and one out of range) is ignored and flagged
    A2, color, cf2, Pc2, Pv2 = setup("aniso9", 20)
    f = np.nonzero(cf2 == 0)[0]
    bad = Pc2.copy()
    bad[f[0], 3] = f[1]
    bad[f[2], 3] = A2.n + 5
    ad.status(clear=True)
    Acb = ad.galerkin(dev_csr(A2, torch.float64), gpu(bad), gpu(Pv2), gpu(cf2))
    assert ad.status(clear=True) & ad.STAT_BAD_INTERP
    clean = bad.copy()
    clean[f[0], 3] = -1
    clean[f[2], 3] = -1
    ref = oracle.galerkin(A2, clean, Pv2, cf2)
    assert np.array_equal(to_np(Acb.val), ref.val)


def test_size_limit_is_an_error():
    """A C point interpolated by more than 64 fine rows (a star) is refused."""
    ad = lib()
    m = 80
    n = m + 1
    rp, ci, va = [0], [], []
    for i in range(n):
        cols = list(range(n)) if i == 0 else [0, i]
        for j in cols:
            ci.append(j)
            va.append(float(m) if (i == j == 0) else (1.0 if i == j else -1.0 / m))
        rp.append(len(ci))
    A = W.CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va))
    cf = np.zeros(n, np.uint8)
    cf[0] = 1
    Pc = np.zeros((n, 1), np.int32)
    Pv = np.ones((n, 1))
    with pytest.raises(ad.AlgdistError):
        ad.galerkin(dev_csr(A, torch.float64), gpu(Pc), gpu(Pv), gpu(cf))


@pytest.mark.parametrize("kind,N", [("aniso9", 24), ("fd7", 32), ("lognormal", 30)])
def test_two_grid_matches_oracle(kind, N):
    say("two-grid %s N=%d" % (kind, N))
    ad = lib()
    A, color, cf, Pc, Pv = setup(kind, N)
    Ac, Ac_ref = compare(A, Pc, Pv, cf)
    E0 = oracle.tv_init(A.n, 4, 13)
    rho_ref, bad, hist_ref = oracle.two_grid(A, color, 2, Pc, Pv, cf, Ac_ref, E0, iters=100)
    assert bad == 0
    rho, hist = ad.two_grid_rate(dev_csr(A, torch.float64), gpu(color), 2, gpu(Pc), gpu(Pv),
                                 gpu(cf), Ac, gpu(E0), iters=100)
    say("  rho %s vs %s; gamma_o %.3f gamma_g %.3f"
        % (np.round(rho, 5), np.round(rho_ref, 5), (A.nnz + Ac.nnz) / A.nnz, Ac.n / A.n))
    assert np.allclose(hist, hist_ref, rtol=1e-8, atol=0)
    assert np.allclose(rho, rho_ref, rtol=1e-9, atol=0)


def test_two_grid_is_exact_with_the_ideal_interpolation():
    ad = lib()
    n = 127
    A = lap1d(n)
    cf, Pc, Pv = linear_1d(n)
    color = (1 - cf).astype(np.int32)
    Ac, _ = compare(A, Pc, Pv, cf)
    E0 = oracle.tv_init(n, 2, 3)
    rho, hist = ad.two_grid_rate(dev_csr(A, torch.float64), gpu(color), 2, gpu(Pc), gpu(Pv),
                                 gpu(cf), Ac, gpu(E0), iters=2, pre=1, post=0)
    assert np.all(hist[1] <= 1e-13 * hist[0])


@pytest.mark.parametrize("where", ["first block", "third block"])
def test_two_grid_refuses_a_coarse_operator_that_is_not_positive_definite(where):
    """A negative diagonal entry makes A_c indefinite: the blocked
    factorisation meets a non-positive pivot (in the first 64-wide block, or
    in the third) and the call fails with AD_ESTRUCT."""
    ad = lib()
    n = 301
    A = lap1d(n)
    cf, Pc, Pv = linear_1d(n)
    i = 1 if where == "first block" else 281  # a C point: coarse index 0 or 140
    val = A.val.copy()
    val[(A.row_ids() == i) & (A.col == i)] = -50.0
    B = W.CSR(n, A.row_ptr, A.col, val)
    Ac, _ = compare(B, Pc, Pv, cf)
    color = (1 - cf).astype(np.int32)
    E0 = oracle.tv_init(n, 2, 3)
    with pytest.raises(ad.AlgdistError, match="AD_ESTRUCT"):
        ad.two_grid_rate(dev_csr(B, torch.float64), gpu(color), 2, gpu(Pc), gpu(Pv), gpu(cf), Ac,
                         gpu(E0), iters=2)
    ad.status(clear=True)


def test_two_grid_with_sixteen_starts():
    """K = 16 columns (the coarse applies take 8 columns per pass over the
    inverse): history and rates against the oracle."""
    ad = lib()
    A, color, cf, Pc, Pv = setup("aniso9", 24)
    Ac, Ac_ref = compare(A, Pc, Pv, cf)
    E0 = oracle.tv_init(A.n, 16, 21)
    rho_ref, bad, hist_ref = oracle.two_grid(A, color, 2, Pc, Pv, cf, Ac_ref, E0, iters=30)
    rho, hist = ad.two_grid_rate(dev_csr(A, torch.float64), gpu(color), 2, gpu(Pc), gpu(Pv),
                                 gpu(cf), Ac, gpu(E0), iters=30)
    assert np.allclose(hist, hist_ref, rtol=1e-8, atol=0)
    assert np.allclose(rho, rho_ref, rtol=1e-9, atol=0)


@pytest.mark.parametrize("eps", [1e-4, 0.0])
def test_table1_grid_aligned_case_on_the_gpu(eps):
    """The whole two-level setup on the GPU for a case Table 1 (Sec. 5.5)
    prints, rho = .05: the 7-point operator with alpha = 0 on 32^2, 8 test
    vectors of 40 Gauss-Seidel sweeps, CR on M^2, the set search on A^4 with
    the functional of eq:modls, A_c and the two-grid rate.  The rate is below
    0.1, and the oracle's two-grid method on the GPU's P and A_c gives the
    same rate and history."""
    ad = lib()
    N = 32
    A = W.rotated_anisotropic_7pt(N, eps, 0.0)
    Ad = dev_csr(A, torch.float64)
    color = W.four_colour_2d(N)
    cd = gpu(color)
    X = ad.setup_testvectors(Ad, 8, seed=3, relax="gs", sweeps=40, color=cd, ncolors=4)
    G2 = ad.power_graph(Ad, 2)
    mu2 = ad.algebraic_distance_graph(Ad, G2, X)
    cf, _, _ = ad.cr_coarsening(Ad, cd, 4, mu2, 0.5, seed=1, G=G2)
    G4 = ad.power_graph(Ad, 4)
    Pc, Pv, _, _ = ad.ls_interp_search(Ad, G4, X, cf, 4, 1.5, target="residual")
    Ac = ad.galerkin(Ad, Pc, Pv, cf)
    E0 = oracle.tv_init(A.n, 2, 13)
    rho, hist = ad.two_grid_rate(Ad, cd, 4, Pc, Pv, cf, Ac, gpu(E0), iters=60)
    say("  eps %g: rho %s, gamma_g %.3f" % (eps, np.round(rho, 4), Ac.n / A.n))
    assert float(max(rho)) < 0.1
    Ac_h = oracle.CoarseCSR(Ac.n, to_np(Ac.row_ptr), to_np(Ac.col), to_np(Ac.val))
    rho_ref, bad, hist_ref = oracle.two_grid(A, color, 4, to_np(Pc), to_np(Pv), to_np(cf), Ac_h,
                                             E0, iters=60)
    assert bad == 0
    assert np.allclose(hist, hist_ref, rtol=1e-8, atol=0)
    assert np.allclose(rho, rho_ref, rtol=1e-9, atol=0)
    assert ad.status(clear=True) == 0
