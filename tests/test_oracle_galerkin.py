"""Pins of the oracle's Galerkin operator A_c = P^T A P and two-grid method
(Sec. 5.2): dense products on tiny cases, the closed form for linear
interpolation on the 1D Laplacian (the coarse operator is half the coarse
Laplacian), P = I, zero row sums carried over when P preserves constants,
exact two-grid convergence with the ideal interpolation and with P = I, and
the two-grid rate against the spectral radius of the error-propagation
matrix assembled densely from the colour-phase splitting."""
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


def dense_p(Pc, Pv, cf):
    cidx = np.cumsum(cf.astype(np.int64)) - 1
    P = np.zeros((len(cf), int(cf.sum())))
    for i in range(len(cf)):
        for q in range(Pc.shape[1]):
            if Pc[i, q] >= 0:
                P[i, cidx[Pc[i, q]]] += Pv[i, q]
    return P


def lap1d(n):
    rp, ci, va = [0], [], []
    for i in range(n):
        for j, v in ((i - 1, -1.0), (i, 2.0), (i + 1, -1.0)):
            if 0 <= j < n:
                ci.append(j)
                va.append(v)
        rp.append(len(ci))
    return W.CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va))


def linear_interpolation_1d(n):
    """C = odd points; an F point takes 1/2 from each C neighbour (the
    Dirichlet boundary contributes nothing)."""
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


def setup(kind, N, seed=1):
    if kind == "aniso9":
        A = W.rotated_anisotropic_9pt(N, 1e-3, math.pi / 6)
    else:
        A = W.lognormal_2d_5pt(N, 1.0, seed)
    color = W.red_black((N, N))
    X = oracle.tv_init(A.n, 8, seed)
    X, _ = oracle.color_gs(A, X, color, 2, 20)
    mu = oracle.algdist(A, X)
    cf, _, _ = oracle.cr_coarsen(A, color, 2, mu, 0.25, seed=seed)
    Pc, Pv, _, _ = oracle.ls_interp(A, X, None, cf, mu, 4)
    return A, color, cf, Pc, Pv


@pytest.mark.parametrize("kind,N", [("aniso9", 9), ("lognormal", 10), ("aniso9", 14)])
def test_galerkin_is_the_dense_triple_product(kind, N):
    A, color, cf, Pc, Pv = setup(kind, N)
    Ac = oracle.galerkin(A, Pc, Pv, cf)
    P = dense_p(Pc, Pv, cf)
    want = P.T @ dense(A) @ P
    got = dense(W.CSR(Ac.n, Ac.row_ptr, Ac.col, Ac.val))
    assert Ac.n == int(cf.sum())
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    # columns sorted per row, every structural product stored
    for I in range(Ac.n):
        c = Ac.col[Ac.row_ptr[I]:Ac.row_ptr[I + 1]]
        assert np.all(np.diff(c) > 0)
    reach = (np.abs(P.T) @ np.abs(dense(A) != 0) @ (np.abs(P) > 0)) > 0
    assert Ac.nnz == int(reach.sum())


def test_linear_interpolation_on_the_1d_laplacian_gives_half_the_coarse_laplacian():
    n = 15
    A = lap1d(n)
    cf, Pc, Pv = linear_interpolation_1d(n)
    Ac = oracle.galerkin(A, Pc, Pv, cf)
    got = dense(W.CSR(Ac.n, Ac.row_ptr, Ac.col, Ac.val))
    m = Ac.n
    want = 0.5 * (2 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1))
    assert np.array_equal(got, want)


def test_identity_interpolation_and_constant_preservation():
    A = W.lognormal_2d_5pt(9, 1.0, 2)
    n = A.n
    cf = np.ones(n, np.uint8)
    Pc = np.arange(n, dtype=np.int32)[:, None]
    Pv = np.ones((n, 1))
    Ac = oracle.galerkin(A, Pc, Pv, cf)
    assert np.array_equal(Ac.row_ptr, A.row_ptr) and np.array_equal(Ac.col, A.col)
    assert np.array_equal(Ac.val, A.val)
    # a graph Laplacian (zero row sums) and rows of P summing to one: A_c 1 = 0
    G = W.rgg_laplacian(400, 8.0, (3, 3), shift=0.0)
    rng = np.random.default_rng(5)
    cf = (rng.random(G.n) < 0.3).astype(np.uint8)
    C = np.nonzero(cf)[0]
    Pc = -np.ones((G.n, 3), np.int32)
    Pv = np.zeros((G.n, 3))
    for i in range(G.n):
        if cf[i]:
            Pc[i, 0], Pv[i, 0] = i, 1.0
        else:
            pick = rng.choice(C, 3, replace=False)
            w = rng.random(3)
            Pc[i], Pv[i] = pick, w / w.sum()
    Ac = oracle.galerkin(G, Pc, Pv, cf)
    rows = np.add.reduceat(Ac.val, Ac.row_ptr[:-1]) if Ac.nnz else np.zeros(0)
    assert np.max(np.abs(rows)) <= 1e-12 * np.max(np.abs(Ac.val))


def test_two_grid_is_exact_with_the_ideal_interpolation_and_with_p_identity():
    """1D Laplacian, C = odd points: F points couple only to C points, so the
    linear interpolation is the ideal one (-A_ff^{-1} A_fc); one pre-sweep
    ends with the F phase and leaves the error in range(P), which the
    coarse-grid correction removes exactly."""
    n = 31
    A = lap1d(n)
    cf, Pc, Pv = linear_interpolation_1d(n)
    color = (1 - cf).astype(np.int32)  # C first (colour 0), then F
    Ac = oracle.galerkin(A, Pc, Pv, cf)
    E0 = oracle.tv_init(n, 3, 4)
    rho, bad, hist = oracle.two_grid(A, color, 2, Pc, Pv, cf, Ac, E0, iters=2, pre=1, post=0)
    assert bad == 0 and np.all(hist[1] <= 1e-13 * hist[0])
    # P = I: A_c = A and the coarse solve is the exact solve
    B = W.lognormal_2d_5pt(8, 1.0, 3)
    cfI = np.ones(B.n, np.uint8)
    PcI = np.arange(B.n, dtype=np.int32)[:, None]
    PvI = np.ones((B.n, 1))
    AcI = oracle.galerkin(B, PcI, PvI, cfI)
    rho, bad, hist = oracle.two_grid(B, W.red_black((8, 8)), 2, PcI, PvI, cfI, AcI,
                                     oracle.tv_init(B.n, 2, 1), iters=1, pre=2, post=2)
    assert bad == 0 and np.all(hist[1] <= 1e-12 * hist[0])


def test_two_grid_rate_is_the_spectral_radius_of_the_error_propagation():
    A, color, cf, Pc, Pv = setup("aniso9", 12)
    Ac = oracle.galerkin(A, Pc, Pv, cf)
    D = dense(A)
    # colour-phase sweep as a splitting: M = diag + couplings to earlier colours
    M = np.where(color[None, :] < color[:, None], D, 0.0) + np.diag(np.diag(D))
    S = np.eye(A.n) - np.linalg.solve(M, D)
    P = dense_p(Pc, Pv, cf)
    Acd = P.T @ D @ P
    T = S @ S @ (np.eye(A.n) - P @ np.linalg.solve(Acd, P.T @ D)) @ S @ S
    lam = np.max(np.abs(np.linalg.eigvals(T)))
    rho, bad, hist = oracle.two_grid(A, color, 2, Pc, Pv, cf, Ac, oracle.tv_init(A.n, 4, 9),
                                     iters=100, pre=2, post=2)
    assert bad == 0
    assert np.all(np.abs(rho - lam) <= 2e-3 * max(lam, 1e-3)), (rho, lam)


@pytest.mark.parametrize("eps", [1e-4, 0.0])
def test_table1_grid_aligned_case(eps):
    """The whole two-level chain on a case Table 1 (Sec. 5.5) prints: the
    7-point operator with alpha = 0 on 32^2, 8 test vectors of 40 Gauss-Seidel
    sweeps, CR on the strength graph M^2 (theta_ad 0.5, nu 5, delta 0.7), the
    set search on A^4 (caliber 4, gamma 1.5, the functional of eq:modls) and
    the two-grid rate with 2 + 2 sweeps.  The paper prints rho = .05 with
    gamma_g .34 for both eps; the chain lands below 0.1 with a coarse grid of
    at most half the points, and the plain target of eq:LSfuncrowi does worse."""
    N = 32
    n = N * N
    A = W.rotated_anisotropic_7pt(N, eps, 0.0)
    color = W.four_colour_2d(N)
    X, _ = oracle.color_gs(A, oracle.tv_init(n, 8, 3), color, 4, 40)
    G2 = oracle.power_pattern(A, 2)
    G4 = oracle.power_pattern(A, 4)
    mu2 = oracle.algdist_graph(A, G2, X)
    cf, rho_f, _ = oracle.cr_coarsen(A, color, 4, mu2, 0.5, seed=1, G=G2)
    assert rho_f[-1] <= 0.7 and 0.3 <= cf.mean() <= 0.5
    E0 = np.random.default_rng(5).uniform(-1.0, 1.0, (n, 2))
    rho = {}
    for tg in (oracle.TARGET_RESIDUAL, oracle.TARGET_PLAIN):
        Pc, Pv = oracle.ls_search(A, G4, X, None, cf, 4, 1.5, tg)[:2]
        Ac = oracle.galerkin(A, Pc, Pv, cf)
        r, bad, _ = oracle.two_grid(A, color, 4, Pc, Pv, cf, Ac, E0, iters=60)
        assert bad == 0
        rho[tg] = float(r.max())
    assert rho[oracle.TARGET_RESIDUAL] < 0.1
    assert rho[oracle.TARGET_RESIDUAL] < rho[oracle.TARGET_PLAIN]
