"""Compatible-relaxation coarsening on the GPU (Sec. 3.2, Sec. 4.2 Algorithm 1)
against the oracle: the F-relaxation run and its rate, the candidate rule,
the independent set (bit-exact: an integer result fixed by the priority
order), and the whole loop -- the same C sets stage by stage when the
oracle's decisions (sigma_i against tol, rho_f against delta) are not within
rounding of their thresholds, which each case checks and reports."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1106_5990_amd import workloads as W
from gpu_common import dev_csr, lib, say, to_np

pytestmark = pytest.mark.gpu


def aniso(N):
    return W.rotated_anisotropic_9pt(N, 1e-3, math.pi / 6)


def operator(kind, N):
    if kind == "aniso9":
        return aniso(N)
    if kind == "lap5":
        return W.laplacian_2d_5pt(N)
    return W.lognormal_2d_5pt(N, 1.0, 3)


def gpu(t, dt=None):
    return torch.as_tensor(t, device="cuda") if dt is None else torch.as_tensor(t, dtype=dt,
                                                                               device="cuda")


@pytest.mark.parametrize("kind,N", [("aniso9", 61), ("lap5", 90), ("lognormal", 47),
                                    ("aniso9", 203)])
def test_cr_rate_matches_oracle(kind, N):
    say("cr_rate %s N=%d" % (kind, N))
    ad = lib()
    A = operator(kind, N)
    color = W.red_black((N, N))
    rng = np.random.default_rng(N)
    cf = (rng.random(A.n) < 0.3).astype(np.uint8)
    r_ref, u_ref = oracle.cr_rate(A, color, 2, cf, 5)
    r, u, norms = ad.cr_rate(dev_csr(A, torch.float64), gpu(color), 2, gpu(cf), 5)
    u = to_np(u)
    assert norms[0] == float((cf == 0).sum())
    assert np.all(u[cf == 1] == 0.0)
    assert np.max(np.abs(u - u_ref)) <= 1e-12 * np.max(np.abs(u_ref))
    assert r == pytest.approx(r_ref, rel=1e-12)
    assert norms[2] == pytest.approx(np.max(np.abs(u_ref[cf == 0])), rel=1e-12)
    # FP32 operator and panel: the same rate to FP32 rounding through 5 sweeps
    r32, u32, _ = ad.cr_rate(dev_csr(A, torch.float32), gpu(color), 2, gpu(cf), 5)
    A32 = W.CSR(A.n, A.row_ptr, A.col, A.val.astype(np.float32).astype(np.float64))
    r_ref32, u_ref32 = oracle.cr_rate(A32, color, 2, cf, 5)
    assert np.max(np.abs(to_np(u32) - u_ref32)) <= 1e-5 * np.max(np.abs(u_ref32))
    assert r32 == pytest.approx(r_ref32, rel=1e-5)
    assert ad.status(clear=True) == 0  # the C rows' missing colour is not reported


def test_cr_rate_edge_cases():
    ad = lib()
    N = 16
    A = W.laplacian_2d_5pt(N)
    color = W.red_black((N, N))
    Ad = dev_csr(A, torch.float64)
    # every F point couples only to C points: one sweep zeroes u_f
    cf = (color == 0).astype(np.uint8)
    r, u, norms = ad.cr_rate(Ad, gpu(color), 2, gpu(cf), 5)
    assert r == 0.0 and torch.count_nonzero(u).item() == 0
    # F empty
    r, u, norms = ad.cr_rate(Ad, gpu(color), 2, gpu(np.ones(A.n, np.uint8)), 3)
    assert r == 0.0 and norms[0] == 0.0
    with pytest.raises(ad.AlgdistError):
        ad.cr_rate(Ad, gpu(color), 2, gpu(cf), 0)


@pytest.mark.parametrize("n", [1, 1000, 70001])
def test_cr_candidates_bitwise(n):
    ad = lib()
    rng = np.random.default_rng(n)
    cf = (rng.random(n) < 0.25).astype(np.uint8)
    u = rng.standard_normal(n)
    u[:: 7] = 0.5  # ties with the threshold below
    m = np.max(np.abs(u[cf == 0])) if (cf == 0).any() else 0.0
    for tol in (0.0, 0.3, 0.5 / m if m else 0.5, 0.99):
        z = ad.cr_candidates(gpu(cf), gpu(u), tol)
        assert np.array_equal(to_np(z), oracle.cr_candidates(cf, u, tol)), tol
    z32 = ad.cr_candidates(gpu(cf), gpu(u, torch.float32), 0.3)
    u32 = u.astype(np.float32).astype(np.float64)
    assert np.array_equal(to_np(z32), oracle.cr_candidates(cf, u32, 0.3))


def drop_offdiagonal(A, frac, seed):
    """A with a random fraction of its off-diagonal entries removed: the
    pattern is no longer structurally symmetric."""
    rng = np.random.default_rng(seed)
    keep = (A.col == A.row_ids()) | (rng.random(A.nnz) >= frac)
    rid = A.row_ids()[keep]
    rp = np.zeros(A.n + 1, np.int64)
    np.cumsum(np.bincount(rid, minlength=A.n), out=rp[1:])
    return W.CSR(A.n, rp.astype(np.int32), A.col[keep], A.val[keep])


@pytest.mark.parametrize("kind,n,p_strong,p_z", [("rgg", 300, 0.5, 0.7), ("rgg", 40000, 0.4, 0.6),
                                                 ("grid", 250, 1.0, 1.0), ("grid", 401, 0.6, 0.3),
                                                 ("rgg", 5000, 0.0, 0.5), ("rgg", 5000, 0.5, 0.0),
                                                 ("asym", 6000, 0.5, 0.6)])
def test_independent_set_bitwise(kind, n, p_strong, p_z):
    """Random strong graphs (not symmetric) on geometric graphs and 9-point
    grids (many equal weights: the hash decides), candidate sets of every
    density, no strong entries (every candidate is chosen), no candidates;
    and a structurally asymmetric pattern (the column index's general
    path)."""
    say("independent set %s n=%d" % (kind, n))
    ad = lib()
    rng = np.random.default_rng(n)
    if kind == "asym":
        A = drop_offdiagonal(W.rgg_laplacian(n, 10.0, (n, 2)), 0.1, n)
    else:
        A = W.rgg_laplacian(n, 10.0, (n, 2)) if kind == "rgg" else aniso(n)
    strong = (rng.random(A.nnz) < p_strong).astype(np.uint8)
    strong[A.col == A.row_ids()] = 0
    z = (rng.random(A.n) < p_z).astype(np.uint8)
    for seed in (0, 12345):
        want = oracle.independent_set(A, strong, z, seed)
        sel, cnt = ad.independent_set(dev_csr(A, torch.float64), gpu(strong), gpu(z), seed)
        assert np.array_equal(to_np(sel), want), seed
        assert cnt == int(want.sum())
    if p_strong == 0.0:
        assert np.array_equal(want, z)


def margins(A, color, mu, theta, nu, delta, cf_stages):
    """Smallest distance of the oracle's decisions to their thresholds over
    the stages it ran: (min |sigma_i - tol|, min |rho - delta|)."""
    ms, mr = np.inf, np.inf
    for cf in cf_stages:
        r, u = oracle.cr_rate(A, color, 2, cf, nu)
        mr = min(mr, abs(r - delta))
        F = cf == 0
        if F.any() and np.max(np.abs(u[F])) > 0:
            sig = np.abs(u[F]) / np.max(np.abs(u[F]))
            ms = min(ms, float(np.min(np.abs(sig - (1.0 - r)))))
    return ms, mr


def oracle_stages(A, color, mu, theta, nu, delta, max_stages, seed):
    """The oracle's loop replayed from its building blocks, keeping each
    stage's C set."""
    cf = np.zeros(A.n, np.uint8)
    out = [cf.copy()]
    r, u = oracle.cr_rate(A, color, 2, cf, nu)
    s = 0
    while r > delta and s < max_stages:
        z = oracle.cr_candidates(cf, u, 1.0 - r)
        strong, _ = oracle.strength(A, mu, theta, fmask=(cf == 0).astype(np.uint8))
        sel = oracle.independent_set(A, strong, z, seed + s)
        if not sel.any():
            break
        cf = cf | sel
        out.append(cf.copy())
        s += 1
        r, u = oracle.cr_rate(A, color, 2, cf, nu)
    return out


@pytest.mark.parametrize("kind,N,seed,delta", [
    ("aniso9", 64, 3, 0.7), ("aniso9", 150, 11, 0.7), ("lap5", 96, 5, 0.7),
    ("lognormal", 80, 7, 0.7),
    # smaller delta: several stages (up to the stage limit)
    ("aniso9", 64, 3, 0.4), ("aniso9", 100, 5, 0.3), ("lognormal", 80, 7, 0.2),
    ("lap5", 60, 2, 0.2)])
def test_cr_coarsening_matches_oracle(kind, N, seed, delta):
    say("cr_coarsening %s N=%d delta=%g" % (kind, N, delta))
    ad = lib()
    A = operator(kind, N)
    color = W.red_black((N, N))
    X = oracle.tv_init(A.n, 8, seed)
    X, _ = oracle.color_gs(A, X, color, 2, 5)
    mu = oracle.algdist(A, X)
    cf_ref, rho_ref, nc_ref = oracle.cr_coarsen(A, color, 2, mu, 0.25, nu=5, delta=delta,
                                                max_stages=20, seed=seed)
    ms, mr = margins(A, color, mu, 0.25, 5, delta,
                     oracle_stages(A, color, mu, 0.25, 5, delta, 20, seed))
    say("  stages %d |C| %s rho %s; margins sigma %.3g rho %.3g"
        % (len(rho_ref) - 1, list(nc_ref), np.round(rho_ref, 4).tolist(), ms, mr))
    assert ms > 1e-9 and mr > 1e-9  # no decision within rounding of its threshold
    cf, rho, nc = ad.cr_coarsening(dev_csr(A, torch.float64), gpu(color), 2, gpu(mu), 0.25, nu=5,
                                   delta=delta, max_stages=20, seed=seed)
    assert np.array_equal(to_np(cf), cf_ref)
    assert nc == list(nc_ref)
    assert np.allclose(rho, rho_ref, rtol=1e-12, atol=0)
    assert ad.status(clear=True) == 0


@pytest.mark.parametrize("kind,N,seed,delta", [("aniso9", 64, 3, 0.7), ("lognormal", 80, 7, 0.4),
                                                ("lap5", 60, 2, 0.3)])
def test_cr_coarsening_on_the_graph_of_a_squared(kind, N, seed, delta):
    """Algorithm 1 with M^2 (Sec. 4.2): strength graph and independent set
    on the pattern of A^2 (the GPU's, equal to the oracle's), distances on
    it; C points bit for bit the oracle's, rho_f per stage to 1e-12."""
    say("cr_coarsening on A^2: %s N=%d delta=%g" % (kind, N, delta))
    ad = lib()
    A = operator(kind, N)
    color = W.red_black((N, N))
    X = oracle.tv_init(A.n, 8, seed)
    X, _ = oracle.color_gs(A, X, color, 2, 5)
    Gh = oracle.power_pattern(A, 2)
    mu = oracle.algdist_graph(A, Gh, X)
    cf_ref, rho_ref, nc_ref = oracle.cr_coarsen(A, color, 2, mu, 0.25, nu=5, delta=delta,
                                                max_stages=20, seed=seed, G=Gh)
    Ad = dev_csr(A, torch.float64)
    G = ad.power_graph(Ad, 2)
    assert np.array_equal(to_np(G.row_ptr), Gh.row_ptr) and np.array_equal(to_np(G.col), Gh.col)
    cf, rho, nc = ad.cr_coarsening(Ad, gpu(color), 2, gpu(mu), 0.25, nu=5, delta=delta,
                                   max_stages=20, seed=seed, G=G)
    say("  stages %d |C| %s rho %s" % (len(rho_ref) - 1, list(nc_ref), np.round(rho_ref, 4).tolist()))
    assert np.array_equal(to_np(cf), cf_ref)
    assert nc == list(nc_ref)
    assert np.allclose(rho, rho_ref, rtol=1e-12, atol=0)
    # G = A's own pattern gives the plain call's result
    mu1 = gpu(oracle.algdist(A, X))
    c1, r1, _ = ad.cr_coarsening(Ad, gpu(color), 2, mu1, 0.25, seed=seed,
                                 G=ad.Pattern(Ad.row_ptr, Ad.col))
    c2, r2, _ = ad.cr_coarsening(Ad, gpu(color), 2, mu1, 0.25, seed=seed)
    assert torch.equal(c1, c2) and r1 == r2
    assert ad.status(clear=True) == 0


def test_cr_coarsening_from_a_given_c0_and_limits():
    ad = lib()
    N = 48
    A = aniso(N)
    color = W.red_black((N, N))
    X = oracle.tv_init(A.n, 8, 2)
    X, _ = oracle.color_gs(A, X, color, 2, 5)
    mu = oracle.algdist(A, X)
    c0 = np.zeros(A.n, np.uint8)
    c0[:: 17] = 1
    cf_ref, rho_ref, nc_ref = oracle.cr_coarsen(A, color, 2, mu, 0.25, max_stages=1, seed=4,
                                                cf0=c0)
    cf, rho, nc = ad.cr_coarsening(dev_csr(A, torch.float64), gpu(color), 2, gpu(mu), 0.25,
                                   max_stages=1, seed=4, cf=gpu(c0))
    assert np.array_equal(to_np(cf), cf_ref) and nc == list(nc_ref) and len(rho) == 2
    assert np.all(to_np(cf) >= c0)
    # delta above the first rate: nothing to do
    cf2, rho2, nc2 = ad.cr_coarsening(dev_csr(A, torch.float64), gpu(color), 2, gpu(mu), 0.25,
                                      delta=0.999, seed=4)
    assert len(rho2) == 1 and nc2 == [0] and torch.count_nonzero(cf2).item() == 0


def test_cr_coarsening_fp32_invariants():
    """FP32 operator and distances: the decisions may differ from the FP64
    chain's near their thresholds, so the loop's invariants are checked: C
    only grows, each stage adds an independent set of the candidates on its
    strength graph, and the loop ends below delta or at a stop rule."""
    ad = lib()
    N = 96
    A = aniso(N)
    color = W.red_black((N, N))
    Ad = dev_csr(A, torch.float32)
    X = ad.setup_testvectors(Ad, 8, seed=3, relax="gs", sweeps=5, color=gpu(color), ncolors=2)
    mu = ad.algebraic_distance(Ad, X)
    cf, rho, nc = ad.cr_coarsening(Ad, gpu(color), 2, mu, 0.25, seed=8)
    assert len(rho) >= 2 and rho[-1] <= 0.7
    assert all(b > a for a, b in zip(nc, nc[1:])) and nc[-1] == torch.count_nonzero(cf).item()
    A32 = W.CSR(A.n, A.row_ptr, A.col, A.val.astype(np.float32).astype(np.float64))
    r_ref, _ = oracle.cr_rate(A32, color, 2, to_np(cf), 5)
    assert rho[-1] == pytest.approx(r_ref, rel=1e-4)
