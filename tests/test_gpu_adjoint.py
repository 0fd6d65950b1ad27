"""The adjoint of the LS interpolation loss on the GPU: against the oracle's
gradient (every entry), against central finite differences of the GPU loss
at the full 512^2 size (omega, sampled entries including diagonals and
boundary rows, random directions), checkpoint-interval invariance and the
torch.autograd.Function."""
import numpy as np
import pytest
import torch

import oracle
from paper_1106_5990_amd import workloads as W
from gpu_common import lib, say, to_np

pytestmark = pytest.mark.gpu


def skewed(A, seed):
    """Same pattern, values made non-symmetric (a_ij != a_ji)."""
    rid = A.row_ids()
    f = 1.0 + 0.3 * np.random.default_rng(seed).random(A.nnz)
    return W.CSR(A.n, A.row_ptr, A.col, np.where(A.col != rid, A.val * f, A.val))


def gpu_loss_and_grad(A, K, seed, sweeps, omega, cf, cal, w=None, ce=2):
    ad = lib()
    vals = torch.as_tensor(A.val, dtype=torch.float64, device="cuda").requires_grad_(True)
    om = torch.tensor(omega, dtype=torch.float64, device="cuda", requires_grad=True)
    rp = torch.as_tensor(A.row_ptr, device="cuda")
    col = torch.as_tensor(A.col, device="cuda")
    cft = torch.as_tensor(cf, device="cuda")
    wt = None if w is None else torch.as_tensor(w, device="cuda")
    L = ad.LSInterpLoss.apply(vals, om, rp, col, K, seed, sweeps, cft, cal, ce, wt)
    gv, go = torch.autograd.grad(L, (vals, om))
    return float(L.detach()), to_np(gv), float(go)


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("skew", [False, True])
def test_adjoint_matches_oracle(weighted, skew):
    say("adjoint vs oracle weighted=%s skew=%s" % (weighted, skew))
    N, K, sweeps, omega, cal = 40, 16, 6, 0.7, 4
    A = W.lognormal_2d_5pt(N, 1.0, 5995)
    if skew:
        A = skewed(A, 3)
    cf = W.cf_red_is_coarse((N, N))
    w = (0.5 + np.random.default_rng(1).random(K)) if weighted else None
    L, g, gw = gpu_loss_and_grad(A, K, 1111, sweeps, omega, cf, cal, w)
    Lr, gr, gwr = oracle.ls_loss_grad(A, oracle.tv_init(A.n, K, 1111), sweeps, omega, w, cf, cal)
    say("  L %.12g vs %.12g; domega %.12g vs %.12g" % (L, Lr, gw, gwr))
    assert abs(L - Lr) <= 1e-12 * abs(Lr)
    assert abs(gw - gwr) <= 1e-10 * abs(gwr)
    scale = np.abs(gr).max()
    err = np.abs(g - gr)
    say("  max |dg| / max|g| = %.3g" % (err.max() / scale))
    assert np.all(err <= 1e-10 * np.maximum(np.abs(gr), 1e-3 * scale))
    assert lib().status(clear=True) == 0


def test_checkpoint_interval_does_not_change_the_gradient():
    say("adjoint checkpoint intervals")
    N, K = 32, 8
    A = skewed(W.lognormal_2d_5pt(N, 1.0, 7), 9)
    cf = W.cf_red_is_coarse((N, N))
    ref = None
    for ce in (1, 2, 3, 6, 7):
        L, g, gw = gpu_loss_and_grad(A, K, 5, 6, 0.6, cf, 4, ce=ce)
        if ref is None:
            ref = (L, g, gw)
        assert L == ref[0] and np.array_equal(g, ref[1]) and gw == ref[2], ce


def test_zero_sweeps():
    ad = lib()
    say("adjoint: zero sweeps")
    N, K = 12, 4
    A = W.lognormal_2d_5pt(N, 1.0, 2)
    cf = W.cf_red_is_coarse((N, N))
    L, g, gw = gpu_loss_and_grad(A, K, 3, 0, 0.5, cf, 4)
    Lr, gr, gwr = oracle.ls_loss_grad(A, oracle.tv_init(A.n, K, 3), 0, 0.5, None, cf, 4)
    assert abs(L - Lr) <= 1e-12 * Lr and np.all(g == 0) and gw == 0.0 and np.all(gr == 0)
    assert ad.status(clear=True) == 0


def drop_entries(A, rows, seed):
    """A with one off-diagonal entry removed from each of `rows` (chosen at
    random in the row): the pattern is no longer structurally symmetric."""
    rng = np.random.default_rng(seed)
    rid = A.row_ids()
    keep = np.ones(A.nnz, bool)
    for r in rows:
        offd = np.nonzero((rid == r) & (A.col != r))[0]
        keep[rng.choice(offd)] = False
    counts = np.bincount(rid[keep], minlength=A.n)
    rp = np.concatenate([[0], np.cumsum(counts)]).astype(A.row_ptr.dtype)
    return W.CSR(A.n, rp, A.col[keep], A.val[keep])


@pytest.mark.parametrize("skew", [False, True])
def test_adjoint_asymmetric_pattern_matches_oracle(skew):
    """Entries (i, j) without (j, i): A^T y and the transpose of P gather
    through the column-major index, so every gradient entry still matches the
    oracle (which scatters over the stored entries directly)."""
    ad = lib()
    say("adjoint: structurally asymmetric pattern, skew=%s" % skew)
    N, K, sweeps, omega, cal = 24, 8, 4, 0.7, 4
    A = W.lognormal_2d_5pt(N, 1.0, 41)
    A = drop_entries(A, np.random.default_rng(5).choice(A.n, A.n // 3, replace=False), 6)
    if skew:
        A = skewed(A, 8)
    cf = W.cf_red_is_coarse((N, N))
    L, g, gw = gpu_loss_and_grad(A, K, 77, sweeps, omega, cf, cal)
    Lr, gr, gwr = oracle.ls_loss_grad(A, oracle.tv_init(A.n, K, 77), sweeps, omega, None, cf, cal)
    say("  L %.12g vs %.12g; domega %.12g vs %.12g" % (L, Lr, gw, gwr))
    assert abs(L - Lr) <= 1e-12 * abs(Lr)
    assert abs(gw - gwr) <= 1e-10 * abs(gwr)
    scale = np.abs(gr).max()
    err = np.abs(g - gr)
    say("  max |dg| / max|g| = %.3g" % (err.max() / scale))
    assert np.all(err <= 1e-10 * np.maximum(np.abs(gr), 1e-3 * scale))
    assert ad.status(clear=True) == 0


def test_adjoint_against_central_differences_full_size():
    """Workload 5 at full size (512^2 log-normal 5-point, K = 16, 6 sweeps,
    learnable omega, checkpoints every 2 sweeps): central differences on
    omega, 4096 sampled entries (diagonals and boundary rows included) and 16
    random directions, at two steps:
      h = 1e-6 max(1, |theta|) and h = 1e-4 max(1, |theta|):
      |g - g_FD| <= 1e-5 |g_FD| + 1e-9 max|g| + 4 eps |L| / h.
    The last term is the rounding floor of a central difference of a loss
    evaluated to relative precision ~eps (2 eps |L| / (2 h), doubled); here
    L ~ 270 while max|g| ~ 0.07, so for h = 1e-6 it dominates and the larger
    step gives the sharper check (its truncation error is O(h^2))."""
    ad = lib()
    wl = W.workload(5)
    A = wl.A
    say("adjoint FD, workload %s" % wl.name)
    K, sweeps, omega, cal = wl.K, wl.sweeps, wl.omega, wl.caliber
    dev = "cuda"
    rp = torch.as_tensor(A.row_ptr, device=dev)
    col = torch.as_tensor(A.col, device=dev)
    cf = torch.as_tensor(wl.cf, device=dev)
    v0 = torch.as_tensor(A.val, dtype=torch.float64, device=dev)
    nck = -(-sweeps // 2)
    ck = torch.empty((nck, A.n, K), dtype=torch.float64, device=dev)
    X = torch.empty((A.n, K), dtype=torch.float64, device=dev)
    mu = torch.empty(A.nnz, dtype=torch.float64, device=dev)
    outs = [torch.empty((A.n, cal), dtype=torch.int32, device=dev),
            torch.empty((A.n, cal), dtype=torch.float64, device=dev),
            torch.empty(A.n, dtype=torch.float64, device=dev),
            torch.empty(A.n, dtype=torch.int32, device=dev),
            torch.empty(1, dtype=torch.float64, device=dev)]

    def loss(vals, om):
        Ad = ad.Csr(rp, col, vals)
        ad.setup_testvectors(Ad, K, seed=wl.tv_seed, relax="jacobi", sweeps=sweeps, omega=om,
                             out=X, ckpt=ck, ckpt_every=2)
        ad.algebraic_distance(Ad, X, mu=mu)
        ad.ls_interp(Ad, X, cf, mu, cal, P_col=outs[0], P_val=outs[1], ls_val=outs[2],
                     row_status=outs[3], ls_sum=outs[4], want_sum=True)
        return float(outs[4])

    L0 = loss(v0, omega)
    Ad = ad.Csr(rp, col, v0)
    one = torch.ones(1, dtype=torch.float64, device=dev)
    g, gw = ad.ls_interp_loss_backward(Ad, K, ck, 2, sweeps, omega, cf, outs[0], outs[1], X, one)
    g = to_np(g)
    gw = float(gw)
    gmax = np.abs(g).max()
    say("  L = %.10g, dL/domega = %.10g, max|g| = %.4g" % (L0, gw, gmax))

    eps = np.finfo(np.float64).eps

    def check(fd, an, what, h):
        lim = 1e-5 * abs(fd) + 1e-9 * gmax + 4 * eps * abs(L0) / h
        assert abs(an - fd) <= lim, "%s (h=%g): adjoint %.10g FD %.10g" % (what, h, an, fd)
        return abs(an - fd) / lim

    for rel in (1e-6, 1e-4):
        h = rel * max(1.0, abs(omega))
        check((loss(v0, omega + h) - loss(v0, omega - h)) / (2 * h), gw, "omega", h)
    rng = np.random.default_rng(0)
    rid = A.row_ids()
    diag = np.nonzero(A.col == rid)[0]
    N = A.grid[0]
    iy, ix = np.divmod(rid, N)
    boundary = np.nonzero((ix == 0) | (iy == 0) | (ix == N - 1) | (iy == N - 1))[0]
    sample = np.unique(np.concatenate([rng.choice(A.nnz, 3584, replace=False),
                                       rng.choice(diag, 256, replace=False),
                                       rng.choice(boundary, 256, replace=False)]))
    for rel in (1e-6, 1e-4):
        worst = 0.0
        for e in sample:
            he = rel * max(1.0, abs(A.val[e]))
            vp = v0.clone()
            vp[e] += he
            vm = v0.clone()
            vm[e] -= he
            fd = (loss(vp, omega) - loss(vm, omega)) / (2 * he)
            worst = max(worst, check(fd, g[e], "entry %d" % e, he))
        say("  h=%g: %d entries, worst err / bound = %.3g" % (rel, len(sample), worst))
    for q in range(16):
        d = rng.standard_normal(A.nnz)
        dw = rng.standard_normal()
        dt = torch.as_tensor(d, device=dev)
        for hd in (1e-6, 1e-4):
            fd = (loss(v0 + hd * dt, omega + hd * dw) - loss(v0 - hd * dt, omega - hd * dw)) / (2 * hd)
            an = float(g @ d + gw * dw)
            check(fd, an, "direction %d" % q, hd)
    assert ad.status(clear=True) == 0
