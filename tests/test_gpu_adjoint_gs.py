"""The gradient of the LS-interpolation loss through colour-phase Gauss-Seidel
test vectors and with respect to the LS weights, on the GPU: against the
oracle's gradient (every entry, and dL/dw), for two and four colours, a
9-point operator and non-symmetric values; checkpoint-interval invariance;
one colour against the damped-Jacobi path at omega = 1; dL/dw of the Jacobi
path; held rows; the autograd Function against central differences of the
GPU loss; and the full 512^2 log-normal operator."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1106_5990_amd import workloads as W
from gpu_common import lib, say, to_np

pytestmark = pytest.mark.gpu


def skewed(A, seed):
    rid = A.row_ids()
    f = 1.0 + 0.3 * np.random.default_rng(seed).random(A.nnz)
    return W.CSR(A.n, A.row_ptr, A.col, np.where(A.col != rid, A.val * f, A.val))


def gpu_loss_grad(A, K, seed, sweeps, color, nc, cf, cal, w, ce=1):
    ad = lib()
    vals = torch.as_tensor(A.val, dtype=torch.float64, device="cuda").requires_grad_(True)
    wt = torch.as_tensor(w, dtype=torch.float64, device="cuda").requires_grad_(True)
    rp = torch.as_tensor(A.row_ptr, device="cuda")
    col = torch.as_tensor(A.col, device="cuda")
    L = ad.LSInterpLossGS.apply(vals, wt, rp, col, K, seed, sweeps,
                                torch.as_tensor(color, device="cuda"), nc,
                                torch.as_tensor(cf, device="cuda"), cal, ce)
    gv, gw = torch.autograd.grad(L, (vals, wt))
    return float(L.detach()), to_np(gv), to_np(gw)


def check(g, gr, what):
    scale = np.abs(gr).max()
    err = np.abs(g - gr)
    say("  %s: max |dg| / max|g| = %.3g" % (what, err.max() / scale))
    assert np.all(err <= 1e-10 * np.maximum(np.abs(gr), 1e-3 * scale)), what


def case(kind):
    if kind == "aniso9-rb":
        N = 40
        A = skewed(W.rotated_anisotropic_9pt(N, 1e-2, math.pi / 6), 3)
        color, nc = W.red_black((N, N)), 2
    else:
        N = 36
        A = skewed(W.lognormal_2d_5pt(N, 1.0, 11), 5)
        color, nc = W.four_colour_2d(N), 4
    return A, color, nc, W.cf_red_is_coarse((N, N))


@pytest.mark.parametrize("kind", ["aniso9-rb", "lognormal-4c"])
@pytest.mark.parametrize("weighted", [False, True])
def test_gs_gradient_matches_oracle(kind, weighted):
    say("GS adjoint vs oracle %s weighted=%s" % (kind, weighted))
    A, color, nc, cf = case(kind)
    K, sweeps, cal = 16, 5, 4
    w = (0.5 + np.random.default_rng(2).random(K)) if weighted else np.ones(K)
    L, g, gw = gpu_loss_grad(A, K, 77, sweeps, color, nc, cf, cal, w, ce=2)
    Lr, gr, gwr = oracle.ls_loss_grad_gs(A, oracle.tv_init(A.n, K, 77), sweeps, color, nc,
                                         None if not weighted else w, cf, cal)
    say("  L %.12g vs %.12g" % (L, Lr))
    assert abs(L - Lr) <= 1e-12 * abs(Lr)
    check(g, gr, "dL/dvalues")
    assert np.allclose(gw, gwr, rtol=1e-10, atol=0), (gw, gwr)
    assert lib().status(clear=True) == 0


def test_gs_checkpoint_interval_does_not_change_the_gradient():
    A, color, nc, cf = case("lognormal-4c")
    ref = None
    for ce in (1, 2, 3, 5, 6):
        L, g, gw = gpu_loss_grad(A, 8, 4, 5, color, nc, cf, 4, np.ones(8), ce=ce)
        if ref is None:
            ref = (L, g, gw)
        assert L == ref[0] and np.array_equal(g, ref[1]) and np.array_equal(gw, ref[2]), ce


def test_one_colour_equals_jacobi_at_unit_damping_and_jacobi_weight_gradient():
    say("GS adjoint: one colour vs Jacobi; Jacobi dL/dw")
    ad = lib()
    N, K, sweeps = 30, 8, 4
    A = skewed(W.lognormal_2d_5pt(N, 1.0, 3), 8)
    cf = W.cf_red_is_coarse((N, N))
    one = np.zeros(A.n, np.int32)
    w = 0.5 + np.random.default_rng(4).random(K)
    L1, g1, gw1 = gpu_loss_grad(A, K, 9, sweeps, one, 1, cf, 4, w)
    vals = torch.as_tensor(A.val, dtype=torch.float64, device="cuda")
    Ad = ad.Csr(torch.as_tensor(A.row_ptr, device="cuda"), torch.as_tensor(A.col, device="cuda"),
                vals)
    ck = torch.empty((sweeps, A.n, K), dtype=torch.float64, device="cuda")
    X = ad.setup_testvectors(Ad, K, seed=9, relax="jacobi", sweeps=sweeps, omega=1.0, ckpt=ck,
                             ckpt_every=1)
    cft = torch.as_tensor(cf, device="cuda")
    wt = torch.as_tensor(w, device="cuda")
    _, _, _, Pc, Pv, ls, st, tot = ad.distance_ls(Ad, X, cft, 4, w=wt, fuse=False, want_sum=True)
    dL = torch.ones(1, dtype=torch.float64, device="cuda")
    gv, go, gw = ad.ls_interp_loss_grad(Ad, K, ck, 1, sweeps, cft, Pc, Pv, X, dL, relax="jacobi",
                                        omega=1.0, w=wt)
    assert abs(float(tot) - L1) <= 1e-12 * L1
    check(g1, to_np(gv), "one colour vs Jacobi")
    assert np.allclose(to_np(gw), gw1, rtol=1e-12, atol=0)
    gwr = oracle.ls_grad_w(A, to_np(X), w, cf, 4)
    assert np.allclose(to_np(gw), gwr, rtol=1e-10, atol=0)
    # the old entry point gives the same values and omega gradient
    gv2, go2 = ad.ls_interp_loss_backward(Ad, K, ck, 1, sweeps, 1.0, cft, Pc, Pv, X, dL, w=wt)
    assert torch.equal(gv2, gv) and torch.equal(go2.reshape(1), go.reshape(1))


def test_gs_gradient_with_held_rows():
    """Rows with an invalid colour are held by the sweeps: no phase moves
    them, so gradient reaches them only through A^T."""
    say("GS adjoint: held rows")
    N, K = 24, 8
    A = skewed(W.rotated_anisotropic_9pt(N, 0.05, 0.4), 6)
    color = W.red_black((N, N)).copy()
    color[[3, 100, 333]] = [-1, 5, 2]
    cf = W.cf_red_is_coarse((N, N))
    L, g, gw = gpu_loss_grad(A, K, 21, 3, color, 2, cf, 4, np.ones(K))
    Lr, gr, gwr = oracle.ls_loss_grad_gs(A, oracle.tv_init(A.n, K, 21), 3, color, 2, None, cf, 4)
    assert abs(L - Lr) <= 1e-12 * abs(Lr)
    check(g, gr, "held rows")
    assert np.allclose(gw, gwr, rtol=1e-10, atol=0)
    lib().status(clear=True)


def test_autograd_against_central_differences_of_the_gpu_loss():
    say("GS adjoint: central differences of the GPU loss")
    ad = lib()
    A, color, nc, cf = case("aniso9-rb")
    K, sweeps = 16, 4
    w = 0.5 + np.random.default_rng(9).random(K)
    L, g, gw = gpu_loss_grad(A, K, 5, sweeps, color, nc, cf, 4, w)
    rp = torch.as_tensor(A.row_ptr, device="cuda")
    col = torch.as_tensor(A.col, device="cuda")
    ct = torch.as_tensor(color, device="cuda")
    cft = torch.as_tensor(cf, device="cuda")

    def loss(vals, wv):
        v = torch.as_tensor(vals, dtype=torch.float64, device="cuda")
        return float(ad.LSInterpLossGS.apply(v, torch.as_tensor(wv, device="cuda"), rp, col, K, 5,
                                             sweeps, ct, nc, cft, 4))

    h = 1e-5
    rng = np.random.default_rng(3)
    for e in rng.choice(A.nnz, 12, replace=False):
        vp, vm = A.val.copy(), A.val.copy()
        hv = h * max(1.0, abs(A.val[e]))
        vp[e] += hv
        vm[e] -= hv
        fd = (loss(vp, w) - loss(vm, w)) / (2 * hv)
        assert abs(g[e] - fd) <= 1e-5 * abs(fd) + 1e-7 * np.abs(g).max(), e
    for k in range(0, K, 5):
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (loss(A.val, wp) - loss(A.val, wm)) / (2 * h)
        assert abs(gw[k] - fd) <= 1e-6 * abs(fd) + 1e-12, k


def test_full_size_four_colour_lognormal():
    """The 512^2 log-normal operator (workload 5's) relaxed by four colour
    phases, 6 sweeps, K = 16: every entry against the oracle.  (With the
    red-black colouring and C = red, a 5-point operator makes every F value
    an exact combination of its four C neighbours after each sweep, and the
    loss is rounding noise.)"""
    say("GS adjoint full size")
    w5 = W.workload(5)
    A = w5.A
    N = 512
    color = W.four_colour_2d(N)
    L, g, gw = gpu_loss_grad(A, w5.K, w5.tv_seed, w5.sweeps, color, 4, w5.cf, w5.caliber,
                             np.ones(w5.K), ce=2)
    Lr, gr, gwr = oracle.ls_loss_grad_gs(A, oracle.tv_init(A.n, w5.K, w5.tv_seed), w5.sweeps,
                                         color, 4, None, w5.cf, w5.caliber)
    say("  L %.12g vs %.12g" % (L, Lr))
    assert Lr > 1e-6
    assert abs(L - Lr) <= 1e-12 * abs(Lr)
    check(g, gr, "full size")
    assert np.allclose(gw, gwr, rtol=1e-10, atol=0)
