"""Pins of the oracle's gradient of the LS-interpolation loss through
colour-phase Gauss-Seidel test vectors and with respect to the LS weights
w_k (Sec. 3 test vectors, Sec. 3.1 eq:LSfuncrowi, Sec. 5.2 Gauss-Seidel):
one colour is damped Jacobi with omega = 1 (whose adjoint is pinned
separately), central differences in the matrix values and in w (the latter
refits p, so it also checks that p's own variation drops out), and a
directional Taylor test whose remainder is second order."""
import math

import numpy as np
import pytest

import oracle
from paper_1106_5990_amd import workloads as W


def skewed(A, seed):
    """a_ij != a_ji off the diagonal: A and A^T play different parts."""
    rid = A.row_ids()
    skew = 1.0 + 0.4 * np.random.default_rng(seed).random(A.nnz)
    return W.CSR(A.n, A.row_ptr, A.col, np.where(A.col != rid, A.val * skew, A.val))


def case(kind):
    if kind == "aniso9-rb":
        N = 7
        A = skewed(W.rotated_anisotropic_9pt(N, 0.05, math.pi / 5), 3)
        color, nc = W.red_black((N, N)), 2
    else:  # log-normal 5-point with a four-colouring
        N = 8
        A = skewed(W.lognormal_2d_5pt(N, 1.0, 2), 4)
        color, nc = W.four_colour_2d(N), 4
    cf = W.cf_red_is_coarse((N, N))
    X0 = oracle.tv_init(A.n, 4, 17)
    w = np.array([1.0, 0.5, 2.0, 1.5])
    return A, X0, color, nc, cf, w


def test_one_colour_is_jacobi_with_unit_damping():
    A, X0, _, _, cf, w = case("aniso9-rb")
    one = np.zeros(A.n, np.int32)
    L, g, gw = oracle.ls_loss_grad_gs(A, X0, 3, one, 1, w, cf, 4)
    Lj, gj, _ = oracle.ls_loss_grad(A, X0, 3, 1.0, w, cf, 4)
    assert L == pytest.approx(Lj, rel=1e-13)
    assert np.max(np.abs(g - gj)) <= 1e-12 * np.max(np.abs(gj))
    X = X0.copy()
    X, _ = oracle.jacobi(A, X, 1.0, 3)
    assert np.allclose(gw, oracle.ls_grad_w(A, X, w, cf, 4), rtol=1e-13, atol=0)


@pytest.mark.parametrize("kind", ["aniso9-rb", "lognormal-4c"])
def test_gs_adjoint_matches_central_differences(kind):
    A, X0, color, nc, cf, w = case(kind)
    sweeps, cal = 3, 4
    L, g, gw = oracle.ls_loss_grad_gs(A, X0, sweeps, color, nc, w, cf, cal)
    assert L > 1e-8
    assert L == pytest.approx(oracle.ls_loss_gs(A, X0, sweeps, color, nc, w, cf, cal), rel=1e-14)
    h = 1e-6
    rng = np.random.default_rng(1)
    for e in list(rng.choice(A.nnz, 30, replace=False)) + [0, int(A.row_ptr[9]) + 1]:
        hv = h * max(1.0, abs(A.val[e]))
        vp, vm = A.val.copy(), A.val.copy()
        vp[e] += hv
        vm[e] -= hv
        fd = (oracle.ls_loss_gs(A, X0, sweeps, color, nc, w, cf, cal, val=vp)
              - oracle.ls_loss_gs(A, X0, sweeps, color, nc, w, cf, cal, val=vm)) / (2 * hv)
        assert abs(g[e] - fd) <= 1e-5 * abs(fd) + 1e-8 * np.abs(g).max(), e
    # the weights: p is refitted by each evaluation
    for k in range(len(w)):
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (oracle.ls_loss_gs(A, X0, sweeps, color, nc, wp, cf, cal)
              - oracle.ls_loss_gs(A, X0, sweeps, color, nc, wm, cf, cal)) / (2 * h)
        assert abs(gw[k] - fd) <= 1e-6 * abs(fd) + 1e-12, k


def test_gs_adjoint_taylor_remainder_is_second_order():
    A, X0, color, nc, cf, w = case("lognormal-4c")
    L, g, gw = oracle.ls_loss_grad_gs(A, X0, 2, color, nc, w, cf, 4)
    rng = np.random.default_rng(2)
    d = rng.standard_normal(A.nnz)
    dw = rng.standard_normal(len(w))
    rem = []
    for h in (1e-2, 5e-3, 2.5e-3):
        Lh = oracle.ls_loss_gs(A, X0, 2, color, nc, w + h * dw, cf, 4, val=A.val + h * d)
        rem.append(abs(Lh - L - h * (g @ d + gw @ dw)))
    assert rem[1] / rem[0] < 0.3 and rem[2] / rem[1] < 0.3
