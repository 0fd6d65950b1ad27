"""Shared helpers of the GPU parity tests (imported only by `gpu` tests).

Tolerances (each derived from the arithmetic of the step it bounds):
* relaxation, FP64 end to end: |dx| <= 1e-12 max|x|;
* relaxation, FP32, one sweep from identical FP32 inputs:
  |dx_ik| <= 2^-23 ((nnz_i + 2) sum_j |a_ij z_jk| / |a_ii| + |x_ik|);
* mu, FP64: |dmu| <= 1e-10 mu + 1e-14 S_aa;  FP32: |dmu| <= 1e-4 mu + 1e-12 S_aa
  (S_aa = sum_k w_k t_k^2 of the row);
* strength mask and counts: bit-exact given the same mu;
* LS rows: columns and status bit-exact given the same mu; weights
  |dp| <= 1e-6 max(1, |p|); ls_val relative 1e-6 plus 1e-12 sum w t^2
  (both panel types: the normal equations are formed and solved in FP64).
"""
import sys

import numpy as np
import torch

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def lib():
    from paper_1106_5990_amd import algdist
    return algdist


def to_np(t):
    return t.detach().cpu().numpy()


def dev_csr(A, dtype):
    return lib().Csr.from_host(A, dtype=dtype)


def row_abs_bound(A, Z, X, omega, nnz_slack=2.0, eps=2.0 ** -23, rows=None):
    """Per-entry bound for one relaxation step in the panel precision:
    eps * ((nnz_i + 2) * omega * sum_j |a_ij z_j| / |a_ii| + |x_i|)."""
    rp = np.asarray(A.row_ptr, np.int64)
    rows = np.arange(A.n) if rows is None else np.asarray(rows)
    out = np.empty((len(rows), Z.shape[1]))
    for r, i in enumerate(rows):
        s, e = rp[i], rp[i + 1]
        cols = A.col[s:e]
        a = A.val[s:e]
        d = abs(a[cols == i][0])
        acc = (np.abs(a)[:, None] * np.abs(Z[cols])).sum(0)
        out[r] = eps * ((e - s + nnz_slack) * omega * acc / d + np.abs(X[i]))
    return out


def saa_per_edge(A, T, w=None):
    """S_aa = sum_k w_k t_ik^2 of each entry's row."""
    w = np.ones(T.shape[1]) if w is None else np.asarray(w)
    saa = (T * T * w).sum(1)
    return saa[A.row_ids()]


def residual_target(A, X):
    """t_i = x_i - (A x)_i / a_ii in FP64 (rows with a zero diagonal keep x_i)."""
    import scipy.sparse as sp
    S = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
    d = S.diagonal()
    Y = S @ X
    T = X.copy()
    nz = d != 0
    T[nz] = X[nz] - Y[nz] / d[nz][:, None]
    return T


def check_mu(mu_gpu, mu_ref, saa, dtype, what=""):
    if dtype == torch.float32:
        rtol, afl = 1e-4, 1e-12
    else:
        rtol, afl = 1e-10, 1e-14
    err = np.abs(mu_gpu - mu_ref)
    lim = rtol * np.abs(mu_ref) + afl * saa
    bad = np.nonzero(err > lim)[0]
    floor_only = int(np.count_nonzero((err > rtol * np.abs(mu_ref)) & (err <= lim)))
    say("  mu %s: max rel err %.3g, edges passing only by the floor: %d"
        % (what, float(np.max(err / np.maximum(np.abs(mu_ref), 1e-300))) if len(err) else 0.0,
           floor_only))
    assert len(bad) == 0, "mu mismatch at %s: gpu %s ref %s" % (
        bad[:5], mu_gpu[bad[:5]], mu_ref[bad[:5]])


def check_ls(gpu, ref, dtype, wsum_tt):
    Pc, Pv, ls, st = gpu
    Rc, Rv, Rl, Rs = ref
    assert np.array_equal(Pc, Rc), "P_col differ at rows %s" % np.nonzero((Pc != Rc).any(1))[0][:5]
    assert np.array_equal(st, Rs), "row_status differ at %s" % np.nonzero(st != Rs)[0][:5]
    tol = 1e-6
    perr = np.abs(Pv - Rv) / np.maximum(1.0, np.abs(Rv))
    say("  P_val max scaled err %.3g" % (perr.max() if perr.size else 0))
    assert np.all(perr <= tol), "P_val differ at rows %s" % np.nonzero((perr > tol).any(1))[0][:5]
    lerr = np.abs(ls - Rl)
    lim = tol * np.abs(Rl) + 1e-12 * wsum_tt
    assert np.all(lerr <= lim), "ls_val differ at rows %s" % np.nonzero(lerr > lim)[0][:5]
