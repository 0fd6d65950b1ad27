"""Python access to the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  It does not
import the GPU package; matrices are passed as any object with `n`,
`row_ptr`, `col` and `val` attributes (or as explicit arrays).

Each function is the definition written out in oracle.c; see the comments
there for the paper passage it follows.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

TARGET_PLAIN = 0
TARGET_RESIDUAL = 1

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build()
        L = C.CDLL(path)
        P = C.c_void_p
        i32, i64, u64, f64 = C.c_int, C.c_int64, C.c_uint64, C.c_double
        sig = {
            "oracle_splitmix64_nth": (u64, [u64, u64]),
            "oracle_tv_init": (None, [i64, i64, i32, u64, P]),
            "oracle_jacobi": (i32, [i32, P, P, P, i32, f64, i32, P]),
            "oracle_jacobi_rows": (None, [i32, P, P, P, i32, f64, P, i32, P, P]),
            "oracle_color_gs": (i32, [i32, P, P, P, i32, P, i32, i32, P]),
            "oracle_color_gs_rows": (None, [i32, P, P, P, i32, P, i32, P, P, i32, P, P]),
            "oracle_algdist": (i32, [i32, P, P, P, i32, P, P, i32, i32, P, P, P]),
            "oracle_strength": (None, [i32, P, P, P, f64, P, P, P]),
            "oracle_ls_interp": (None, [i32, P, P, P, i32, P, P, P, P, i32, i32, i32, P, P, P, P, P]),
            "oracle_ls_loss": (f64, [i32, P, P, P, i32, P, i32, f64, P, P, i32]),
            "oracle_ls_loss_grad": (f64, [i32, P, P, P, i32, P, i32, f64, P, P, i32, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _csr(A):
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col, dtype=np.int32)
    va = np.ascontiguousarray(A.val, dtype=np.float64)
    return int(A.n), rp, ci, va


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _rows(rows):
    return None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)


def splitmix64_nth(seed: int, n: int) -> int:
    return int(lib().oracle_splitmix64_nth(seed & (2**64 - 1), n))


def tv_init(nrows: int, K: int, seed: int, row0: int = 0) -> np.ndarray:
    X = np.empty((nrows, K), dtype=np.float64)
    lib().oracle_tv_init(row0, nrows, K, seed & (2**64 - 1), _p(X))
    return X


def jacobi(A, X0, omega: float, sweeps: int):
    n, rp, ci, va = _csr(A)
    X = _f64(X0).copy()
    K = X.shape[1]
    z = lib().oracle_jacobi(n, _p(rp), _p(ci), _p(va), K, float(omega), int(sweeps), _p(X))
    return X, z


def jacobi_rows(A, X, omega: float, rows):
    n, rp, ci, va = _csr(A)
    X = _f64(X)
    rows = _rows(rows)
    out = np.empty((len(rows), X.shape[1]))
    lib().oracle_jacobi_rows(n, _p(rp), _p(ci), _p(va), X.shape[1], float(omega), _p(X),
                             len(rows), _p(rows), _p(out))
    return out


def color_gs(A, X0, color, ncolors: int, sweeps: int):
    n, rp, ci, va = _csr(A)
    X = _f64(X0).copy()
    col = np.ascontiguousarray(color, dtype=np.int32)
    h = lib().oracle_color_gs(n, _p(rp), _p(ci), _p(va), X.shape[1], _p(col), int(ncolors),
                              int(sweeps), _p(X))
    return X, h


def color_gs_rows(A, color, ncolors: int, Xold, Xnew, rows):
    n, rp, ci, va = _csr(A)
    Xold, Xnew = _f64(Xold), _f64(Xnew)
    col = np.ascontiguousarray(color, dtype=np.int32)
    rows = _rows(rows)
    out = np.empty((len(rows), Xold.shape[1]))
    lib().oracle_color_gs_rows(n, _p(rp), _p(ci), _p(va), Xold.shape[1], _p(col), int(ncolors),
                               _p(Xold), _p(Xnew), len(rows), _p(rows), _p(out))
    return out


def packed_len(A, rows) -> int:
    rp = np.asarray(A.row_ptr, dtype=np.int64)
    if rows is None:
        return int(rp[-1])
    rows = np.asarray(rows, dtype=np.int64)
    return int((rp[rows + 1] - rp[rows]).sum())


def algdist(A, X, w=None, target: int = TARGET_PLAIN, rows=None, want_p: bool = False):
    """mu (and p) per stored entry of the selected rows, packed in row order."""
    n, rp, ci, va = _csr(A)
    X = _f64(X)
    w = None if w is None else _f64(w)
    r = _rows(rows)
    m = packed_len(A, rows)
    mu = np.empty(m)
    p = np.empty(m) if want_p else None
    bad = lib().oracle_algdist(n, _p(rp), _p(ci), _p(va), X.shape[1], _p(X), _p(w), int(target),
                               0 if r is None else len(r), _p(r), _p(mu), _p(p))
    return (mu, p, bad) if want_p else mu


def strength(A, mu, theta: float, fmask=None):
    n, rp, ci, va = _csr(A)
    mu = _f64(mu)
    fm = None if fmask is None else np.ascontiguousarray(fmask, dtype=np.uint8)
    strong = np.empty(len(ci), dtype=np.uint8)
    ns = np.empty(n, dtype=np.int32)
    lib().oracle_strength(n, _p(rp), _p(ci), _p(mu), float(theta), _p(fm), _p(strong), _p(ns))
    return strong, ns


def ls_interp(A, X, w, cf, mu, caliber: int, target: int = TARGET_PLAIN, rows=None):
    n, rp, ci, va = _csr(A)
    X = _f64(X)
    w = None if w is None else _f64(w)
    cf = np.ascontiguousarray(cf, dtype=np.uint8)
    mu = _f64(mu)
    r = _rows(rows)
    m = n if r is None else len(r)
    Pc = np.empty((m, caliber), dtype=np.int32)
    Pv = np.empty((m, caliber))
    ls = np.empty(m)
    st = np.empty(m, dtype=np.int32)
    lib().oracle_ls_interp(n, _p(rp), _p(ci), _p(va), X.shape[1], _p(X), _p(w), _p(cf), _p(mu),
                           int(caliber), int(target), 0 if r is None else len(r), _p(r),
                           _p(Pc), _p(Pv), _p(ls), _p(st))
    return Pc, Pv, ls, st


def ls_loss(A, X0, sweeps: int, omega: float, w, cf, caliber: int, val=None) -> float:
    n, rp, ci, va = _csr(A)
    if val is not None:
        va = _f64(val)
    X0 = _f64(X0)
    w = None if w is None else _f64(w)
    cf = np.ascontiguousarray(cf, dtype=np.uint8)
    return float(lib().oracle_ls_loss(n, _p(rp), _p(ci), _p(va), X0.shape[1], _p(X0), int(sweeps),
                                      float(omega), _p(w), _p(cf), int(caliber)))


def ls_loss_grad(A, X0, sweeps: int, omega: float, w, cf, caliber: int):
    n, rp, ci, va = _csr(A)
    X0 = _f64(X0)
    w = None if w is None else _f64(w)
    cf = np.ascontiguousarray(cf, dtype=np.uint8)
    g = np.empty(len(ci))
    gw = C.c_double(0.0)
    L = lib().oracle_ls_loss_grad(n, _p(rp), _p(ci), _p(va), X0.shape[1], _p(X0), int(sweeps),
                                  float(omega), _p(w), _p(cf), int(caliber), _p(g), C.byref(gw))
    return float(L), g, float(gw.value)


# ---------------------------------------------------------------- long range
def _sig_longrange(L):
    P = C.c_void_p
    i32, i64, f64 = C.c_int, C.c_int64, C.c_double
    for name, res, args in (
            ("oracle_power_counts", i64, [i32, P, P, i32, P]),
            ("oracle_power_fill", None, [i32, P, P, i32, P, P]),
            ("oracle_algdist_graph", i32, [i32, P, P, P, P, P, i32, P, P, i32, i32, P, P, P]),
            ("oracle_ls_fit_sets", None, [i32, P, P, P, i32, P, P, i32, i32, i32, P, P, P, P, P]),
            ("oracle_ls_search", None, [i32, P, P, P, P, P, i32, P, P, P, i32, f64, i32, i32, P,
                                        P, P, P, P, P, P])):
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


class Pattern:
    """A sparsity pattern in CSR form (row_ptr, col), no values."""

    def __init__(self, n, row_ptr, col):
        self.n = int(n)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)

    @property
    def nnz(self):
        return int(self.row_ptr[-1])

    def row_ids(self):
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))


def power_pattern(A, d: int) -> Pattern:
    """Structural pattern of A^d (eq. graph): per row, the vertices within
    graph distance d, sorted."""
    L = _sig_longrange(lib())
    n, rp, ci, _ = _csr(A)
    cnt = np.empty(n, dtype=np.int32)
    L.oracle_power_counts(n, _p(rp), _p(ci), int(d), _p(cnt))
    rpd = np.concatenate([[0], np.cumsum(cnt, dtype=np.int64)])
    assert rpd[-1] < 2 ** 31
    rpd = rpd.astype(np.int32)
    cid = np.empty(int(rpd[-1]), dtype=np.int32)
    L.oracle_power_fill(n, _p(rp), _p(ci), int(d), _p(rpd), _p(cid))
    return Pattern(n, rpd, cid)


def algdist_graph(A, G, X, w=None, target: int = TARGET_PLAIN, rows=None, want_p: bool = False):
    """mu (and p) per entry of the pattern G (e.g. power_pattern(A, d)), the
    targets formed from A; packed in row order over the selected rows."""
    L = _sig_longrange(lib())
    n, rp, ci, va = _csr(A)
    X = _f64(X)
    w = None if w is None else _f64(w)
    r = _rows(rows)
    m = packed_len(G, rows)
    mu = np.empty(m)
    p = np.empty(m) if want_p else None
    L.oracle_algdist_graph(n, _p(rp), _p(ci), _p(va), _p(G.row_ptr), _p(G.col), X.shape[1], _p(X),
                           _p(w), int(target), 0 if r is None else len(r), _p(r), _p(mu), _p(p))
    return (mu, p) if want_p else mu


def ls_fit_sets(A, X, w, sets, rows, target: int = TARGET_PLAIN):
    """LS fit of each row of `rows` by its given set (row r of `sets`, -1
    padded): (P_val, ls_val, rankdef)."""
    L = _sig_longrange(lib())
    n, rp, ci, va = _csr(A)
    X = _f64(X)
    w = None if w is None else _f64(w)
    sets = np.ascontiguousarray(sets, dtype=np.int32)
    r = _rows(rows)
    cal = sets.shape[1]
    Pv = np.empty((len(r), cal))
    ls = np.empty(len(r))
    rd = np.empty(len(r), dtype=np.int32)
    L.oracle_ls_fit_sets(n, _p(rp), _p(ci), _p(va), X.shape[1], _p(X), _p(w), int(target), cal,
                         len(r), _p(r), _p(sets), _p(Pv), _p(ls), _p(rd))
    return Pv, ls, rd


def ls_search(A, G, X, w, cf, caliber: int, gamma: float = 1.5, target: int = TARGET_PLAIN,
              rows=None):
    """Interpolatory sets by search over the C-points of G's rows (Sec. 4.3):
    (P_col, P_val, ls_val, status, best, ncand); best[r] = (S, best_1/S, ...,
    best_caliber/S)."""
    L = _sig_longrange(lib())
    n, rp, ci, va = _csr(A)
    X = _f64(X)
    w = None if w is None else _f64(w)
    cf = np.ascontiguousarray(cf, dtype=np.uint8)
    r = _rows(rows)
    m = n if r is None else len(r)
    Pc = np.empty((m, caliber), dtype=np.int32)
    Pv = np.empty((m, caliber))
    ls = np.empty(m)
    st = np.empty(m, dtype=np.int32)
    best = np.empty((m, caliber + 1))
    nc = np.empty(m, dtype=np.int32)
    L.oracle_ls_search(n, _p(rp), _p(ci), _p(va), _p(G.row_ptr), _p(G.col), X.shape[1], _p(X),
                       _p(w), _p(cf), int(caliber), float(gamma), int(target),
                       0 if r is None else len(r), _p(r), _p(Pc), _p(Pv), _p(ls), _p(st),
                       _p(best), _p(nc))
    return Pc, Pv, ls, st, best, nc


def _sig_cr(L):
    P = C.c_void_p
    i32, u64, f64 = C.c_int, C.c_uint64, C.c_double
    for name, res, args in (
            ("oracle_cr_rate", f64, [i32, P, P, P, P, i32, P, i32, P]),
            ("oracle_cr_candidates", None, [i32, P, P, f64, P]),
            ("oracle_independent_set", i32, [i32, P, P, P, P, u64, P]),
            ("oracle_cr_coarsen", i32, [i32, P, P, P, P, i32, P, f64, i32, f64, i32, u64, P, P,
                                        P]),
            ("oracle_cr_coarsen_graph", i32, [i32, P, P, P, P, P, P, i32, P, f64, i32, f64, i32,
                                              u64, P, P, P])):
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


def cr_rate(A, color, ncolors: int, cf, nu: int):
    """nu F-relaxation sweeps (eq:frelax) from the constant start, C held at
    zero: (rho_f of eq:meas1, u^nu)."""
    L = _sig_cr(lib())
    n, rp, ci, va = _csr(A)
    col = np.ascontiguousarray(color, dtype=np.int32)
    cf = np.ascontiguousarray(cf, dtype=np.uint8)
    u = np.empty(n)
    r = L.oracle_cr_rate(n, _p(rp), _p(ci), _p(va), _p(col), int(ncolors), _p(cf), int(nu), _p(u))
    return float(r), u


def cr_candidates(cf, u, tol: float):
    """F points with |u_i| / max_F |u| > tol."""
    L = _sig_cr(lib())
    cf = np.ascontiguousarray(cf, dtype=np.uint8)
    u = _f64(u)
    z = np.empty(len(cf), dtype=np.uint8)
    L.oracle_cr_candidates(len(cf), _p(cf), _p(u), float(tol), _p(z))
    return z


def independent_set(A, strong, z, seed: int):
    """Greedy maximal independent set of the candidates z on the symmetric
    closure of the strong graph, in decreasing (|S_i^T|, hash, index)."""
    L = _sig_cr(lib())
    n, rp, ci, _ = _csr(A)
    strong = np.ascontiguousarray(strong, dtype=np.uint8)
    z = np.ascontiguousarray(z, dtype=np.uint8)
    sel = np.empty(n, dtype=np.uint8)
    L.oracle_independent_set(n, _p(rp), _p(ci), _p(strong), _p(z), seed & (2**64 - 1), _p(sel))
    return sel


def cr_coarsen(A, color, ncolors: int, mu, theta: float, nu: int = 5, delta: float = 0.7,
               max_stages: int = 20, seed: int = 0, cf0=None, G=None):
    """Algorithm 1 of Sec. 4.2: (cf, rho per stage, |C| per stage).  With a
    pattern G (e.g. power_pattern(A, d)) the strength graph M^d and the
    independent set live on G, mu given per entry of G; CR relaxes with A."""
    L = _sig_cr(lib())
    n, rp, ci, va = _csr(A)
    col = np.ascontiguousarray(color, dtype=np.int32)
    mu = _f64(mu)
    cf = (np.zeros(n, dtype=np.uint8) if cf0 is None
          else np.ascontiguousarray(cf0, dtype=np.uint8).copy())
    rho = np.zeros(max_stages + 1)
    nc = np.zeros(max_stages + 1, dtype=np.int64)
    if G is None:
        s = L.oracle_cr_coarsen(n, _p(rp), _p(ci), _p(va), _p(col), int(ncolors), _p(mu),
                                float(theta), int(nu), float(delta), int(max_stages),
                                seed & (2**64 - 1), _p(cf), _p(rho), _p(nc))
    else:
        rpg = np.ascontiguousarray(G.row_ptr, dtype=np.int32)
        cig = np.ascontiguousarray(G.col, dtype=np.int32)
        assert len(mu) == len(cig)
        s = L.oracle_cr_coarsen_graph(n, _p(rp), _p(ci), _p(va), _p(rpg), _p(cig), _p(col),
                                      int(ncolors), _p(mu), float(theta), int(nu), float(delta),
                                      int(max_stages), seed & (2**64 - 1), _p(cf), _p(rho),
                                      _p(nc))
    return cf, rho[:s + 1], nc[:s + 1]


def _sig_gs_grad(L):
    P = C.c_void_p
    i32, f64 = C.c_int, C.c_double
    for name, res, args in (
            ("oracle_ls_loss_gs", f64, [i32, P, P, P, i32, P, i32, P, i32, P, P, i32]),
            ("oracle_ls_grad_w", None, [i32, P, P, P, i32, P, P, P, i32, P]),
            ("oracle_ls_loss_grad_gs", f64, [i32, P, P, P, i32, P, i32, P, i32, P, P, i32, P, P])):
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


def ls_loss_gs(A, X0, sweeps: int, color, ncolors: int, w, cf, caliber: int, val=None) -> float:
    """L = sum over F of ls_val after colour-phase Gauss-Seidel sweeps."""
    L = _sig_gs_grad(lib())
    n, rp, ci, va = _csr(A)
    if val is not None:
        va = _f64(val)
    X0 = _f64(X0)
    col = np.ascontiguousarray(color, dtype=np.int32)
    w = None if w is None else _f64(w)
    cf = np.ascontiguousarray(cf, dtype=np.uint8)
    return float(L.oracle_ls_loss_gs(n, _p(rp), _p(ci), _p(va), X0.shape[1], _p(X0), int(sweeps),
                                     _p(col), int(ncolors), _p(w), _p(cf), int(caliber)))


def ls_grad_w(A, X, w, cf, caliber: int):
    """dL/dw_k at the final panel X."""
    L = _sig_gs_grad(lib())
    n, rp, ci, va = _csr(A)
    X = _f64(X)
    w = None if w is None else _f64(w)
    cf = np.ascontiguousarray(cf, dtype=np.uint8)
    gw = np.empty(X.shape[1])
    L.oracle_ls_grad_w(n, _p(rp), _p(ci), _p(va), X.shape[1], _p(X), _p(w), _p(cf), int(caliber),
                       _p(gw))
    return gw


def ls_loss_grad_gs(A, X0, sweeps: int, color, ncolors: int, w, cf, caliber: int):
    """(L, dL/dvals, dL/dw) through colour-phase Gauss-Seidel sweeps."""
    L = _sig_gs_grad(lib())
    n, rp, ci, va = _csr(A)
    X0 = _f64(X0)
    col = np.ascontiguousarray(color, dtype=np.int32)
    w = None if w is None else _f64(w)
    cf = np.ascontiguousarray(cf, dtype=np.uint8)
    gv = np.empty(len(ci))
    gw = np.empty(X0.shape[1])
    Lv = L.oracle_ls_loss_grad_gs(n, _p(rp), _p(ci), _p(va), X0.shape[1], _p(X0), int(sweeps),
                                  _p(col), int(ncolors), _p(w), _p(cf), int(caliber), _p(gv), _p(gw))
    return float(Lv), gv, gw


def _sig_galerkin(L):
    P = C.c_void_p
    i32 = C.c_int
    for name, res, args in (
            ("oracle_galerkin_counts", i32, [i32, P, P, i32, P, P, P, P]),
            ("oracle_galerkin_fill", None, [i32, P, P, P, i32, P, P, P, P, P, P]),
            ("oracle_two_grid", i32, [i32, P, P, P, P, i32, i32, P, P, P, P, P, P, i32, P, i32, i32,
                                      i32, P, P])):
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


class CoarseCSR:
    """A coarse operator: nc rows, CSR with sorted columns, FP64 values."""

    def __init__(self, nc, row_ptr, col, val):
        self.n = int(nc)
        self.row_ptr = row_ptr
        self.col = col
        self.val = val

    @property
    def nnz(self):
        return int(self.row_ptr[-1])


def galerkin(A, P_col, P_val, cf) -> CoarseCSR:
    """A_c = P^T A P (Sec. 5.2), coarse points numbered in fine order."""
    L = _sig_galerkin(lib())
    n, rp, ci, va = _csr(A)
    Pc = np.ascontiguousarray(P_col, dtype=np.int32)
    Pv = _f64(P_val)
    cf = np.ascontiguousarray(cf, dtype=np.uint8)
    cal = Pc.shape[1]
    cnt = np.empty(max(1, int(cf.astype(bool).sum())), dtype=np.int32)
    nc = L.oracle_galerkin_counts(n, _p(rp), _p(ci), cal, _p(Pc), _p(Pv), _p(cf), _p(cnt))
    rpc = np.concatenate([[0], np.cumsum(cnt[:nc], dtype=np.int64)]).astype(np.int32)
    colc = np.empty(max(1, int(rpc[-1])), dtype=np.int32)
    valc = np.empty(max(1, int(rpc[-1])))
    L.oracle_galerkin_fill(n, _p(rp), _p(ci), _p(va), cal, _p(Pc), _p(Pv), _p(cf), _p(rpc), _p(colc),
                           _p(valc))
    m = int(rpc[-1])
    return CoarseCSR(nc, rpc, colc[:m], valc[:m])


def two_grid(A, color, ncolors: int, P_col, P_val, cf, Ac: CoarseCSR, E0, iters: int = 100,
             pre: int = 2, post: int = 2):
    """Two-grid rate per column of E0 (Sec. 5.2): (rho[K], status, hist),
    hist[t, k] = ||e^t||_A."""
    L = _sig_galerkin(lib())
    n, rp, ci, va = _csr(A)
    col = np.ascontiguousarray(color, dtype=np.int32)
    Pc = np.ascontiguousarray(P_col, dtype=np.int32)
    Pv = _f64(P_val)
    cf = np.ascontiguousarray(cf, dtype=np.uint8)
    E0 = _f64(E0)
    K = E0.shape[1]
    rho = np.empty(K)
    hist = np.zeros((iters + 1, K))
    bad = L.oracle_two_grid(n, _p(rp), _p(ci), _p(va), _p(col), int(ncolors), Pc.shape[1], _p(Pc),
                            _p(Pv), _p(cf), _p(np.ascontiguousarray(Ac.row_ptr, dtype=np.int32)),
                            _p(np.ascontiguousarray(Ac.col, dtype=np.int32)), _p(_f64(Ac.val)), K,
                            _p(E0), int(iters), int(pre), int(post), _p(rho), _p(hist))
    return rho, int(bad), hist
