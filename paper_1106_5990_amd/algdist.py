"""Thin ctypes binding of libalgdist.so (C ABI in include/algdist.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  torch tensors provide device memory (data_ptr) and the stream
(torch.cuda.current_stream()).  Outputs not passed in are allocated here
with torch.empty on the input's device.  A non-zero status raises
AlgdistError with the library's message.

Importing this module raises ImportError when libalgdist.so has not been
built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libalgdist.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libalgdist.so is not built (expected at %s); run `python -m paper_1106_5990_amd.build`"
        % LIB_PATH)

_lib = C.CDLL(LIB_PATH)

AD_F32, AD_F64 = 0, 1
AD_JACOBI, AD_MULTICOLOR_GS = 0, 1
AD_TARGET_PLAIN, AD_TARGET_RESIDUAL = 0, 1

STAT_ZERO_DIAG = 0x01
STAT_BAD_COLOR = 0x02
STAT_NONFINITE = 0x04
STAT_CSR_ROWPTR = 0x08
STAT_CSR_COLS = 0x10
STAT_CSR_NODIAG = 0x20
STAT_SEARCH_CAP = 0x40
STAT_PATTERN = 0x80
STAT_BAD_INTERP = 0x100

STATUS_NAMES = {0: "AD_OK", 1: "AD_EINVAL", 2: "AD_EDTYPE", 3: "AD_ECALIBER", 4: "AD_ESTRUCT",
                5: "AD_EDEVICE", 6: "AD_ENOMEM", 7: "AD_EUNSUPPORTED"}


class ad_csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p), ("dtype", C.c_int32)]


_P = C.c_void_p
_i32, _i64, _u64, _f64 = C.c_int32, C.c_int64, C.c_uint64, C.c_double
_CSRP = C.POINTER(ad_csr)

_SIGS = {
    "algdist_version": (_i32, []),
    "algdist_create": (_i32, [C.POINTER(C.c_void_p), C.c_int]),
    "algdist_destroy": (_i32, [_P]),
    "algdist_status": (_i32, [_P, C.POINTER(C.c_uint32), C.c_int]),
    "algdist_last_error": (C.c_char_p, [_P]),
    "algdist_timing": (_i32, [_P, C.c_int]),
    "algdist_timing_report": (C.c_char_p, [_P]),
    "algdist_autotune": (_i32, [_P, _CSRP, _i32, _i32, _P, _i32, _P, _i32, C.c_char_p, _P]),
    "algdist_autotune_batched": (_i32, [_P, _i32, _CSRP, _i32, _i32, C.c_char_p, _P]),
    "algdist_set_launch": (_i32, [_P, C.c_char_p, _i32, _i32, _i32, _i32, _i32, _i32]),
    "csr_validate": (_i32, [_P, _CSRP, _P]),
    "setup_testvectors": (_i32, [_P, _CSRP, _i32, _u64, _P, _i32, _i32, _f64, _P, _i32, _P, _P,
                                 _i32, _P]),
    "algebraic_distance": (_i32, [_P, _CSRP, _i32, _P, _P, _i32, _P, _P, _f64, _P, _P, _P, _P]),
    "strength_graph": (_i32, [_P, _CSRP, _P, _f64, _P, _P, _P, _P]),
    "ls_interp": (_i32, [_P, _CSRP, _i32, _P, _P, _P, _P, _i32, _i32, _P, _P, _P, _P, _P, _P]),
    "distance_ls": (_i32, [_P, _CSRP, _i32, _P, _P, _i32, _P, _f64, _P, _P, _P, _P, _i32, _P, _P, _P,
                           _P, _P, _P]),
    "distance_ls_noalloc": (_i32, [_P, _CSRP, _i32, _P, _P, _i32, _P, _f64, _P, _P, _P, _P, _i32, _P,
                                   _P, _P, _P, _P, _P]),
    "power_graph_rows": (_i32, [_P, _CSRP, _i32, _P, C.POINTER(C.c_int64), _P]),
    "power_graph_cols": (_i32, [_P, _CSRP, _i32, _P, _P, _P]),
    "algebraic_distance_graph": (_i32, [_P, _CSRP, _i64, _P, _P, _i32, _P, _P, _i32, _P, _P, _f64,
                                        _P, _P, _P, _P]),
    "ls_interp_search": (_i32, [_P, _CSRP, _i64, _P, _P, _i32, _P, _P, _P, _i32, _f64, _i32, _P, _P,
                                _P, _P, _P]),
    "relax_algdist_batched": (_i32, [_P, _i32, _CSRP, _i32, _u64, _i32, _i32, _f64, _P, _P, _P,
                                     _f64, _P, _P, _P]),
    "ls_interp_loss_backward": (_i32, [_P, _CSRP, _i32, _P, _i32, _i32, _f64, _P, _P, _P, _P, _i32,
                                       _P, _P, _P, _P, _P]),
    "ls_interp_loss_grad": (_i32, [_P, _CSRP, _i32, _i32, _P, _i32, _P, _i32, _i32, _f64, _P, _P,
                                   _P, _P, _i32, _P, _P, _P, _P, _P, _P]),
    "galerkin_rows": (_i32, [_P, _CSRP, _i32, _P, _P, _P, C.POINTER(C.c_int32), _P,
                             C.POINTER(C.c_int64), _P]),
    "galerkin_cols": (_i32, [_P, _CSRP, _i32, _P, _P, _P, _i32, _P, _P, _P, _P]),
    "two_grid_rate": (_i32, [_P, _CSRP, _P, _i32, _i32, _P, _P, _P, _i32, _P, _P, _P, _i32, _P,
                             _i32, _i32, _i32, _P, _P, _P]),
    "cr_rate": (_i32, [_P, _CSRP, _P, _i32, _P, _i32, _P, C.POINTER(C.c_double), _P, _P]),
    "cr_candidates": (_i32, [_P, _i32, _i32, _P, _P, _f64, _P, _P]),
    "independent_set": (_i32, [_P, _CSRP, _P, _P, _u64, _P, C.POINTER(C.c_int64), _P]),
    "cr_coarsening": (_i32, [_P, _CSRP, _P, _i32, _P, _f64, _i32, _f64, _i32, _u64, _P, _P, _P,
                             C.POINTER(C.c_int32), _P]),
    "cr_coarsening_graph": (_i32, [_P, _CSRP, _i64, _P, _P, _P, _i32, _P, _f64, _i32, _f64, _i32,
                                   _u64, _P, _P, _P, C.POINTER(C.c_int32), _P]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class AlgdistError(RuntimeError):
    pass


_handles = {}


def handle(device: Optional[int] = None):
    dev = torch.cuda.current_device() if device is None else int(device)
    h = _handles.get(dev)
    if h is None:
        hp = C.c_void_p()
        rc = _lib.algdist_create(C.byref(hp), dev)
        if rc != 0:
            raise AlgdistError("algdist_create(device=%d) failed: %s" % (dev, STATUS_NAMES.get(rc, rc)))
        h = hp.value
        _handles[dev] = h
    return h


def _check(rc: int, h, what: str):
    if rc != 0:
        msg = _lib.algdist_last_error(h).decode() if h else ""
        raise AlgdistError("%s: %s %s" % (what, STATUS_NAMES.get(rc, rc), msg))


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _dtype_code(dt: torch.dtype) -> int:
    if dt == torch.float32:
        return AD_F32
    if dt == torch.float64:
        return AD_F64
    raise AlgdistError("unsupported dtype %s" % dt)


class Csr:
    """Device CSR: int32 row_ptr[n+1], int32 col[nnz], val[nnz] (float32/64)."""

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor):
        for t, name in ((row_ptr, "row_ptr"), (col, "col")):
            if t.dtype != torch.int32 or not t.is_contiguous():
                raise AlgdistError("%s must be a contiguous int32 tensor" % name)
        if not val.is_contiguous():
            raise AlgdistError("val must be contiguous")
        self.row_ptr, self.col, self.val = row_ptr, col, val
        self.n = row_ptr.numel() - 1
        self.nnz = col.numel()
        self.dtype = val.dtype
        self.device = val.device
        self._s = ad_csr(self.n, self.nnz, row_ptr.data_ptr(), col.data_ptr(), val.data_ptr(),
                         _dtype_code(val.dtype))

    @classmethod
    def from_host(cls, A, dtype=torch.float64, device="cuda"):
        """From any object with numpy row_ptr/col/val (e.g. workloads.CSR)."""
        return cls(torch.as_tensor(A.row_ptr).to(device=device, dtype=torch.int32).contiguous(),
                   torch.as_tensor(A.col).to(device=device, dtype=torch.int32).contiguous(),
                   torch.as_tensor(A.val).to(device=device, dtype=dtype).contiguous())

    def with_values(self, val: torch.Tensor) -> "Csr":
        return Csr(self.row_ptr, self.col, val)

    def ref(self):
        return C.byref(self._s)


def status(clear: bool = False, device: Optional[int] = None) -> int:
    """Sticky device status bits (synchronises the device)."""
    h = handle(device)
    bits = C.c_uint32(0)
    _check(_lib.algdist_status(h, C.byref(bits), int(clear)), h, "algdist_status")
    return int(bits.value)


def timing(enable: bool, device: Optional[int] = None) -> None:
    """Start (enable=True, fresh record) or stop per-kernel HIP-event timing."""
    h = handle(device)
    _check(_lib.algdist_timing(h, int(enable)), h, "algdist_timing")


def timing_report(device: Optional[int] = None) -> dict:
    """{label: (launches, total_ms)} of the kernels timed since timing(True)."""
    h = handle(device)
    txt = _lib.algdist_timing_report(h).decode()
    out = {}
    for line in txt.splitlines():
        lab, cnt, ms = line.split()
        out[lab] = (int(cnt), float(ms))
    return out


def set_launch(kernel: str, dtype: torch.dtype, K: int, lanes_per_row: int = 0,
               rows_per_lane: int = 1, xcd_map: int = 1, bucket: int = -1,
               device: Optional[int] = None) -> None:
    """Force the launch shape of one kernel family (see algdist_set_launch);
    xcd_map: 0 plain block order, 1 contiguous tiles per XCD, c >= 2 chunks of
    8c tiles with c per XCD."""
    h = handle(device)
    rc = _lib.algdist_set_launch(h, kernel.encode(), _dtype_code(dtype), K, bucket, lanes_per_row,
                                 rows_per_lane, int(xcd_map))
    _check(rc, h, "algdist_set_launch")


def autotune(A: Csr, K: int, relax: str = "jacobi", color: Optional[torch.Tensor] = None,
             ncolors: int = 0, cf: Optional[torch.Tensor] = None, caliber: int = 0,
             cache_json: Optional[str] = None, stream=None) -> None:
    """Time every launch shape on A and install the fastest (algdist_autotune)."""
    h = handle(A.device.index)
    kind = {"jacobi": AD_JACOBI, "gs": AD_MULTICOLOR_GS}[relax]
    rc = _lib.algdist_autotune(h, A.ref(), K, kind, _ptr(color), ncolors, _ptr(cf), caliber,
                               None if cache_json is None else cache_json.encode(), _stream(stream))
    _check(rc, h, "algdist_autotune")


def autotune_batched(mats, K: int, sweeps: int, cache_json: Optional[str] = None,
                     stream=None) -> None:
    """Time every launch shape of relax_algdist_batched on this batch and
    install the fastest (algdist_autotune_batched)."""
    h = handle(mats[0].device.index)
    arr = (ad_csr * len(mats))(*[m._s for m in mats])
    rc = _lib.algdist_autotune_batched(h, len(mats), arr, K, sweeps,
                                       None if cache_json is None else cache_json.encode(),
                                       _stream(stream))
    _check(rc, h, "algdist_autotune_batched")


def csr_validate(A: Csr, stream=None) -> None:
    h = handle(A.device.index)
    _check(_lib.csr_validate(h, A.ref(), _stream(stream)), h, "csr_validate")


def setup_testvectors(A: Csr, K: int, seed: int = 0, X0: Optional[torch.Tensor] = None,
                      relax: str = "jacobi", sweeps: int = 1, omega: float = 2.0 / 3.0,
                      color: Optional[torch.Tensor] = None, ncolors: int = 0,
                      out: Optional[torch.Tensor] = None, ckpt: Optional[torch.Tensor] = None,
                      ckpt_every: int = 0, stream=None) -> torch.Tensor:
    h = handle(A.device.index)
    X = out if out is not None else torch.empty((A.n, K), dtype=A.dtype, device=A.device)
    kind = {"jacobi": AD_JACOBI, "gs": AD_MULTICOLOR_GS}[relax]
    rc = _lib.setup_testvectors(h, A.ref(), K, seed & (2 ** 64 - 1), _ptr(X0), kind, sweeps,
                                float(omega), _ptr(color), ncolors, _ptr(X), _ptr(ckpt),
                                ckpt_every, _stream(stream))
    _check(rc, h, "setup_testvectors")
    return X


def algebraic_distance(A: Csr, X: torch.Tensor, w: Optional[torch.Tensor] = None,
                       target: str = "plain", mu: Optional[torch.Tensor] = None,
                       p: Optional[torch.Tensor] = None, want_p: bool = False,
                       theta: float = 0.0, fmask: Optional[torch.Tensor] = None,
                       strong: Optional[torch.Tensor] = None,
                       nstrong: Optional[torch.Tensor] = None, fuse: bool = False, stream=None):
    """Returns mu, or (mu, strong, nstrong) when fuse=True, plus p if want_p."""
    h = handle(A.device.index)
    K = X.shape[1]
    mu = mu if mu is not None else torch.empty(A.nnz, dtype=A.dtype, device=A.device)
    if want_p and p is None:
        p = torch.empty(A.nnz, dtype=torch.float64, device=A.device)
    if fuse:
        strong = strong if strong is not None else torch.empty(A.nnz, dtype=torch.uint8, device=A.device)
        nstrong = nstrong if nstrong is not None else torch.empty(A.n, dtype=torch.int32, device=A.device)
    tg = {"plain": AD_TARGET_PLAIN, "residual": AD_TARGET_RESIDUAL}[target]
    rc = _lib.algebraic_distance(h, A.ref(), K, _ptr(X), _ptr(w), tg, _ptr(mu), _ptr(p),
                                 float(theta), _ptr(fmask), _ptr(strong) if fuse else None,
                                 _ptr(nstrong) if fuse else None, _stream(stream))
    _check(rc, h, "algebraic_distance")
    res = (mu, strong, nstrong) if fuse else (mu,)
    if want_p:
        res = res + (p,)
    return res if len(res) > 1 else res[0]


def strength_graph(A: Csr, mu: torch.Tensor, theta: float, fmask: Optional[torch.Tensor] = None,
                   strong: Optional[torch.Tensor] = None, nstrong: Optional[torch.Tensor] = None,
                   stream=None):
    h = handle(A.device.index)
    strong = strong if strong is not None else torch.empty(A.nnz, dtype=torch.uint8, device=A.device)
    nstrong = nstrong if nstrong is not None else torch.empty(A.n, dtype=torch.int32, device=A.device)
    rc = _lib.strength_graph(h, A.ref(), _ptr(mu), float(theta), _ptr(fmask), _ptr(strong),
                             _ptr(nstrong), _stream(stream))
    _check(rc, h, "strength_graph")
    return strong, nstrong


def ls_interp(A: Csr, X: torch.Tensor, cf: torch.Tensor, mu: torch.Tensor, caliber: int,
              w: Optional[torch.Tensor] = None, target: str = "plain",
              P_col: Optional[torch.Tensor] = None, P_val: Optional[torch.Tensor] = None,
              ls_val: Optional[torch.Tensor] = None, row_status: Optional[torch.Tensor] = None,
              ls_sum: Optional[torch.Tensor] = None, want_sum: bool = False, stream=None):
    """Returns (P_col, P_val, ls_val, row_status) and ls_sum if want_sum."""
    h = handle(A.device.index)
    K = X.shape[1]
    dev = A.device
    P_col = P_col if P_col is not None else torch.empty((A.n, caliber), dtype=torch.int32, device=dev)
    P_val = P_val if P_val is not None else torch.empty((A.n, caliber), dtype=torch.float64, device=dev)
    ls_val = ls_val if ls_val is not None else torch.empty(A.n, dtype=torch.float64, device=dev)
    row_status = row_status if row_status is not None else torch.empty(A.n, dtype=torch.int32, device=dev)
    if want_sum and ls_sum is None:
        ls_sum = torch.empty(1, dtype=torch.float64, device=dev)
    tg = {"plain": AD_TARGET_PLAIN, "residual": AD_TARGET_RESIDUAL}[target]
    rc = _lib.ls_interp(h, A.ref(), K, _ptr(X), _ptr(w), _ptr(cf), _ptr(mu), caliber, tg,
                        _ptr(P_col), _ptr(P_val), _ptr(ls_val), _ptr(row_status),
                        _ptr(ls_sum) if want_sum else None, _stream(stream))
    _check(rc, h, "ls_interp")
    out = (P_col, P_val, ls_val, row_status)
    return out + (ls_sum,) if want_sum else out


def distance_ls(A: Csr, X: torch.Tensor, cf: torch.Tensor, caliber: int,
                w: Optional[torch.Tensor] = None, target: str = "plain", theta: float = 0.25,
                fuse: bool = True, fmask: Optional[torch.Tensor] = None,
                mu: Optional[torch.Tensor] = None, strong: Optional[torch.Tensor] = None,
                nstrong: Optional[torch.Tensor] = None, P_col: Optional[torch.Tensor] = None,
                P_val: Optional[torch.Tensor] = None, ls_val: Optional[torch.Tensor] = None,
                row_status: Optional[torch.Tensor] = None, ls_sum: Optional[torch.Tensor] = None,
                want_sum: bool = False, stream=None):
    """Distances (+ strength row when fuse) and LS rows in one pass
    (distance_ls).  Returns (mu, strong, nstrong, P_col, P_val, ls_val,
    row_status, ls_sum); strong/nstrong None when not fuse, ls_sum None when
    not want_sum."""
    h = handle(A.device.index)
    n, dev = A.n, A.device
    mu = mu if mu is not None else torch.empty(A.nnz, dtype=A.dtype, device=dev)
    if fuse:
        strong = strong if strong is not None else torch.empty(A.nnz, dtype=torch.uint8, device=dev)
        nstrong = nstrong if nstrong is not None else torch.empty(n, dtype=torch.int32, device=dev)
    else:
        strong = nstrong = None
    P_col = P_col if P_col is not None else torch.empty((n, caliber), dtype=torch.int32, device=dev)
    P_val = P_val if P_val is not None else torch.empty((n, caliber), dtype=torch.float64, device=dev)
    ls_val = ls_val if ls_val is not None else torch.empty(n, dtype=torch.float64, device=dev)
    row_status = row_status if row_status is not None else torch.empty(n, dtype=torch.int32, device=dev)
    if want_sum and ls_sum is None:
        ls_sum = torch.empty(1, dtype=torch.float64, device=dev)
    tg = {"plain": AD_TARGET_PLAIN, "residual": AD_TARGET_RESIDUAL}[target]
    rc = _lib.distance_ls(h, A.ref(), X.shape[1], _ptr(X), _ptr(w), tg, _ptr(mu), float(theta),
                          _ptr(fmask), _ptr(strong), _ptr(nstrong), _ptr(cf), caliber, _ptr(P_col),
                          _ptr(P_val), _ptr(ls_val), _ptr(row_status),
                          _ptr(ls_sum) if want_sum else None, _stream(stream))
    _check(rc, h, "distance_ls")
    return mu, strong, nstrong, P_col, P_val, ls_val, row_status, (ls_sum if want_sum else None)


def distance_ls_noalloc(A: Csr, X: torch.Tensor, cf: torch.Tensor, caliber: int, *,
                        mu: torch.Tensor, P_col: torch.Tensor, P_val: torch.Tensor,
                        ls_val: torch.Tensor, row_status: torch.Tensor,
                        strong: Optional[torch.Tensor] = None,
                        nstrong: Optional[torch.Tensor] = None,
                        ls_sum: Optional[torch.Tensor] = None, w: Optional[torch.Tensor] = None,
                        target: str = "plain", theta: float = 0.25,
                        fmask: Optional[torch.Tensor] = None, stream=None) -> None:
    """distance_ls_noalloc: distance_ls without any device allocation, here
    or in the library (the caller passes every output; ls_sum, if given,
    receives the F-row sum)."""
    h = handle(A.device.index)
    tg = {"plain": AD_TARGET_PLAIN, "residual": AD_TARGET_RESIDUAL}[target]
    rc = _lib.distance_ls_noalloc(h, A.ref(), X.shape[1], _ptr(X), _ptr(w), tg, _ptr(mu),
                                  float(theta), _ptr(fmask), _ptr(strong), _ptr(nstrong), _ptr(cf),
                                  caliber, _ptr(P_col), _ptr(P_val), _ptr(ls_val),
                                  _ptr(row_status), _ptr(ls_sum), _stream(stream))
    _check(rc, h, "distance_ls_noalloc")



class Pattern:
    """A device sparsity pattern of n rows (int32 row_ptr[n+1], int32 col)."""

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor):
        self.row_ptr, self.col = row_ptr, col
        self.n = row_ptr.numel() - 1
        self.nnz = col.numel()


def power_graph(A: Csr, d: int, stream=None) -> Pattern:
    """Pattern of A^d (power_graph_rows, which synchronises, then
    power_graph_cols)."""
    h = handle(A.device.index)
    rp = torch.empty(A.n + 1, dtype=torch.int32, device=A.device)
    nnz = C.c_int64(0)
    _check(_lib.power_graph_rows(h, A.ref(), int(d), _ptr(rp), C.byref(nnz), _stream(stream)), h,
           "power_graph_rows")
    col = torch.empty(int(nnz.value), dtype=torch.int32, device=A.device)
    _check(_lib.power_graph_cols(h, A.ref(), int(d), _ptr(rp), _ptr(col), _stream(stream)), h,
           "power_graph_cols")
    return Pattern(rp, col)


def algebraic_distance_graph(A: Csr, G: Pattern, X: torch.Tensor, w: Optional[torch.Tensor] = None,
                             target: str = "plain", mu: Optional[torch.Tensor] = None,
                             p: Optional[torch.Tensor] = None, want_p: bool = False,
                             theta: float = 0.0, fmask: Optional[torch.Tensor] = None,
                             strong: Optional[torch.Tensor] = None,
                             nstrong: Optional[torch.Tensor] = None, fuse: bool = False,
                             stream=None):
    """Distances over G's entries (targets from A).  Returns mu, or (mu,
    strong, nstrong) when fuse=True, plus p if want_p."""
    h = handle(A.device.index)
    K = X.shape[1]
    mu = mu if mu is not None else torch.empty(G.nnz, dtype=A.dtype, device=A.device)
    if want_p and p is None:
        p = torch.empty(G.nnz, dtype=torch.float64, device=A.device)
    if fuse:
        strong = strong if strong is not None else torch.empty(G.nnz, dtype=torch.uint8, device=A.device)
        nstrong = nstrong if nstrong is not None else torch.empty(A.n, dtype=torch.int32, device=A.device)
    tg = {"plain": AD_TARGET_PLAIN, "residual": AD_TARGET_RESIDUAL}[target]
    rc = _lib.algebraic_distance_graph(h, A.ref(), G.nnz, _ptr(G.row_ptr), _ptr(G.col), K, _ptr(X),
                                       _ptr(w), tg, _ptr(mu), _ptr(p), float(theta), _ptr(fmask),
                                       _ptr(strong) if fuse else None,
                                       _ptr(nstrong) if fuse else None, _stream(stream))
    _check(rc, h, "algebraic_distance_graph")
    res = (mu, strong, nstrong) if fuse else (mu,)
    if want_p:
        res = res + (p,)
    return res if len(res) > 1 else res[0]


def ls_interp_search(A: Csr, G: Pattern, X: torch.Tensor, cf: torch.Tensor, caliber: int,
                     gamma: float = 1.5, w: Optional[torch.Tensor] = None, target: str = "plain",
                     P_col: Optional[torch.Tensor] = None, P_val: Optional[torch.Tensor] = None,
                     ls_val: Optional[torch.Tensor] = None,
                     row_status: Optional[torch.Tensor] = None, stream=None):
    """Interpolatory sets by search over the C-points of G's rows:
    (P_col, P_val, ls_val, row_status)."""
    h = handle(A.device.index)
    n, dev = A.n, A.device
    P_col = P_col if P_col is not None else torch.empty((n, caliber), dtype=torch.int32, device=dev)
    P_val = P_val if P_val is not None else torch.empty((n, caliber), dtype=torch.float64, device=dev)
    ls_val = ls_val if ls_val is not None else torch.empty(n, dtype=torch.float64, device=dev)
    row_status = row_status if row_status is not None else torch.empty(n, dtype=torch.int32, device=dev)
    tg = {"plain": AD_TARGET_PLAIN, "residual": AD_TARGET_RESIDUAL}[target]
    rc = _lib.ls_interp_search(h, A.ref(), G.nnz, _ptr(G.row_ptr), _ptr(G.col), X.shape[1], _ptr(X),
                               _ptr(w), _ptr(cf), caliber, float(gamma), tg, _ptr(P_col),
                               _ptr(P_val), _ptr(ls_val), _ptr(row_status), _stream(stream))
    _check(rc, h, "ls_interp_search")
    return P_col, P_val, ls_val, row_status


def relax_algdist_batched(mats, K: int, seed: int = 0, sweeps: int = 4, omega: float = 2.0 / 3.0,
                          w: Optional[torch.Tensor] = None, theta: float = 0.25, fuse: bool = True,
                          relax: str = "jacobi",
                          X: Optional[torch.Tensor] = None, mu: Optional[torch.Tensor] = None,
                          strong: Optional[torch.Tensor] = None,
                          nstrong: Optional[torch.Tensor] = None, stream=None):
    """Start + Jacobi sweeps + distances (+ strength) for a list of Csr, one
    launch per stage over the tiles of all members (replayed from a captured
    graph on repeated calls).  Returns (X, mu, strong, nstrong), concatenated in list
    order (strong/nstrong None when fuse=False)."""
    dev = mats[0].device
    h = handle(dev.index)
    dt = mats[0].dtype
    rows = sum(m.n for m in mats)
    ents = sum(m.nnz for m in mats)
    X = X if X is not None else torch.empty((rows, K), dtype=dt, device=dev)
    mu = mu if mu is not None else torch.empty(ents, dtype=dt, device=dev)
    if fuse:
        strong = strong if strong is not None else torch.empty(ents, dtype=torch.uint8, device=dev)
        nstrong = nstrong if nstrong is not None else torch.empty(rows, dtype=torch.int32, device=dev)
    arr = (ad_csr * len(mats))(*[m._s for m in mats])
    rk = {"jacobi": AD_JACOBI, "gs": AD_MULTICOLOR_GS}[relax]
    rc = _lib.relax_algdist_batched(h, len(mats), arr, K, seed & (2 ** 64 - 1), rk, sweeps,
                                    float(omega), _ptr(w), _ptr(X), _ptr(mu), float(theta),
                                    _ptr(strong) if fuse else None, _ptr(nstrong) if fuse else None,
                                    _stream(stream))
    _check(rc, h, "relax_algdist_batched")
    return X, mu, (strong if fuse else None), (nstrong if fuse else None)


def ls_interp_loss_backward(A: Csr, K: int, ckpt: torch.Tensor, ckpt_every: int, sweeps: int,
                            omega: float, cf: torch.Tensor, P_col: torch.Tensor,
                            P_val: torch.Tensor, X_final: torch.Tensor, dL: torch.Tensor,
                            w: Optional[torch.Tensor] = None, grad_val: Optional[torch.Tensor] = None,
                            grad_omega: Optional[torch.Tensor] = None, stream=None):
    """(grad_val[nnz], grad_omega[1]) of the LS loss; see ls_interp_loss_backward in algdist.h."""
    h = handle(A.device.index)
    grad_val = grad_val if grad_val is not None else torch.empty(A.nnz, dtype=torch.float64, device=A.device)
    grad_omega = grad_omega if grad_omega is not None else torch.empty(1, dtype=torch.float64, device=A.device)
    rc = _lib.ls_interp_loss_backward(h, A.ref(), K, _ptr(ckpt), ckpt_every, sweeps, float(omega),
                                      _ptr(w), _ptr(cf), _ptr(P_col), _ptr(P_val), P_col.shape[1],
                                      _ptr(X_final), _ptr(dL), _ptr(grad_val), _ptr(grad_omega),
                                      _stream(stream))
    _check(rc, h, "ls_interp_loss_backward")
    return grad_val, grad_omega


class LSInterpLoss(torch.autograd.Function):
    """L(values, omega) = sum over F rows of the LS interpolation functional
    after `sweeps` damped-Jacobi sweeps of K test vectors (plain target).

    apply(values, omega, row_ptr, col, K, seed, sweeps, cf, caliber,
          ckpt_every=2, w=None, X0=None) -> 0-dim FP64 tensor.
    values: FP64 CSR values (requires_grad); omega: 0-dim or 1-element FP64
    tensor (requires_grad).  Forward: setup_testvectors (checkpointed), then
    the distances (which pick C_i) and the LS rows with their F-row sum in one
    pass (distance_ls).
    Backward: ls_interp_loss_backward.
    """

    @staticmethod
    def forward(ctx, values, omega, row_ptr, col, K, seed, sweeps, cf, caliber, ckpt_every=2,
                w=None, X0=None):
        A = Csr(row_ptr, col, values.detach().contiguous())
        om = float(omega.detach().reshape(-1)[0])
        nck = max(1, -(-sweeps // ckpt_every))
        ck = torch.empty((nck, A.n, K), dtype=torch.float64, device=A.device)
        X = setup_testvectors(A, K, seed=seed, X0=X0, relax="jacobi", sweeps=sweeps, omega=om,
                              ckpt=ck, ckpt_every=ckpt_every)
        _, _, _, Pc, Pv, ls, st, tot = distance_ls(A, X, cf, caliber, w=w, fuse=False,
                                                   want_sum=True)
        ctx.save_for_backward(values, ck, X, Pc, Pv, cf)
        ctx.meta = (row_ptr, col, K, sweeps, ckpt_every, om, w, omega.shape)
        return tot.reshape(())

    @staticmethod
    def backward(ctx, gL):
        values, ck, X, Pc, Pv, cf = ctx.saved_tensors
        row_ptr, col, K, sweeps, ce, om, w, oshape = ctx.meta
        A = Csr(row_ptr, col, values.detach().contiguous())
        dL = gL.detach().reshape(1).to(torch.float64).contiguous()
        gv, go = ls_interp_loss_backward(A, K, ck, ce, sweeps, om, cf, Pc, Pv, X, dL, w=w)
        return gv, go.reshape(oshape), None, None, None, None, None, None, None, None, None, None


def ls_interp_loss_grad(A: Csr, K: int, ckpt: torch.Tensor, ckpt_every: int, sweeps: int,
                        cf: torch.Tensor, P_col: torch.Tensor, P_val: torch.Tensor,
                        X_final: torch.Tensor, dL: torch.Tensor, relax: str = "gs",
                        color: Optional[torch.Tensor] = None, ncolors: int = 0,
                        omega: float = 1.0, w: Optional[torch.Tensor] = None, stream=None):
    """(dL/dvalues, dL/domega, dL/dw) of the LS loss (ls_interp_loss_grad)."""
    h = handle(A.device.index)
    gv = torch.empty(A.nnz, dtype=torch.float64, device=A.device)
    go = torch.empty(1, dtype=torch.float64, device=A.device)
    gw = torch.empty(K, dtype=torch.float64, device=A.device)
    rk = {"jacobi": AD_JACOBI, "gs": AD_MULTICOLOR_GS}[relax]
    rc = _lib.ls_interp_loss_grad(h, A.ref(), K, rk, _ptr(color), int(ncolors), _ptr(ckpt),
                                  int(ckpt_every), int(sweeps), float(omega), _ptr(w), _ptr(cf),
                                  _ptr(P_col), _ptr(P_val), P_col.shape[1], _ptr(X_final), _ptr(dL),
                                  _ptr(gv), _ptr(go), _ptr(gw), _stream(stream))
    _check(rc, h, "ls_interp_loss_grad")
    return gv, go, gw


class LSInterpLossGS(torch.autograd.Function):
    """L(values, w) = sum over F rows of the LS interpolation functional
    after `sweeps` colour-phase Gauss-Seidel sweeps of K test vectors (plain
    target), differentiable in the CSR values and the LS weights w.

    apply(values, w, row_ptr, col, K, seed, sweeps, color, ncolors, cf, caliber,
          ckpt_every=1, X0=None) -> 0-dim FP64 tensor.
    Forward: setup_testvectors (checkpointed), then distance_ls.  Backward:
    ls_interp_loss_grad."""

    @staticmethod
    def forward(ctx, values, w, row_ptr, col, K, seed, sweeps, color, ncolors, cf, caliber,
                ckpt_every=1, X0=None):
        A = Csr(row_ptr, col, values.detach().contiguous())
        wd = w.detach().contiguous()
        nck = max(1, -(-sweeps // ckpt_every))
        ck = torch.empty((nck, A.n, K), dtype=torch.float64, device=A.device)
        X = setup_testvectors(A, K, seed=seed, X0=X0, relax="gs", sweeps=sweeps, color=color,
                              ncolors=ncolors, ckpt=ck, ckpt_every=ckpt_every)
        _, _, _, Pc, Pv, ls, st, tot = distance_ls(A, X, cf, caliber, w=wd, fuse=False,
                                                   want_sum=True)
        ctx.save_for_backward(values, wd, ck, X, Pc, Pv, cf, color)
        ctx.meta = (row_ptr, col, K, sweeps, ckpt_every, ncolors)
        return tot.reshape(())

    @staticmethod
    def backward(ctx, gL):
        values, wd, ck, X, Pc, Pv, cf, color = ctx.saved_tensors
        row_ptr, col, K, sweeps, ce, ncolors = ctx.meta
        A = Csr(row_ptr, col, values.detach().contiguous())
        dL = gL.detach().reshape(1).to(torch.float64).contiguous()
        gv, _, gw = ls_interp_loss_grad(A, K, ck, ce, sweeps, cf, Pc, Pv, X, dL, relax="gs",
                                        color=color, ncolors=ncolors, w=wd)
        return (gv, gw) + (None,) * 11


# ------------------------------------------------------------------ compatible relaxation
def cr_rate(A: Csr, color: torch.Tensor, ncolors: int, cf: torch.Tensor, nu: int = 5,
            u: Optional[torch.Tensor] = None, stream=None):
    """One CR run (cr_rate): (rho_f, u^nu, (|F|, sum u^2, max |u|))."""
    h = handle(A.device.index)
    u = u if u is not None else torch.empty(A.n, dtype=A.dtype, device=A.device)
    rho = C.c_double(0.0)
    norms = (C.c_double * 3)()
    _check(_lib.cr_rate(h, A.ref(), _ptr(color), int(ncolors), _ptr(cf), int(nu), _ptr(u),
                        C.byref(rho), norms, _stream(stream)), h, "cr_rate")
    return rho.value, u, tuple(norms)


def cr_candidates(cf: torch.Tensor, u: torch.Tensor, tol: float,
                  z: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """F points with |u_i| / max_F |u| > tol (cr_candidates)."""
    h = handle(u.device.index)
    z = z if z is not None else torch.empty(u.numel(), dtype=torch.uint8, device=u.device)
    _check(_lib.cr_candidates(h, u.numel(), _dtype_code(u.dtype), _ptr(cf), _ptr(u), float(tol),
                              _ptr(z), _stream(stream)), h, "cr_candidates")
    return z


def independent_set(A: Csr, strong: torch.Tensor, z: torch.Tensor, seed: int,
                    sel: Optional[torch.Tensor] = None, stream=None):
    """Greedy maximal independent set of z on the strong graph: (sel, count)."""
    h = handle(A.device.index)
    sel = sel if sel is not None else torch.empty(A.n, dtype=torch.uint8, device=A.device)
    cnt = C.c_int64(0)
    _check(_lib.independent_set(h, A.ref(), _ptr(strong), _ptr(z), seed & (2 ** 64 - 1), _ptr(sel),
                                C.byref(cnt), _stream(stream)), h, "independent_set")
    return sel, cnt.value


def cr_coarsening(A: Csr, color: torch.Tensor, ncolors: int, mu: torch.Tensor, theta: float = 0.25,
                  nu: int = 5, delta: float = 0.7, max_stages: int = 20, seed: int = 0,
                  cf: Optional[torch.Tensor] = None, G: Optional[Pattern] = None, stream=None):
    """Algorithm 1 (cr_coarsening): (cf, rho per stage, |C| per stage); cf
    is updated in place when given (its entries are C_0).  With a pattern G
    (e.g. power_graph(A, d)) the strength graph and the independent set
    live on G and mu holds one distance per entry of G
    (cr_coarsening_graph)."""
    h = handle(A.device.index)
    cf = cf if cf is not None else torch.zeros(A.n, dtype=torch.uint8, device=A.device)
    rho = (C.c_double * (max_stages + 1))()
    nc = (C.c_int64 * (max_stages + 1))()
    ns = C.c_int32(0)
    if G is None:
        rc = _lib.cr_coarsening(h, A.ref(), _ptr(color), int(ncolors), _ptr(mu), float(theta),
                                int(nu), float(delta), int(max_stages), seed & (2 ** 64 - 1),
                                _ptr(cf), rho, nc, C.byref(ns), _stream(stream))
        _check(rc, h, "cr_coarsening")
    else:
        rc = _lib.cr_coarsening_graph(h, A.ref(), G.nnz, _ptr(G.row_ptr), _ptr(G.col), _ptr(color),
                                      int(ncolors), _ptr(mu), float(theta), int(nu), float(delta),
                                      int(max_stages), seed & (2 ** 64 - 1), _ptr(cf), rho, nc,
                                      C.byref(ns), _stream(stream))
        _check(rc, h, "cr_coarsening_graph")
    k = ns.value + 1
    return cf, list(rho)[:k], list(nc)[:k]


# ------------------------------------------------------------------ Galerkin operator, two-grid
class CoarseOperator:
    """A_c = P^T A P on the device: nc rows, CSR (row_ptr, col), FP64 val."""

    def __init__(self, nc, row_ptr, col, val):
        self.n = int(nc)
        self.row_ptr = row_ptr
        self.col = col
        self.val = val

    @property
    def nnz(self):
        return int(self.col.numel())


def galerkin(A: Csr, P_col: torch.Tensor, P_val: torch.Tensor, cf: torch.Tensor,
             stream=None) -> CoarseOperator:
    """A_c = P^T A P (galerkin_rows, then galerkin_cols)."""
    h = handle(A.device.index)
    cal = P_col.shape[1]
    rp = torch.empty(A.n + 1, dtype=torch.int32, device=A.device)
    nc = C.c_int32(0)
    nnz = C.c_int64(0)
    _check(_lib.galerkin_rows(h, A.ref(), cal, _ptr(P_col), _ptr(P_val), _ptr(cf), C.byref(nc),
                              _ptr(rp), C.byref(nnz), _stream(stream)), h, "galerkin_rows")
    rp = rp[:nc.value + 1].clone()
    col = torch.empty(int(nnz.value), dtype=torch.int32, device=A.device)
    val = torch.empty(int(nnz.value), dtype=torch.float64, device=A.device)
    _check(_lib.galerkin_cols(h, A.ref(), cal, _ptr(P_col), _ptr(P_val), _ptr(cf), nc.value,
                              _ptr(rp), _ptr(col), _ptr(val), _stream(stream)), h, "galerkin_cols")
    return CoarseOperator(nc.value, rp, col, val)


def two_grid_rate(A: Csr, color: torch.Tensor, ncolors: int, P_col: torch.Tensor,
                  P_val: torch.Tensor, cf: torch.Tensor, Ac: CoarseOperator, E0: torch.Tensor,
                  iters: int = 100, pre: int = 2, post: int = 2, stream=None):
    """Two-grid rate per column of E0 (two_grid_rate): (rho[K], hist[iters+1, K])."""
    import numpy as _np
    h = handle(A.device.index)
    K = E0.shape[1]
    rho = _np.empty(K)
    hist = _np.empty((iters + 1, K))
    _check(_lib.two_grid_rate(h, A.ref(), _ptr(color), int(ncolors), P_col.shape[1], _ptr(P_col),
                              _ptr(P_val), _ptr(cf), Ac.n, _ptr(Ac.row_ptr), _ptr(Ac.col),
                              _ptr(Ac.val), K, _ptr(E0), int(iters), int(pre), int(post),
                              hist.ctypes.data_as(C.c_void_p), rho.ctypes.data_as(C.c_void_p),
                              _stream(stream)), h, "two_grid_rate")
    return rho, hist
