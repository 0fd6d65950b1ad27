"""distance_ls_noalloc (the entry point for callers that cannot allocate)
against distance_ls: bitwise the same outputs, on two calls in a row, the
second on a smaller input; and the size limit of its static scratch."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1106_5990_amd import workloads as W
from gpu_common import dev_csr, lib, say

pytestmark = pytest.mark.gpu


def outputs(A, K, caliber, dt):
    n, nnz = A.n, A.nnz
    return dict(mu=torch.empty(nnz, dtype=dt, device="cuda"),
                strong=torch.empty(nnz, dtype=torch.uint8, device="cuda"),
                nstrong=torch.empty(n, dtype=torch.int32, device="cuda"),
                P_col=torch.empty((n, caliber), dtype=torch.int32, device="cuda"),
                P_val=torch.empty((n, caliber), dtype=torch.float64, device="cuda"),
                ls_val=torch.empty(n, dtype=torch.float64, device="cuda"),
                row_status=torch.empty(n, dtype=torch.int32, device="cuda"),
                ls_sum=torch.empty(1, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_noalloc_matches_distance_ls_on_two_calls(dt):
    ad = lib()
    for N in (301, 97):  # the second call is the smaller input
        say("distance_ls_noalloc vs distance_ls, 9-point %d^2, %s" % (N, dt))
        w = W.workload(2, size=N)
        A = w.A
        Ad = dev_csr(A, dt)
        color = torch.as_tensor(w.color, device="cuda")
        cf = torch.as_tensor(w.cf, device="cuda")
        X = ad.setup_testvectors(Ad, w.K, seed=w.tv_seed, relax="gs", sweeps=w.sweeps, color=color,
                                 ncolors=w.ncolors)
        ref = ad.distance_ls(Ad, X, cf, w.caliber, theta=w.theta, want_sum=True)
        torch.cuda.synchronize()
        o = outputs(A, w.K, w.caliber, dt)
        for t in o.values():
            t.fill_(-7)  # stale contents must not survive
        ad.distance_ls_noalloc(Ad, X, cf, w.caliber, theta=w.theta, **o)
        torch.cuda.synchronize()
        names = ["mu", "strong", "nstrong", "P_col", "P_val", "ls_val", "row_status", "ls_sum"]
        for name, r in zip(names, ref):
            assert torch.equal(o[name], r), name
        assert ad.status(clear=True) == 0


def test_noalloc_without_sum_and_size_limit():
    """Without ls_sum nothing is staged; a fused pass that would need more
    partials than the static array holds is refused with AD_ESTRUCT before
    anything is enqueued."""
    ad = lib()
    w = W.workload(2, size=64)
    A = w.A
    Ad = dev_csr(A, torch.float32)
    cf = torch.as_tensor(w.cf, device="cuda")
    X = ad.setup_testvectors(Ad, w.K, seed=3, relax="jacobi", sweeps=2, omega=0.7)
    ref = ad.distance_ls(Ad, X, cf, w.caliber, theta=w.theta)
    o = outputs(A, w.K, w.caliber, torch.float32)
    o["ls_sum"] = None
    ad.distance_ls_noalloc(Ad, X, cf, w.caliber, theta=w.theta, **o)
    torch.cuda.synchronize()
    for name, r in zip(["mu", "strong", "nstrong", "P_col", "P_val", "ls_val", "row_status"], ref):
        assert torch.equal(o[name], r), name
    # a row count whose fused pass needs more than 131072 partials: the host
    # check refuses it from the sizes alone (no kernel runs, so the arrays
    # are never read).  The launch shape is pinned to 64 rows per workgroup
    # (4 lanes per row, one row step, contiguous XCD ranges), which makes
    # 2^30 rows 2^24 workgroups.
    ad.set_launch("distance_ls", torch.float32, w.K, lanes_per_row=4, rows_per_lane=1, xcd_map=1)
    n_big = 1 << 30
    big = ad.ad_csr(n_big, n_big, Ad._s.row_ptr, Ad._s.col, Ad._s.val, ad.AD_F32)
    s = torch.empty(1, dtype=torch.float64, device="cuda")
    h = ad.handle(0)
    rc = ad._lib.distance_ls_noalloc(h, C.byref(big), w.K, X.data_ptr(), None, 0,
                                     o["mu"].data_ptr(), 0.25, None, None, None, cf.data_ptr(),
                                     w.caliber, o["P_col"].data_ptr(), o["P_val"].data_ptr(),
                                     o["ls_val"].data_ptr(), o["row_status"].data_ptr(),
                                     s.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert rc == 4, rc  # AD_ESTRUCT
    assert b"static scratch" in ad._lib.algdist_last_error(h)
    assert ad.status(clear=True) == 0
