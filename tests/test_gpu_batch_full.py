"""The batched path at the full size of workload 4 (512 random-geometric-graph
Laplacians, 2k-200k rows each, K = 16, 4 Jacobi sweeps, FP32) in the launch
configuration bench.py times (shapes from the batch autotuner, graph replay),
checked member by member on sampled members against the oracle: the start
bitwise, the last sweep within its one-sweep rounding bound, the distances on
sampled rows to the FP32 bar, the strength rows bit-exact given the distances.

The members are built in a child process (worker processes there never touch
the GPU) and handed over through a file."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1106_5990_amd import workloads as W
from gpu_common import check_mu, lib, row_abs_bound, say, to_np

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

BUILD = r"""
import os, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from paper_1106_5990_amd import workloads as W
mats = W.batch_workload(512, workers=min(16, os.cpu_count() or 1))
ns = np.array([m.n for m in mats], np.int64)
nz = np.array([m.nnz for m in mats], np.int64)
np.savez(sys.argv[2], n=ns, nnz=nz,
         row_ptr=np.concatenate([m.row_ptr for m in mats]),
         col=np.concatenate([m.col for m in mats]),
         val=np.concatenate([m.val for m in mats]).astype(np.float32))
print("batch written", int(ns.sum()), int(nz.sum()), flush=True)
"""


def members_from_file(path):
    z = np.load(path)
    ns, nz = z["n"], z["nnz"]
    rp_all, col_all, val_all = z["row_ptr"], z["col"], z["val"]
    out, ro, eo = [], 0, 0
    for n, nnz in zip(ns, nz):
        out.append(W.CSR(int(n), rp_all[ro:ro + n + 1], col_all[eo:eo + nnz],
                         val_all[eo:eo + nnz].astype(np.float64)))
        ro += n + 1
        eo += nnz
    return out


def test_full_batch_bench_configuration(tmp_path):
    ad = lib()
    path = str(tmp_path / "batch.npz")
    say("building the 512-member batch in a child process")
    r = subprocess.run([sys.executable, "-c", BUILD, ROOT, path], capture_output=True, text=True,
                       timeout=900)
    assert r.returncode == 0, r.stderr[-2000:]
    say("  " + r.stdout.strip())
    mats = members_from_file(path)
    K, S, om, th = W.BATCH_K, W.BATCH_SWEEPS, W.BATCH_OMEGA, W.BATCH_THETA
    seed = W.TV_SEED_BASE + 4
    dt = torch.float32
    dm = [ad.Csr.from_host(m, dtype=dt) for m in mats]
    try:
        ad.autotune_batched(dm, K, S)
        ad.status(clear=True)
        X0, _, _, _ = ad.relax_algdist_batched(dm, K, seed=seed, sweeps=0, theta=th)
        X0 = to_np(X0)
        Xp, _, _, _ = ad.relax_algdist_batched(dm, K, seed=seed, sweeps=S - 1, omega=om, theta=th)
        Xp = to_np(Xp)
        for _ in range(2):  # the first call captures the stage graph, the second replays it
            X, mu, s, ns = ad.relax_algdist_batched(dm, K, seed=seed, sweeps=S, omega=om, theta=th)
        x_all, mu_all = to_np(X), to_np(mu)
        s_all, ns_all = to_np(s), to_np(ns)
        assert ad.status(clear=True) == 0
    finally:
        ad.set_launch("batched", dt, K, 0, 1, 1)
        ad.set_launch("batched_distance", dt, K, 0, 1, 1)
    sizes = np.array([m.n for m in mats])
    rng = np.random.default_rng(4)
    pick = sorted(set([int(sizes.argmin()), int(sizes.argmax())]
                      + [int(q) for q in rng.choice(len(mats), 5, replace=False)]))
    row0 = np.concatenate([[0], np.cumsum(sizes)])
    e0 = np.concatenate([[0], np.cumsum([m.nnz for m in mats])])
    for m in pick:
        A = mats[m]
        A32 = W.CSR(A.n, A.row_ptr, A.col, A.val.astype(np.float32).astype(np.float64))
        r0, r1 = row0[m], row0[m + 1]
        # start: the global counter stream, rounded to FP32
        want0 = oracle.tv_init(A.n, K, seed, row0=int(r0)).astype(np.float32)
        assert np.array_equal(X0[r0:r1], want0), m
        # last sweep on sampled rows, from the GPU's own previous iterate
        rows = np.unique(np.concatenate([rng.choice(A.n, min(A.n, 512), replace=False),
                                         [0, A.n - 1]])).astype(np.int32)
        xp, x = Xp[r0:r1].astype(np.float64), x_all[r0:r1].astype(np.float64)
        want = oracle.jacobi_rows(A32, xp, om, rows)
        bound = row_abs_bound(A32, xp, xp, om, rows=rows)
        assert np.all(np.abs(x[rows] - want) <= bound), m
        # distances on the sampled rows; strength rows of the whole member
        mu_m = mu_all[e0[m]:e0[m + 1]].astype(np.float64)
        rp = A.row_ptr.astype(np.int64)
        got = np.concatenate([mu_m[rp[i]:rp[i + 1]] for i in rows])
        saa = np.repeat((x[rows] ** 2).sum(1), np.diff(rp)[rows])
        check_mu(got, oracle.algdist(A32, x, rows=rows), saa, dt, "member %d" % m)
        sr, nsr = oracle.strength(A, mu_m, th)
        assert np.array_equal(s_all[e0[m]:e0[m + 1]], sr), m
        assert np.array_equal(ns_all[r0:r1], nsr), m
        say("  member %d (%d rows) ok" % (m, A.n))
