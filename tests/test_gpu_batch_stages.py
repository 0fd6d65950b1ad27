"""The batched path (one launch per stage over the row tiles of all members,
replayed from a captured graph) against the single-matrix kernels run on the
block-diagonal concatenation of the batch -- bitwise, since both use the same
per-row code and the same start stream -- and against the oracle; graph
replay, tile shapes, XCD mapping, empty and one-row members, weights, zero
sweeps, timing mode and the batch autotuner."""

import numpy as np
import pytest
import torch

import oracle
from paper_1106_5990_amd import workloads as W
from gpu_common import check_mu, lib, say, to_np

pytestmark = pytest.mark.gpu


def members(sizes, seed):
    return [W.rgg_laplacian(int(n), 6.0 + (q * 7) % 23, (seed, q)) for q, n in enumerate(sizes)]


def concat_reference(mats, dt, K, seed, sweeps, omega, theta, w=None):
    ad = lib()
    B = W.concat_csr(mats)
    Bd = ad.Csr.from_host(B, dtype=dt)
    X = ad.setup_testvectors(Bd, K, seed=seed, relax="jacobi", sweeps=sweeps, omega=omega)
    wt = None if w is None else torch.as_tensor(w, device="cuda")
    mu, s, ns = ad.algebraic_distance(Bd, X, w=wt, fuse=True, theta=theta)
    return B, X, mu, s, ns


def assert_same(got, ref, what):
    X, mu, s, ns = got
    _, Xr, mur, sr, nsr = ref
    assert torch.equal(X, Xr), what + ": X"
    assert torch.equal(mu, mur), what + ": mu"
    assert torch.equal(s, sr) and torch.equal(ns, nsr), what + ": strength"


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
@pytest.mark.parametrize("K", [16, 8])
def test_batch_equals_concatenated_single_matrix_path(dt, K):
    ad = lib()
    say("batch stages vs concatenation: %s K=%d" % (dt, K))
    mats = members([300, 2500, 9000, 17000, 40000, 1200, 6100, 23000], seed=1)
    dm = [ad.Csr.from_host(m, dtype=dt) for m in mats]
    ad.status(clear=True)
    got = ad.relax_algdist_batched(dm, K, seed=42, sweeps=4, omega=2 / 3, theta=0.25)
    ref = concat_reference(mats, dt, K, 42, 4, 2 / 3, 0.25)
    assert_same(got, ref, "default shape")
    assert ad.status(clear=True) == 0
    # the concatenation itself against the oracle
    B = ref[0]
    X, mu, s, ns = got
    x = to_np(X).astype(np.float64)
    vals = torch.as_tensor(B.val).to(dt).to(torch.float64).numpy()
    Bo = W.CSR(B.n, B.row_ptr, B.col, vals)
    mu_ref = oracle.algdist(Bo, x)
    check_mu(to_np(mu).astype(np.float64), mu_ref, (x * x).sum(1)[B.row_ids()], dt)
    s_ref, ns_ref = oracle.strength(B, to_np(mu).astype(np.float64), 0.25)
    assert np.array_equal(to_np(s), s_ref) and np.array_equal(to_np(ns), ns_ref)


def test_batch_replay_tiles_and_edge_members():
    ad = lib()
    say("batch stages: replay, tile shapes, empty and one-row members")
    dt, K = torch.float32, 16
    mats = members([5000, 1, 30000, 700], seed=2)
    mats.insert(1, W.CSR(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0)))
    dm = [ad.Csr.from_host(m, dtype=dt) for m in mats]
    ref = concat_reference(mats, dt, K, 7, 3, 0.6, 0.3)
    try:
        for it, xcd in ((1, 1), (3, 1), (16, 0), (2, 0), (1, 4), (2, 16)):
            ad.set_launch("batched", dt, K, 0, it, xcd)
            for rep in range(3):  # the first call captures the graph, later ones replay it
                got = ad.relax_algdist_batched(dm, K, seed=7, sweeps=3, omega=0.6, theta=0.3)
                assert_same(got, ref, "iter %d xcd %d rep %d" % (it, xcd, rep))
                # eager work between replays
                torch.cuda.synchronize()
                got[0].zero_()
        ad.timing(True)
        got = ad.relax_algdist_batched(dm, K, seed=7, sweeps=3, omega=0.6, theta=0.3)
        rep = ad.timing_report()
        ad.timing(False)
        assert_same(got, ref, "timing mode")
        assert rep["batch_jacobi"][0] == 3 and rep["batch_algdist"][0] == 1, rep
    finally:
        ad.set_launch("batched", dt, K, 0, 1, True)
    assert ad.status(clear=True) == 0
    # zero sweeps: the start itself, then distances
    got = ad.relax_algdist_batched(dm, K, seed=9, sweeps=0, theta=0.3)
    assert_same(got, concat_reference(mats, dt, K, 9, 0, 0.6, 0.3), "zero sweeps")
    # graph keyed on the arguments: another seed after a replay
    got = ad.relax_algdist_batched(dm, K, seed=11, sweeps=3, omega=0.6, theta=0.3)
    assert_same(got, concat_reference(mats, dt, K, 11, 3, 0.6, 0.3), "new seed")


def test_batch_every_lane_shape_and_weights():
    ad = lib()
    dt, K = torch.float32, 16
    mats = members([4000, 15000, 800], seed=3)
    dm = [ad.Csr.from_host(m, dtype=dt) for m in mats]
    w = 0.5 + np.random.default_rng(4).random(K)
    wt = torch.as_tensor(w, device="cuda")
    for lpr in (1, 2, 4):
        say("batch stages lpr=%d" % lpr)
        try:
            ad.set_launch("batched", dt, K, lpr, 2, True)
            ad.set_launch("batched_distance", dt, K, lpr, 3, 4)
            ad.set_launch("algdist", dt, K, lpr, 1, True)
            got = ad.relax_algdist_batched(dm, K, seed=5, sweeps=4, omega=2 / 3, theta=0.25)
            assert_same(got, concat_reference(mats, dt, K, 5, 4, 2 / 3, 0.25), "lpr %d" % lpr)
            got = ad.relax_algdist_batched(dm, K, seed=5, sweeps=4, omega=2 / 3, w=wt, theta=0.25)
            assert_same(got, concat_reference(mats, dt, K, 5, 4, 2 / 3, 0.25, w), "lpr %d, w" % lpr)
        finally:
            ad.set_launch("batched", dt, K, 0, 1, True)
            ad.set_launch("batched_distance", dt, K, 0, 1, True)
            ad.set_launch("algdist", dt, K, 0, 1, True)
    assert ad.status(clear=True) == 0


def test_batch_autotune_installs_a_shape(tmp_path):
    ad = lib()
    say("batch autotune")
    dt, K = torch.float32, 16
    mats = members([3000, 12000, 500, 20000], seed=6)
    dm = [ad.Csr.from_host(m, dtype=dt) for m in mats]
    cache = str(tmp_path / "tune.jsonl")
    ad.autotune_batched(dm, K, 4, cache_json=cache)
    lines = open(cache).read().splitlines()
    assert len(lines) == 2 and '"kernel": "batched"' in lines[0], lines
    assert '"kernel": "batched_distance"' in lines[1], lines
    # a second handle state reads the cache instead of timing
    ad.autotune_batched(dm, K, 4, cache_json=cache)
    assert open(cache).read().splitlines() == lines
    got = ad.relax_algdist_batched(dm, K, seed=3, sweeps=4, omega=2 / 3, theta=0.25)
    X, mu, s, ns = got
    ref = concat_reference(mats, dt, K, 3, 4, 2 / 3, 0.25)
    # relaxation is bitwise whatever the shape; distances to the FP32 bar
    assert torch.equal(X, ref[1])
    x = to_np(X).astype(np.float64)
    check_mu(to_np(mu).astype(np.float64), to_np(ref[2]).astype(np.float64),
             (x * x).sum(1)[ref[0].row_ids()], dt)
    assert ad.status(clear=True) == 0
    ad.set_launch("batched", dt, K, 0, 1, True)
    ad.set_launch("batched_distance", dt, K, 0, 1, True)


def test_batch_argument_errors():
    ad = lib()
    dt, K = torch.float32, 16
    mats = members([100, 200], seed=8)
    dm = [ad.Csr.from_host(m, dtype=dt) for m in mats]
    with pytest.raises(ad.AlgdistError):
        ad.relax_algdist_batched(dm, 12, seed=1, sweeps=2)
    with pytest.raises(ad.AlgdistError):
        ad.relax_algdist_batched(dm, K, seed=1, sweeps=-1)
    with pytest.raises(ad.AlgdistError):
        ad.relax_algdist_batched(dm, K, seed=1, sweeps=2, theta=1.5)
    mixed = [dm[0], ad.Csr.from_host(mats[1], dtype=torch.float64)]
    with pytest.raises(ad.AlgdistError):
        ad.relax_algdist_batched(mixed, K, seed=1, sweeps=2)
