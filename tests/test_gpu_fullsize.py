"""Parity at the full workload sizes, in the launch configuration bench.py
times: the 2048^2 rotated anisotropic 9-point operator (K = 16, 5 red-black
colour-phase GS sweeps) and the 160^3 log-normal 7-point operator (K = 32,
4 Jacobi sweeps, omega = 0.8).

FP64 path: every output against the oracle run on the whole workload.
FP32 path: each step against the oracle fed the same FP32 inputs (promoted
exactly) -- the last sweep and the LS rows on sampled rows, the distances on
sampled rows, the strength graph on every row -- and the FP32 chain against
the all-FP64 chain as a reported error distribution."""
import numpy as np
import pytest
import torch

import oracle
from paper_1106_5990_amd import workloads as W
from gpu_common import (check_ls, check_mu, dev_csr, lib, row_abs_bound, saa_per_edge, say,
                        to_np)

pytestmark = pytest.mark.gpu

_cache = {}


def wl(i):
    if i not in _cache:
        say("generating workload %d" % i)
        _cache[i] = W.workload(i)
    return _cache[i]


def run_setup(w, Ad, dtype, sweeps):
    ad = lib()
    color = None if w.color is None else torch.as_tensor(w.color, device="cuda")
    return ad.setup_testvectors(Ad, w.K, seed=w.tv_seed, relax=w.relax, sweeps=sweeps,
                                omega=w.omega, color=color, ncolors=w.ncolors)


def sample_rows(n, m=2048, seed=0):
    rng = np.random.default_rng(seed)
    rows = np.unique(np.concatenate([rng.choice(n, m, replace=False), [0, 1, n - 2, n - 1]]))
    return rows.astype(np.int32)


def packed(A, vec, rows):
    rp = A.row_ptr.astype(np.int64)
    return np.concatenate([vec[rp[r]:rp[r + 1]] for r in rows])


@pytest.mark.parametrize("i", [2, 3])
def test_fullsize_fp32_steps(i):
    ad = lib()
    w = wl(i)
    A = w.A
    say("full-size FP32 steps, workload %s" % w.name)
    A32 = W.CSR(A.n, A.row_ptr, A.col, A.val.astype(np.float32).astype(np.float64))
    Ad = dev_csr(A, torch.float32)
    ad.status(clear=True)
    Xp = to_np(run_setup(w, Ad, torch.float32, w.sweeps - 1)).astype(np.float64)
    X = run_setup(w, Ad, torch.float32, w.sweeps)
    x = to_np(X).astype(np.float64)
    rows = sample_rows(A.n)
    # last sweep on sampled rows
    if w.relax == "gs":
        want = oracle.color_gs_rows(A32, w.color, w.ncolors, Xp, x, rows)
        Z = np.where((w.color == 0)[:, None], x, Xp)
        bound = np.maximum(row_abs_bound(A32, Z, Xp, 1.0, rows=rows),
                           row_abs_bound(A32, Xp, Xp, 1.0, rows=rows))
    else:
        want = oracle.jacobi_rows(A32, Xp, w.omega, rows)
        bound = row_abs_bound(A32, Xp, Xp, w.omega, rows=rows)
    err = np.abs(x[rows] - want)
    say("  last sweep: max err/bound %.3g" % np.max(err / bound))
    assert np.all(err <= bound)
    # distances (+ fused strength) as bench runs them
    mu, strong, ns = ad.algebraic_distance(Ad, X, fuse=True, theta=w.theta)
    mu_h = to_np(mu).astype(np.float64)
    mu_ref = oracle.algdist(A32, x, rows=rows)
    saa = (x[rows] ** 2).sum(1)
    saa_e = np.repeat(saa, np.diff(A.row_ptr.astype(np.int64))[rows])
    check_mu(packed(A, mu_h, rows), mu_ref, saa_e, torch.float32, "sampled rows")
    s_ref, ns_ref = oracle.strength(A, mu_h, w.theta)
    assert np.array_equal(to_np(strong), s_ref)
    assert np.array_equal(to_np(ns), ns_ref)
    # LS rows on the sampled rows
    cf = torch.as_tensor(w.cf, device="cuda")
    Pc, Pv, ls, st, tot = ad.ls_interp(Ad, X, cf, mu, w.caliber, want_sum=True)
    ref = oracle.ls_interp(A32, x, None, w.cf, mu_h, w.caliber, rows=rows)
    got = tuple(to_np(t)[rows] for t in (Pc, Pv, ls, st))
    check_ls(got, ref, torch.float32, (x[rows] ** 2).sum(1))
    lsn = to_np(ls)
    assert abs(float(tot) - lsn[w.cf == 0].sum()) <= 1e-12 * lsn.sum()
    assert ad.status(clear=True) == 0


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_fullsize_bench_configuration(dt):
    """The step exactly as bench.py times it on workload 2: shapes from the
    autotuner on this matrix, the colour-phase start and sweeps, then the
    fused distances + strength + LS rows (distance_ls).  Last sweep and
    distances on sampled rows, the strength graph on every row, the LS rows
    on sampled rows, the F-row sum against the rows."""
    ad = lib()
    w = wl(2)
    A = w.A
    say("full-size bench configuration %s, workload %s" % (dt, w.name))
    Av = A if dt == torch.float64 else W.CSR(A.n, A.row_ptr, A.col,
                                             A.val.astype(np.float32).astype(np.float64))
    Ad = dev_csr(A, dt)
    color = torch.as_tensor(w.color, device="cuda")
    cf = torch.as_tensor(w.cf, device="cuda")
    try:
        ad.autotune(Ad, w.K, relax=w.relax, color=color, ncolors=w.ncolors, cf=cf,
                    caliber=w.caliber)
        ad.status(clear=True)
        Xp = to_np(run_setup(w, Ad, dt, w.sweeps - 1)).astype(np.float64)
        X = run_setup(w, Ad, dt, w.sweeps)
        x = to_np(X).astype(np.float64)
        rows = sample_rows(A.n, seed=7)
        want = oracle.color_gs_rows(Av, w.color, w.ncolors, Xp, x, rows)
        err = np.abs(x[rows] - want)
        if dt == torch.float32:
            Z = np.where((w.color == 0)[:, None], x, Xp)
            bound = np.maximum(row_abs_bound(Av, Z, Xp, 1.0, rows=rows),
                               row_abs_bound(Av, Xp, Xp, 1.0, rows=rows))
        else:
            bound = 1e-13 * np.abs(Xp).max() + 0 * err
        say("  last sweep: max err/bound %.3g" % np.max(err / bound))
        assert np.all(err <= bound)
        mu, strong, ns, Pc, Pv, ls, st, tot = ad.distance_ls(Ad, X, cf, w.caliber, theta=w.theta,
                                                             want_sum=True)
        mu_h = to_np(mu).astype(np.float64)
        saa = (x[rows] ** 2).sum(1)
        saa_e = np.repeat(saa, np.diff(A.row_ptr.astype(np.int64))[rows])
        check_mu(packed(A, mu_h, rows), oracle.algdist(Av, x, rows=rows), saa_e, dt, "sampled")
        s_ref, ns_ref = oracle.strength(A, mu_h, w.theta)
        assert np.array_equal(to_np(strong), s_ref) and np.array_equal(to_np(ns), ns_ref)
        ref = oracle.ls_interp(Av, x, None, w.cf, mu_h, w.caliber, rows=rows)
        got = tuple(to_np(t)[rows] for t in (Pc, Pv, ls, st))
        check_ls(got, ref, dt, saa)
        lsn = to_np(ls)
        assert abs(float(tot) - lsn[w.cf == 0].sum()) <= 1e-12 * lsn.sum()
        assert ad.status(clear=True) == 0
    finally:
        for kern in ("gs_phase", "algdist", "ls_interp", "distance_ls"):
            ad.set_launch(kern, dt, w.K, 0, 1, 1)


@pytest.mark.parametrize("i", [2, 3])
def test_fullsize_fp64_whole_path(i):
    ad = lib()
    w = wl(i)
    A = w.A
    say("full-size FP64 whole path, workload %s" % w.name)
    Ad = dev_csr(A, torch.float64)
    X = run_setup(w, Ad, torch.float64, w.sweeps)
    X0 = oracle.tv_init(A.n, w.K, w.tv_seed)
    if w.relax == "gs":
        xr, _ = oracle.color_gs(A, X0, w.color, w.ncolors, w.sweeps)
    else:
        xr, _ = oracle.jacobi(A, X0, w.omega, w.sweeps)
    x = to_np(X)
    del X0
    rel = np.max(np.abs(x - xr)) / np.max(np.abs(xr))
    say("  relaxation max rel err %.3g" % rel)
    assert rel <= 1e-12
    mu, strong, ns = ad.algebraic_distance(Ad, X, fuse=True, theta=w.theta)
    mu_h = to_np(mu)
    mu_ref = oracle.algdist(A, x)
    check_mu(mu_h, mu_ref, saa_per_edge(A, x), torch.float64, "all edges")
    s_ref, ns_ref = oracle.strength(A, mu_h, w.theta)
    assert np.array_equal(to_np(strong), s_ref) and np.array_equal(to_np(ns), ns_ref)
    cf = torch.as_tensor(w.cf, device="cuda")
    got = ad.ls_interp(Ad, X, cf, mu, w.caliber)
    ref = oracle.ls_interp(A, x, None, w.cf, mu_h, w.caliber)
    check_ls(tuple(to_np(t) for t in got), ref, torch.float64, (x * x).sum(1))


@pytest.mark.parametrize("i", [2, 3])
def test_fullsize_fp32_chain_against_fp64_chain(i):
    """The FP32 chain end to end (FP32 relaxation and distances, FP64 LS
    solves; the fused pass bench.py times) against the all-FP64 chain, at
    full size: the per-result statement bench.py reports (precision), with
    the bounds asserted where they hold for a chain whose test vectors differ
    by FP32 rounding of the relaxation:
      * a strong-mask flip only for an edge whose threshold margin lies
        inside twice the measured distance error of the edge and its row;
      * every LS row whose C_i agree has finite weights and functional, and
        at most 1% of the F rows change C_i (a change needs near-equal
        distances of two C-neighbours).
    The mu and weight error distributions are printed (the per-step bounds
    of 1e-4 and 1e-6 hold for identical inputs and are asserted in the
    per-step tests)."""
    import bench
    ad = lib()
    w = wl(i)
    A = w.A
    say("FP32 chain vs FP64 chain, workload %s" % w.name)
    out = {}
    cf = torch.as_tensor(w.cf, device="cuda")
    for dt in (torch.float32, torch.float64):
        Ad = dev_csr(A, dt)
        X = run_setup(w, Ad, dt, w.sweeps)
        mu, strong, ns, Pc, Pv, ls, st, _ = ad.distance_ls(Ad, X, cf, w.caliber, theta=w.theta)
        out[dt] = {"mu": to_np(mu), "strong": to_np(strong), "Pc": to_np(Pc), "Pv": to_np(Pv),
                   "ls": to_np(ls), "st": to_np(st)}
        del X, mu, strong, Pc, Pv
    assert ad.status(clear=True) == 0
    r = bench.precision_statement(w, out[torch.float32], out[torch.float64])
    say("  mu rel err: %s" % r["mu_rel_err"])
    say("  mask: %s" % r["mask"])
    say("  P_val scaled err: %s" % r["P_val_scaled_err"])
    say("  ls_val rel err: %s" % r["ls_val_rel_err"])
    assert r["mask"]["flips_outside_twice_measured_error"] == 0
    pv = r["P_val_scaled_err"]
    assert pv["rows_C_differ"] <= 0.01 * pv["F_rows"]
    assert np.isfinite(pv["max"]) and np.isfinite(r["ls_val_rel_err"]["max"])


def test_workload1_end_to_end_exact_config():
    """Workload 1 at its exact configuration (5-point Laplacian on a 32^2
    interior grid, K = 8, 4 weighted-Jacobi sweeps with omega = 2/3, all
    edges, theta = 0.25, caliber 4 on the red C/F split), FP64 and FP32,
    through the separate calls and the fused pass, against the oracle."""
    ad = lib()
    w = W.workload(1)
    A = w.A
    assert (A.n, A.nnz, A.n_edges, w.K, w.sweeps) == (1024, 4992, 3968, 8, 4)
    assert w.relax == "jacobi" and w.omega == pytest.approx(2.0 / 3.0) and w.theta == 0.25
    cf = torch.as_tensor(w.cf, device="cuda")
    X0 = oracle.tv_init(A.n, w.K, w.tv_seed)
    for dt in (torch.float64, torch.float32):
        say("workload 1 end to end, %s" % dt)
        Ad = dev_csr(A, dt)
        X = run_setup(w, Ad, dt, w.sweeps)
        x = to_np(X).astype(np.float64)
        if dt == torch.float64:
            xr, _ = oracle.jacobi(A, X0, w.omega, w.sweeps)
            assert np.max(np.abs(x - xr)) <= 1e-12 * np.max(np.abs(xr))
            x0 = to_np(run_setup(w, Ad, dt, 0))
            assert np.array_equal(x0, X0)
        else:
            # last sweep from the device's own previous iterate
            xp = to_np(run_setup(w, Ad, dt, w.sweeps - 1)).astype(np.float64)
            xr = oracle.jacobi_rows(A, xp, w.omega, np.arange(A.n, dtype=np.int32))
            assert np.all(np.abs(x - xr) <= row_abs_bound(A, xp, xp, w.omega))
        mu, strong, ns = ad.algebraic_distance(Ad, X, fuse=True, theta=w.theta)
        mu_h = to_np(mu).astype(np.float64)
        check_mu(mu_h, oracle.algdist(A, x), saa_per_edge(A, x), dt, "workload 1")
        s_ref, ns_ref = oracle.strength(A, mu_h, w.theta)
        assert np.array_equal(to_np(strong), s_ref) and np.array_equal(to_np(ns), ns_ref)
        got = ad.ls_interp(Ad, X, cf, mu, w.caliber)
        ref = oracle.ls_interp(A, x, None, w.cf, mu_h, w.caliber)
        check_ls(tuple(to_np(t) for t in got), ref, dt, (x * x).sum(1))
        f = ad.distance_ls(Ad, X, cf, w.caliber, theta=w.theta, want_sum=True)
        fm = to_np(f[0]).astype(np.float64)
        check_mu(fm, oracle.algdist(A, x), saa_per_edge(A, x), dt, "workload 1 fused")
        s_ref, ns_ref = oracle.strength(A, fm, w.theta)
        assert np.array_equal(to_np(f[1]), s_ref) and np.array_equal(to_np(f[2]), ns_ref)
        ref = oracle.ls_interp(A, x, None, w.cf, fm, w.caliber)
        check_ls(tuple(to_np(t) for t in f[3:7]), ref, dt, (x * x).sum(1))
        F = w.cf == 0
        tot = float(to_np(f[7])[0])
        assert abs(tot - ref[2][F].sum()) <= 1e-9 * abs(ref[2][F].sum())
        assert ad.status(clear=True) == 0
