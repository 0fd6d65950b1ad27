"""Host-side logic of bench.py, without a GPU: the one-GPU guard, the
algorithmic byte model, and the counter-summary reader (used only when its
source hash matches the current kernel sources)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1106_5990_amd import workloads as W  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_byte_model_on_a_small_anisotropic_grid():
    wl = W.workload(2, size=16)
    A = wl.A
    n, nnz, K = A.n, A.nnz, wl.K
    for s in (4, 8):
        kb = bench.kernel_bytes(wl, s)
        panel = n * K * s
        assert kb["jacobi"] == (n + 1) * 4 + nnz * (4 + s) + 2 * panel
        # two colour phases: together they read the CSR once, the panel twice
        # and write it once
        deg = np.diff(A.row_ptr.astype(np.int64))
        both = sum(int((wl.color == c).sum()) * 4 + int(deg[wl.color == c].sum()) * (4 + s)
                   + panel + int((wl.color == c).sum()) * K * s
                   + int((wl.color == c).sum()) * 4 / wl.sweeps for c in range(2))
        assert kb["gs_phase"] == pytest.approx(both / 2)
        F = wl.cf == 0
        assert kb["distance_ls"] == (n + 1) * 4 + nnz * 4 + panel + n + nnz * s + nnz + 4 * n \
            + n * wl.caliber * 12 + 12 * n
        step = bench.step_bytes(wl, s, kb)
        assert step == kb["tv_init"] + kb["distance_ls"] + kb["color_partition"] \
            + wl.sweeps * 2 * kb["gs_phase"]
        assert bench.step_bytes(wl, s, kb, fused=False) == pytest.approx(
            step - kb["distance_ls"] + kb["algdist"] + kb["ls_interp"])
        assert F.sum() > 0


def test_counter_summary_is_used_only_for_matching_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    body = ["# scale: 2.0 1.0",
            "kernel | dispatches | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch",
            "ad::gs_phase_perm_kernel<float, 16, 2> | 10 | 100 | 50",
            "ad::gs_phase_perm_kernel<float, 16, 4> | 30 | 300 | 150",
            "ad::dist_ls_kernel<float, 16, 1, 4, false> | 1 | 7 | 9"]
    here = os.path.join(str(tmp_path), "bench.py")
    monkeypatch.setattr(bench, "__file__", here)
    path = prof / "hbm_counters_x-fp32.txt"
    path.write_text("\n".join(["# source-hash: " + bench.source_hash()] + body) + "\n")
    # sources under tmp_path: none, so its hash differs from the real one
    monkeypatch.setattr(bench, "source_hash", lambda: "abc")
    assert bench.counter_traffic("x-fp32", "gs_phase") is None
    path.write_text("\n".join(["# source-hash: abc"] + body) + "\n")
    got = bench.counter_traffic("x-fp32", "gs_phase")
    # dispatch-weighted mean of (FETCH * 2 + WRITE) KiB
    want = (10 * (100 * 2 + 50) + 30 * (300 * 2 + 150)) / 40 * 1024
    assert got == pytest.approx(want)
    assert bench.counter_traffic("x-fp32", "distance_ls") == pytest.approx((7 * 2 + 9) * 1024)
    assert bench.counter_traffic("missing", "gs_phase") is None
    # a summary taken with another launch shape of the kernel is not used
    shp = {"gs_phase": {"lpr": 4, "iter": 2, "xcd": 0}}
    path.write_text("\n".join(["# source-hash: abc", "# shapes: " + json.dumps(shp)] + body) + "\n")
    assert bench.counter_traffic("x-fp32", "gs_phase", shapes=shp) == pytest.approx(want)
    other = {"gs_phase": {"lpr": 4, "iter": 4, "xcd": 16}}
    assert bench.counter_traffic("x-fp32", "gs_phase", shapes=other) is None
    assert bench.counter_traffic("x-fp32", "gs_phase", shapes="defaults") is None
    # families the summary does not record are not checked
    assert bench.counter_traffic("x-fp32", "distance_ls", shapes=other) == pytest.approx((7 * 2 + 9) * 1024)


def test_model_bytes_reproduce_the_planned_table():
    """The step byte model on the full-size anisotropic (9-point, 2048^2,
    K = 16, 5 sweeps) and 3D log-normal (160^3, K = 32, 4 sweeps) workloads:
    5.30 / 9.37 GB and 6.46 / 12.07 GB (FP32 / FP64); a colour phase is half
    a sweep."""
    w2 = W.workload(2)
    m32, m64 = bench.model_bytes(w2, 4), bench.model_bytes(w2, 8)
    assert m32["step"] / 1e9 == pytest.approx(5.30, abs=0.006)
    assert m64["step"] / 1e9 == pytest.approx(9.37, abs=0.006)
    assert m32["sweep"] / 1e6 == pytest.approx(855.4, abs=0.1)
    assert bench.kernel_model_bytes(w2, 4)["gs_phase"] == pytest.approx(m32["sweep"] / 2)
    w3 = W.workload(3)
    assert bench.model_bytes(w3, 4)["step"] / 1e9 == pytest.approx(6.46, abs=0.006)
    assert bench.model_bytes(w3, 8)["step"] / 1e9 == pytest.approx(12.07, abs=0.006)


@pytest.mark.parametrize("idx", [2, 3])
def test_threaded_oracle_pass_equals_the_single_threaded_one(idx):
    """The all-cores CPU baseline runs the oracle's row functions on row
    blocks in threads: bitwise the single-threaded pass."""
    import oracle
    wl = W.workload(idx, "f64", size=24 if idx == 2 else 10)
    a = bench.oracle_pass(oracle, wl, 1)
    b = bench.oracle_pass(oracle, wl, 4)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    for x, y in zip(a[3], b[3]):
        assert np.array_equal(x, y)


def test_precision_statement_counts_flips_by_band():
    """Host arithmetic of the FP32-vs-FP64 statement on a planted case."""
    wl = W.workload(1)
    A = wl.A
    rng = np.random.default_rng(0)
    mu64 = rng.random(A.nnz) + 0.5
    rid = A.row_ids()
    mu64[A.col == rid] = 0.0
    import oracle
    s64, _ = oracle.strength(A, mu64, wl.theta)
    mu32 = mu64 * (1 + 1e-7)
    s32 = s64.copy()
    n, cal = A.n, wl.caliber
    Pc = np.tile(np.arange(cal, dtype=np.int32), (n, 1))
    Pv = rng.random((n, cal))
    ls = rng.random(n)
    st = np.zeros(n, np.int32)
    r64 = {"mu": mu64, "strong": s64, "Pc": Pc, "Pv": Pv, "ls": ls, "st": st}
    Pv32 = Pv + 1e-8
    Pc32 = Pc.copy()
    Pc32[3] = -1  # one row whose C_i differ
    r32 = {"mu": mu32.astype(np.float32), "strong": s32, "Pc": Pc32, "Pv": Pv32, "ls": ls, "st": st}
    # flip one strong edge: it lies far from the threshold
    e = int(np.nonzero(s64)[0][0])
    r32["strong"] = s32.copy()
    r32["strong"][e] ^= 1
    out = bench.precision_statement(wl, r32, r64)
    assert out["mask"]["flips"] == 1
    assert out["mask"]["flips_outside_twice_measured_error"] == 1
    assert sum(out["mask"]["flips_by_margin"].values()) == 1
    F = wl.cf == 0
    assert out["P_val_scaled_err"]["rows_C_differ"] == int(F[3])
    assert out["P_val_scaled_err"]["max"] == pytest.approx(1e-8, rel=1e-3)
    assert out["mu_rel_err"]["max"] < 2e-7


def test_table1_cases():
    """The quality leg's copy of Table 1 (Sec. 5.5): three anisotropies
    times four angles, each with rho (gamma_g, gamma_o) for N = 32, 64, 128,
    every value in the range the table prints; spot entries as printed."""
    T = bench.TABLE1
    assert sorted({e for e, _ in T}) == [0.0, 1e-4, 0.1]
    assert set(bench.ALPHAS) == {a for _, a in T} == {"pi/4", "-pi/4", "pi/8", "0"}
    assert len(T) == 12
    for key, rows in T.items():
        assert len(rows) == 3, key
        for rho, gg, go in rows:
            assert 0.0 < rho < 1.0 and 0.2 < gg < 0.5 and 1.0 < go < 2.0, key
    assert T[(0.1, "pi/4")][0] == (.10, .35, 1.5)
    assert T[(1e-4, "0")][2] == (.06, .38, 1.7)
    assert T[(0.0, "pi/8")][1] == (.49, .38, 1.8)
