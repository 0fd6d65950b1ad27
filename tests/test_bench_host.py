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
