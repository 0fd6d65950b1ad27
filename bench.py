#!/usr/bin/env python3
"""Throughput of the algebraic-distance AMG setup hot path on one MI355X.

One step = the whole path over one synthetic operator resident in HBM:
  test-vector start + relaxation (setup_testvectors)
  -> per-edge distances with the fused strength graph (algebraic_distance)
  -> LS interpolation rows with their F-row sum (ls_interp).
The metric is edges/s: off-diagonal CSR entries (the directed pairs on which
distances are computed) per second of step time.

Default workload: the rotated anisotropic diffusion operator (alpha = pi/6,
eps = 1e-3) with the central 9-point stencil on a 2048 x 2048 grid, K = 16
test vectors, 5 red-black colour-phase Gauss-Seidel sweeps, theta = 0.25,
caliber 4 from the red C/F split; FP32 relaxation and distances with FP64
interpolation solves.  The plain FP64 path on the same workload is timed
beside it, and the CPU oracle on a bounded sample of the same workload on the
host cores.  Prints ONE JSON line.

  python bench.py [--steps K] [--warmup W] [--workload aniso2d|varcoef3d|laplace2d]
"""
import argparse
import json
import math
import os
import sys
import tempfile
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="aniso2d", choices=["aniso2d", "varcoef3d", "laplace2d"])
    ap.add_argument("--size", type=int, default=None, help="grid side override (tests only)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=None, help="grid side of the oracle sample")
    ap.add_argument("--graph", action="store_true", help="replay the step as a captured HIP graph")
    ap.add_argument("--no-graph-replay", action="store_true",
                    help="skip the extra graph-replay timing of the FP32 step")
    ap.add_argument("--batched", action="store_true",
                    help="run the batched leg (workload 4; the default unless --size is given)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched leg")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes instead of the autotuner's")
    ap.add_argument("--separate", action="store_true",
                    help="distances and LS rows as two calls instead of the fused pass")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file (JSON lines); shapes found there are used without "
                         "timing, new ones are appended (default: a fresh temporary file)")
    ap.add_argument("--batch-size", type=int, default=512)
    ap.add_argument("--batch-workers", type=int, default=None,
                    help="processes building the batch (default: up to 16; 1 builds it in this "
                         "process, as a run under a profiler must)")
    ap.add_argument("--adjoint", action="store_true",
                    help="also time the LS-loss forward and adjoint (workload 5; the default "
                         "unless --size is given)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device-to-device copy (a kernel of known traffic "
                         "for scaling hardware byte counters)")
    a = ap.parse_args()
    # the batched and adjoint legs run by default on the full-size workloads
    a.batched = not a.no_batched and (a.batched or a.size is None)
    a.adjoint = not a.no_adjoint and (a.adjoint or a.size is None)
    return a


WORKLOAD_INDEX = {"laplace2d": 1, "aniso2d": 2, "varcoef3d": 3}


def build_inputs(wl, dtype, torch, ad):
    A = ad.Csr.from_host(wl.A, dtype=dtype)
    dev = A.device
    n, nnz, K = wl.A.n, wl.A.nnz, wl.K
    buf = {
        "A": A,
        "X": torch.empty((n, K), dtype=dtype, device=dev),
        "mu": torch.empty(nnz, dtype=dtype, device=dev),
        "strong": torch.empty(nnz, dtype=torch.uint8, device=dev),
        "ns": torch.empty(n, dtype=torch.int32, device=dev),
        "cf": torch.as_tensor(wl.cf, device=dev),
        "Pc": torch.empty((n, wl.caliber), dtype=torch.int32, device=dev),
        "Pv": torch.empty((n, wl.caliber), dtype=torch.float64, device=dev),
        "ls": torch.empty(n, dtype=torch.float64, device=dev),
        "st": torch.empty(n, dtype=torch.int32, device=dev),
        "lsum": torch.empty(1, dtype=torch.float64, device=dev),
        "color": None if wl.color is None else torch.as_tensor(wl.color, device=dev),
    }
    return buf


def make_step(wl, b, ad, fused=True):
    """One pass of the path: test vectors, then distances with the strength
    row and the LS rows -- in one fused pass (distance_ls) or as the two
    separate calls."""
    def step():
        ad.setup_testvectors(b["A"], wl.K, seed=wl.tv_seed, relax=wl.relax, sweeps=wl.sweeps,
                             omega=wl.omega, color=b["color"], ncolors=wl.ncolors, out=b["X"])
        if fused:
            ad.distance_ls(b["A"], b["X"], b["cf"], wl.caliber, theta=wl.theta, mu=b["mu"],
                           strong=b["strong"], nstrong=b["ns"], P_col=b["Pc"], P_val=b["Pv"],
                           ls_val=b["ls"], row_status=b["st"], ls_sum=b["lsum"], want_sum=True)
            return
        ad.algebraic_distance(b["A"], b["X"], mu=b["mu"], fuse=True, theta=wl.theta,
                              strong=b["strong"], nstrong=b["ns"])
        ad.ls_interp(b["A"], b["X"], b["cf"], b["mu"], wl.caliber, P_col=b["Pc"], P_val=b["Pv"],
                     ls_val=b["ls"], row_status=b["st"], ls_sum=b["lsum"], want_sum=True)
    return step


def timed(step, steps, warmup, torch, ad, graph=False):
    """Run warmup steps, then time `steps` steps bracketed by synchronisation;
    per-kernel HIP events (the library's timing record) run over the same
    timed region."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    g = None
    if graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        g.replay()
        torch.cuda.synchronize()
    run = g.replay if g is not None else step
    ad.timing(not graph)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernels = ad.timing_report() if not graph else {}
    ad.timing(False)
    return e0.elapsed_time(e1) / steps, wall / steps * 1e3, kernels


def kernel_bytes(wl, s):
    """Algorithmic HBM bytes per launch of each kernel (s = panel bytes per
    value).  Every operand is read or written once; neighbour re-reads of the
    panel are taken to hit in cache."""
    A = wl.A
    n, nnz, K = A.n, A.nnz, wl.K
    rp = A.row_ptr.astype(np.int64)
    deg = np.diff(rp)
    panel = n * K * s
    out = {"tv_init": panel}
    out["jacobi"] = (n + 1) * 4 + nnz * (4 + s) + 2 * panel
    if wl.color is not None:
        # colour phases run on a colour-major copy of the CSR and permuted
        # panels: a phase reads its rows' pointers, permuted columns and
        # values, every panel row once (new rows of earlier colours, old
        # otherwise), writes its rows once, and in the last sweep reads its
        # rows' natural indices (averaged over the sweeps)
        per = []
        for c in range(wl.ncolors):
            rows = wl.color == c
            nc_, nnzc = int(rows.sum()), int(deg[rows].sum())
            per.append(nc_ * 4 + nnzc * (4 + s) + panel + nc_ * K * s + nc_ * 4 / wl.sweeps)
        out["gs_phase"] = float(np.mean(per))
        # colours and row pointers read by the count and scatter kernels,
        # row list, inverse permutation and colour-major row pointers
        # written, the entry copy's row starts, inverse and permuted starts,
        # the inverse table once, and the entries (columns, values) read and
        # written once
        out["color_partition"] = n * 4 * 11 + nnz * (8 + 2 * s)
        out["tv_init"] = panel + n * 4
    out["algdist"] = (n + 1) * 4 + nnz * 4 + panel + nnz * s + nnz + n * 4
    F = wl.cf == 0
    nnzF = int(deg[F].sum())
    out["ls_interp"] = (n + (n + 1) * 4 + nnzF * (4 + s + 1) + panel
                        + n * wl.caliber * (4 + 8) + n * (8 + 4))
    out["strength"] = (n + 1) * 4 + nnz * (4 + s + 1) + n * 4
    # fused pass: CSR structure, panel and C/F flags read once; mu, mask,
    # counts and the LS rows written once
    out["distance_ls"] = ((n + 1) * 4 + nnz * 4 + panel + n + nnz * s + nnz + n * 4
                          + n * wl.caliber * (4 + 8) + n * (8 + 4))
    return out


def step_bytes(wl, s, kb, fused=True):
    sweeps = wl.sweeps
    b = kb["tv_init"] + (kb["distance_ls"] if fused else kb["algdist"] + kb["ls_interp"])
    if wl.relax == "gs":
        b += kb["color_partition"] + sweeps * wl.ncolors * kb["gs_phase"]
    else:
        b += sweeps * kb["jacobi"]
    return b


KERNEL_SYMBOL = {"gs_phase": "gs_phase_perm_kernel", "jacobi": "jacobi_kernel",
                 "algdist": "algdist_kernel", "ls_interp": "ls_interp_kernel",
                 "tv_init": "start_perm_kernel", "distance_ls": "dist_ls_kernel",
                 "batch_jacobi": "batch_jacobi_kernel",
                 "batch_algdist": "batch_algdist_kernel"}


def source_hash():
    """Hash of the HIP sources: counter summaries are valid only for it."""
    import glob
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(here, "paper_1106_5990_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# launch-shape family (autotuner cache name) of each timed label
SHAPE_FAMILY = {"gs_phase": "gs_phase", "jacobi": "jacobi", "algdist": "algdist",
                "ls_interp": "ls_interp", "distance_ls": "distance_ls",
                "batch_jacobi": "batched", "batch_algdist": "batched_distance"}


def counter_traffic(workload_tag, label, ctype="float", shapes=None):
    """HBM bytes per launch of `label` from the committed rocprofv3 counter
    summary of this workload (FETCH_SIZE x its copy-calibration factor +
    WRITE_SIZE x its factor), or None if absent or taken on other sources.
    Only rows of the kernel instantiated for element type `ctype` count.
    When the summary records the launch shape it was taken with for the
    label's family and `shapes` (this run's) does not give the same one, the
    counters do not describe this run's launches: None."""
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "hbm_counters_%s.txt" % workload_tag)
    if not os.path.exists(path):
        return None
    rows, meta = [], {}
    for line in open(path):
        line = line.strip()
        if line.startswith("# source-hash:"):
            meta["hash"] = line.split(":", 1)[1].strip()
        elif line.startswith("# shapes:"):
            meta["shapes"] = json.loads(line.split(":", 1)[1])
        elif line.startswith("# scale:"):
            f, w = line.split(":", 1)[1].split()
            meta["fs"], meta["ws"] = float(f), float(w)
        elif line and not line.startswith("#") and "|" in line and not line.startswith("kernel"):
            rows.append([c.strip() for c in line.split("|")])
    if meta.get("hash") != source_hash() or "fs" not in meta:
        return None
    fam = SHAPE_FAMILY.get(label)
    if fam in meta.get("shapes", {}):
        if not isinstance(shapes, dict) or shapes.get(fam) != meta["shapes"][fam]:
            return None
    sym = KERNEL_SYMBOL.get(label)
    tot, cnt = 0.0, 0
    for r in rows:
        base, _, targs = r[0].partition("<")
        if sym and base.split("::")[-1] == sym and targs.startswith(ctype):
            d = int(r[1])
            tot += d * (float(r[2]) * meta["fs"] + float(r[3]) * meta["ws"]) * 1024.0
            cnt += d
    return tot / cnt if cnt else None


def btraffic(tag, label, shapes):
    """HBM bytes per launch of a batch kernel from the committed counter
    summary of the 512-matrix batch (FP32 only, same launch shape), or None."""
    if tag != "f32":
        return None
    tr = counter_traffic("rgg-batch-fp32", label, shapes=shapes)
    return None if tr is None else int(tr)


def batched_leg(args, torch, ad, W, mats):
    """Workload 4: the RGG batch through relax_algdist_batched.  The launch
    shape is picked by the batch autotuner (outside the timed region); the
    timed region replays the captured stage graph; a separate pass with
    per-kernel timing gives the sweep kernel's rate for the roofline."""
    K, S, om, th = W.BATCH_K, W.BATCH_SWEEPS, W.BATCH_OMEGA, W.BATCH_THETA
    E = sum(m.n_edges for m in mats)
    rows = sum(m.n for m in mats)
    ents = sum(m.nnz for m in mats)
    nm = len(mats)
    out = {"workload": "rgg-batch-%d (n log-uniform 2k-200k, mean degree U[4,29]), K=%d, %d Jacobi "
                       "sweeps, theta=%g" % (nm, K, S, th),
           "matrices": nm, "rows": rows, "nnz": ents, "edges": E}
    cache = args.tune_cache or os.path.join(tempfile.mkdtemp(prefix="algdist_tune_"), "batch.jsonl")
    for tag, dt, s in (("f32", torch.float32, 4), ("f64", torch.float64, 8)):
        print("[bench] batched leg %s: autotune" % tag, file=sys.stderr, flush=True)
        dm = [ad.Csr.from_host(m, dtype=dt) for m in mats]
        ad.autotune_batched(dm, K, S, cache_json=cache)
        tuned = [json.loads(l) for l in open(cache)]
        shape = {fam: {k: e[k] for k in ("lpr", "iter", "xcd")}
                 for fam in ("batched", "batched_distance")
                 for e in tuned if e["kernel"] == fam and e["dtype"] == ad._dtype_code(dt)}
        X = torch.empty((rows, K), dtype=dt, device="cuda")
        mu = torch.empty(ents, dtype=dt, device="cuda")
        st = torch.empty(ents, dtype=torch.uint8, device="cuda")
        ns = torch.empty(rows, dtype=torch.int32, device="cuda")

        def run():
            ad.relax_algdist_batched(dm, K, seed=W.TV_SEED_BASE + 4, sweeps=S, omega=om, theta=th,
                                     X=X, mu=mu, strong=st, nstrong=ns)
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        steps = max(3, args.steps // 2)
        print("[bench] batched leg %s: %d steps" % (tag, steps), file=sys.stderr, flush=True)
        e0.record()
        for _ in range(steps):
            run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        ad.timing(True)
        run()
        torch.cuda.synchronize()
        rep = ad.timing_report()
        ad.timing(False)
        rp = (rows + nm) * 4
        panel = rows * K * s
        by = {"batch_tv_init": panel,
              "batch_jacobi": rp + ents * (4 + s) + 2 * panel,
              "batch_algdist": rp + ents * 4 + panel + ents * (s + 1) + rows * 4}
        kern = {}
        for lab, b in by.items():
            cnt, tot = rep[lab]
            kern[lab] = {"launches": cnt, "avg_ms": round(tot / cnt, 5),
                         "GB/s": round(b / (tot / cnt * 1e-3) / 1e9, 1)}
        step_bytes = by["batch_tv_init"] + S * by["batch_jacobi"] + by["batch_algdist"]
        out[tag] = {"value": round(E / (ms * 1e-3), 1), "ms_per_step": round(ms, 4),
                    "shapes": shape,
                    "step_hbm_frac": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "kernels": kern,
                    "roofline": {"bound": "hbm", "kernel": "batch_jacobi",
                                 "achieved": kern["batch_jacobi"]["GB/s"], "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s",
                                 "frac": round(kern["batch_jacobi"]["GB/s"] / HBM_PEAK_GBS, 4),
                                 "traffic": btraffic(tag, "batch_jacobi", shape),
                                 "algorithmic_bytes_per_launch": int(by["batch_jacobi"])},
                    "device_status_bits": ad.status(clear=True)}
        del dm, X, mu, st, ns
        torch.cuda.empty_cache()
    out["speedup_f32_over_f64"] = round(out["f64"]["ms_per_step"] / out["f32"]["ms_per_step"], 3)
    return out


def adjoint_leg(args, torch, ad, W):
    """Workload 5: L(values, omega) through LSInterpLoss (FP64, checkpoints
    every 2 sweeps) and its gradient with respect to every stored value and
    omega; forward and forward + backward timed separately."""
    wl = W.workload(5)
    A = wl.A
    dev = "cuda"
    rp = torch.as_tensor(A.row_ptr, device=dev)
    col = torch.as_tensor(A.col, device=dev)
    cf = torch.as_tensor(wl.cf, device=dev)
    vals = torch.as_tensor(A.val, dtype=torch.float64, device=dev).requires_grad_(True)
    om = torch.tensor(wl.omega, dtype=torch.float64, device=dev, requires_grad=True)

    def fwd():
        return ad.LSInterpLoss.apply(vals, om, rp, col, wl.K, wl.tv_seed, wl.sweeps, cf,
                                     wl.caliber, 2)

    def both():
        return torch.autograd.grad(fwd(), (vals, om))
    out = {"workload": wl.name, "K": wl.K, "sweeps": wl.sweeps, "edges": A.n_edges}
    for tag, fn in (("forward", fwd), ("forward_backward", both)):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[tag + "_ms"] = round(e0.elapsed_time(e1) / args.steps, 4)
    out["backward_over_forward"] = round(out["forward_backward_ms"] / out["forward_ms"] - 1.0, 3)
    out["device_status_bits"] = ad.status(clear=True)
    return out


def cpu_baseline(idx, side, min_seconds=10.0, max_passes=8):
    """The oracle, as it stands, on a bounded sample of the same workload
    (the same operator family and parameters, on a smaller grid when `side`
    is given): whole-path passes are repeated until at least `min_seconds`
    of CPU work has been timed (at most `max_passes`)."""
    import oracle
    from paper_1106_5990_amd import workloads as W
    wl = W.workload(idx, "f64", size=side)
    A = wl.A
    passes, dt = 0, 0.0
    while passes < max_passes and (passes == 0 or dt < min_seconds):
        t0 = time.perf_counter()
        X0 = oracle.tv_init(A.n, wl.K, wl.tv_seed)
        if wl.relax == "gs":
            X, _ = oracle.color_gs(A, X0, wl.color, wl.ncolors, wl.sweeps)
        else:
            X, _ = oracle.jacobi(A, X0, wl.omega, wl.sweeps)
        mu = oracle.algdist(A, X)
        oracle.strength(A, mu, wl.theta)
        oracle.ls_interp(A, X, None, wl.cf, mu, wl.caliber)
        dt += time.perf_counter() - t0
        passes += 1
        print("[bench]   cpu baseline pass %d: %.1f s" % (passes, dt), file=sys.stderr, flush=True)
    return {"value": passes * A.n_edges / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": "%s (%d rows, %d edges), %d whole-path passes, single-threaded C oracle, "
                      "%.1f s" % (wl.name, A.n, A.n_edges, passes, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (only its sharding "
              "design); got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)
    from paper_1106_5990_amd import workloads as W
    batch = None
    if args.batched:
        # the batch members are built in worker processes before anything
        # touches the GPU
        print("[bench] building the batch", file=sys.stderr, flush=True)
        workers = args.batch_workers or min(16, os.cpu_count() or 1)

        def progress(k):
            if k % 128 == 0:
                print("[bench]   %d members built" % k, file=sys.stderr, flush=True)
        batch = W.batch_workload(args.batch_size, workers=workers, progress=progress)
    import torch
    from paper_1106_5990_amd import algdist as ad

    idx = WORKLOAD_INDEX[args.workload]
    print("[bench] building %s" % args.workload, file=sys.stderr, flush=True)
    wl = W.workload(idx, "f32", size=args.size)
    E = wl.A.n_edges

    res = {}
    for tag, dtype, steps in (("f32", torch.float32, args.steps),
                              ("f64", torch.float64, max(3, args.steps // 2))):
        if tag == "f64" and args.no_fp64:
            continue
        b = build_inputs(wl, dtype, torch, ad)
        step = make_step(wl, b, ad, fused=not args.separate)
        if not args.no_autotune:
            # launch shapes picked by the library's autotuner on this matrix
            # (outside the timed region)
            print("[bench] autotune %s" % tag, file=sys.stderr, flush=True)
            cache = args.tune_cache or os.path.join(tempfile.mkdtemp(prefix="algdist_tune_"),
                                                    "shapes.jsonl")
            ad.autotune(b["A"], wl.K, relax=wl.relax, color=b["color"], ncolors=wl.ncolors,
                        cf=b["cf"], caliber=wl.caliber, cache_json=cache)
            code = ad._dtype_code(dtype)
            shapes = {e["kernel"]: {k: e[k] for k in ("lpr", "iter", "xcd")}
                      for e in (json.loads(l) for l in open(cache)) if e["dtype"] == code}
        else:
            shapes = "defaults"
        print("[bench] timing %s leg: %d warmup + %d steps" % (tag, args.warmup, steps),
              file=sys.stderr, flush=True)
        ms, wall_ms, kern = timed(step, steps, args.warmup, torch, ad, graph=args.graph)
        bits = ad.status(clear=True)
        gms = None
        if tag == "f32" and not args.graph and not args.no_graph_replay:
            # the same step captured once and replayed (no per-kernel events)
            print("[bench] timing %s leg as a graph replay: %d steps" % (tag, steps),
                  file=sys.stderr, flush=True)
            gms, _, _ = timed(step, steps, 1, torch, ad, graph=True)
            bits |= ad.status(clear=True)
        s = 4 if dtype == torch.float32 else 8
        kb = kernel_bytes(wl, s)
        res[tag] = {"ms": ms, "wall_ms": wall_ms, "kernels": kern, "kb": kb, "shapes": shapes,
                    "graph_ms": gms,
                    "step_bytes": step_bytes(wl, s, kb, fused=not args.separate), "status": bits, "steps": steps}
        del b, step
        torch.cuda.empty_cache()

    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    main_leg = res["f32"]
    kern = main_leg["kernels"]
    ms = main_leg["ms"]
    value = E / (ms * 1e-3)
    roof = None
    kstats = {}
    for lab, (cnt, tot) in kern.items():
        avg = tot / cnt
        by = main_leg["kb"].get(lab)
        kstats[lab] = {"launches_per_step": cnt / main_leg["steps"], "avg_ms": round(avg, 5),
                       "GB/s": None if by is None else round(by / (avg * 1e-3) / 1e9, 1)}
    if kern:
        dom = max(kern, key=lambda k: kern[k][1])
        cnt, tot = kern[dom]
        avg = tot / cnt
        ach = main_leg["kb"][dom] / (avg * 1e-3) / 1e9
        tr = (counter_traffic("%s-fp32" % args.workload, dom, shapes=main_leg["shapes"])
              if args.size is None else None)
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": None if tr is None else int(tr),
                "algorithmic_bytes_per_launch": int(main_leg["kb"][dom]),
                "avg_launch_ms": round(avg, 5)}
    out = {
        "metric": "edges/s (relax+algdist+ls_interp)",
        "value": round(value, 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": main_leg["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": wl.A.n, "nnz": wl.A.nnz, "edges": E, "K": wl.K,
                   "relax": "%d %s sweeps" % (wl.sweeps, "red-black colour-phase GS" if wl.relax == "gs"
                                              else "Jacobi omega=%.3g" % wl.omega),
                   "theta": wl.theta, "caliber": wl.caliber,
                   "precision": "FP32 relaxation and distances, FP64 interpolation solves",
                   "graph": bool(args.graph), "launch_shapes": main_leg["shapes"]},
        "roofline": roof,
        "step_hbm_frac": round(main_leg["step_bytes"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "kernels": kstats,
        "wall_ms_per_step": round(main_leg["wall_ms"], 4),
        "device_status_bits": main_leg["status"],
        "graph_replay": None if main_leg["graph_ms"] is None else {
            "value": round(E / (main_leg["graph_ms"] * 1e-3), 1),
            "ms_per_step": round(main_leg["graph_ms"], 4)},
    }
    if "f64" in res:
        r = res["f64"]
        out["fp64_plain"] = {"value": round(E / (r["ms"] * 1e-3), 1), "ms_per_step": round(r["ms"], 4),
                             "step_hbm_frac": round(r["step_bytes"] / (r["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                             "speedup_f32_over_f64": round(r["ms"] / ms, 3)}
    if args.batched:
        print("[bench] batched leg (workload 4)", file=sys.stderr, flush=True)
        out["batched"] = batched_leg(args, torch, ad, W, batch)
    if args.adjoint:
        print("[bench] adjoint leg (workload 5)", file=sys.stderr, flush=True)
        out["adjoint"] = adjoint_leg(args, torch, ad, W)
    if not args.no_cpu_baseline:
        side = args.cpu_sample or args.size or {1: 32, 2: 2048, 3: 160}[idx]
        print("[bench] cpu baseline: oracle on a side-%d sample" % side, file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(idx, side)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
