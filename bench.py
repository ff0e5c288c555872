#!/usr/bin/env python
"""Benchmark of the RBF terrain hot path on one MI355X.

One step is one odometry frame on a 50 x 50 m map with 10,000 centers
(voxel selection at 0.5 m): the frame's 20,000 ground points are spatially
sorted and absorbed by the Kalman-form recursive ridge update (dense
10k x 10k covariance, FP64), then height, gradient, residual and pose
Jacobian are evaluated at the frame's 200,000 scan points. Inputs are
generated before the timed region and are resident in HBM.

Prints one JSON line: scan updates/s (value), the roofline of the dominant
kernel (the FP64 MFMA covariance product, timed with HIP events on the
library's stream), rbf_eval throughput in FP64 and FP32, and the FP64 CPU
oracle timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

METRIC = ("rbf_eval Mpts/s + scan updates/s (10k centers) at stated err; "
          "% HBM/MFMA peak")
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# HBM bytes of one covariance product (k_syrk_f64 over whole rounds of tiles +
# k_syrk_f64_tail over the rest) at N = 10,000, batch 1024, from rocprofv3
# FETCH_SIZE (x2.0, the copy-kernel calibration) + WRITE_SIZE (x1.0); summary
# in profiles/k_syrk_and_k_eval_hbm_bytes_odometry_n10k.txt. Valid only for
# those kernel versions and that shape (None otherwise).
SYRK_F64_TRAFFIC = {(10000, 1024): 1.9686e9 + 0.8004e9}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--frames", type=int, default=0,
                    help="distinct frames generated (0 = one per warmup and timed step)")
    ap.add_argument("--eval-reps", type=int, default=500)
    ap.add_argument("--eval-fill", type=int, default=20_000_000,
                    help="points of the GPU-filling evaluation launch (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--patches", type=int, default=256,
                    help="patches in the batched-form leg (0 = skip; 256 = full workload)")
    ap.add_argument("--no-tune", action="store_true",
                    help="batched leg with 4 branches and batch 1024 instead of autotuning")
    ap.add_argument("--streams", type=int, default=1, choices=(1, 2),
                    help="schedule of the update (2: next batch's chain overlaps the "
                         "covariance product on a second stream)")
    ap.add_argument("--no-other-schedule", action="store_true",
                    help="skip the FP64 leg with the other update schedule")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip timing the rows outside the per-frame step")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the FP32/BF16 covariance-product legs")
    ap.add_argument("--no-active", action="store_true",
                    help="skip the active-rows update leg")
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 launches), the "
                         "reference for scaling HBM byte counters, and exit")
    return ap.parse_args()


def log(msg):
    """Progress on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def copy_calibrate(mib):
    """A plain copy of known size: each launch reads and writes mib MiB."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_launch": n * 4, "copy_bytes_written_per_launch": n * 4,
                      "launches": 5}), flush=True)


def batched_leg(ctx, api, synth, n_patches, tune, chains=1, tile="128", batch=1024):
    """Many uneven patches: one hipGraph launch of the batched plan vs the
    same update + evaluation calls issued one patch after another."""
    import torch
    from paper_2509_26222_amd import tune as T

    p = api.Params()
    _, raw = synth.patches_case(seed=4, count=n_patches)

    def build():
        out = []
        for r in raw:
            grid = ctx.grid(p, torch.from_numpy(r.centers).cuda())
            N = grid.N
            # points in bin order (setup, untimed), as the odometry frames are
            xs, zs, _ = ctx.sort_points(grid, torch.from_numpy(r.xy).cuda(),
                                        torch.from_numpy(r.z).cuda())
            pts = torch.cat([xs, zs[:, None]], 1).float().contiguous()
            Q = pts.shape[0]
            out.append(dict(grid=grid,
                            w=torch.zeros(N, dtype=torch.float64, device="cuda"),
                            P=torch.eye(N, dtype=torch.float64, device="cuda") * (p.R / p.lam),
                            xy=xs, z=zs,
                            pts=pts, pose=(__import__("numpy").eye(3),
                                           __import__("numpy").zeros(3)),
                            f=torch.empty(Q, dtype=torch.float32, device="cuda"),
                            grad=torch.empty((Q, 2), dtype=torch.float32, device="cuda"),
                            resid=torch.empty(Q, dtype=torch.float32, device="cuda"),
                            jac=torch.empty((Q, 6), dtype=torch.float32, device="cuda")))
        return out

    patches = build()
    table = None
    if tune:
        sample = patches[:: max(1, len(patches) // 16)]
        (chains, tile, batch), table = T.tune_batched(
            ctx, p, sample, chains=(1, 2, 4), tiles=("auto", "128", "sub"),
            batches=(512, 1024, 2048), reps=1)
    # sequential plain calls, one patch after another: with the plan's Kalman
    # batch (the same arithmetic, bit for bit), and with each batch size the
    # tuner tries, the best of which is the stricter baseline
    def sequential(b):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for q in patches:
            ctx.update(p, q["grid"], q["w"], q["P"], q["xy"], q["z"], batch=b, sync=False)
            ctx.eval(p, q["grid"], q["w"], q["pts"], pose=q["pose"])
        torch.cuda.synchronize()
        ctx.sync_status()
        return time.perf_counter() - t0

    seq_by_batch = {b: sequential(b) for b in sorted({512, 1024, 2048, batch})}
    t_seq = seq_by_batch[batch]
    plan = api.Batched(ctx, p, patches, dim=3, eval_prec="f32", gemm_prec="f64",
                       tile=tile, chains=chains, default_batch=batch)
    plan.run()  # capture + first run
    plan.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run()
    plan.sync()
    t_graph = time.perf_counter() - t0
    plan.close()
    t_best = min(seq_by_batch.values())
    out = {"patches": len(patches), "chains": chains, "tile": tile, "batch": batch,
           "sequential_s": t_seq, "graph_s": t_graph, "speedup": t_seq / t_graph,
           "sequential_s_by_batch": {str(b): t for b, t in seq_by_batch.items()},
           "speedup_vs_best_sequential": t_best / t_graph,
           "update_points": int(sum(q["xy"].shape[0] for q in patches))}
    if table:
        out["tuning"] = {f"{c}x{t}x{b}": round(v, 4) for (c, t, b), v in table.items()}
    del patches
    torch.cuda.empty_cache()
    return out


def rows_leg(ctx, api, synth, L, od, allxy, centers, grid, frame, w, p, reps=3):
    """Every hot-path row not inside the per-frame step, timed on its own at
    its workload size (wall time of the library calls, synchronised): center
    selection and binning over the odometry map, Phi and Gram assembly of a
    frame, the sparse solve of the 40k-center information form (FP64 factor,
    FP64 refinement to 1e-10), the adjoint of the evaluation and the growing
    selection on one frame."""
    import torch
    import numpy as np

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    out = {}
    M = allxy.shape[0]
    t = timed(lambda: ctx.select_centers(allxy, od.roi, 0.5, 0.5, 4, L.SELECT_VOXEL))
    out["a1_select_centers_voxel"] = {"ms": t * 1e3, "points": M, "mpts_s": M / t / 1e6}
    t = timed(lambda: ctx.select_centers(allxy, od.roi, 0.5, 0.5, 4, L.SELECT_RADIUS))
    out["a1_select_centers_radius"] = {"ms": t * 1e3, "points": M, "mpts_s": M / t / 1e6}
    t = timed(lambda: ctx.grid(p, centers).close())
    out["a2_bin_centers"] = {"ms": t * 1e3, "centers": int(centers.shape[0])}
    xy, z, pts, pose = frame
    # growing center set: one frame's points added to running counts
    nodes = int(round((od.roi[2] - od.roi[0]) / 0.5 * (od.roi[3] - od.roi[1]) / 0.5))
    counts = torch.zeros(nodes, dtype=torch.int32, device=xy.device)

    def grow_select():
        counts.zero_()
        ctx.select_centers_grow(xy, od.roi, 0.5, 0.5, 4, counts, mode=L.SELECT_VOXEL)

    t = timed(grow_select)
    out["next_select_centers_grow"] = {"ms": t * 1e3, "points": int(xy.shape[0])}
    t = timed(lambda: ctx.assemble_phi(p, grid, xy))
    out["a3_assemble_phi"] = {"ms": t * 1e3, "points": int(xy.shape[0])}
    t = timed(lambda: ctx.gram_pattern(p, grid))
    rowptr, colidx = ctx.gram_pattern(p, grid)
    out["a3_gram_pattern"] = {"ms": t * 1e3, "nnz": int(colidx.shape[0])}
    t = timed(lambda: ctx.assemble_gram(p, grid, xy, z, rowptr, colidx))
    out["a3_assemble_gram"] = {"ms": t * 1e3, "points": int(xy.shape[0])}
    gf = torch.ones(pts.shape[0], dtype=pts.dtype, device=pts.device)
    dw = torch.zeros_like(w)
    dpose = torch.zeros(6, dtype=torch.float64, device=pts.device)
    t = timed(lambda: ctx.eval_adjoint(p, grid, w, pts, pose=pose, gbar_f=gf, gbar_r=gf,
                                       d_w=dw, d_pose=dpose))
    out["a12_adjoint"] = {"ms": t * 1e3, "points": int(pts.shape[0]),
                          "mpts_s": pts.shape[0] / t / 1e6}
    # a9 on the 40k-center map: information form of 800k points
    case = synth.large_case(3)
    g40 = ctx.grid(p, torch.from_numpy(case.centers).cuda())
    lxy, lz = synth.large_points(case, 800_000)
    lxy, lz = torch.from_numpy(lxy).cuda(), torch.from_numpy(lz).cuda()
    rp, ci = ctx.gram_pattern(p, g40)
    vals, b = ctx.assemble_gram(p, g40, lxy, lz, rp, ci)
    t = timed(lambda: ctx.assemble_gram(p, g40, lxy, lz, rp, ci))
    out["a3_assemble_gram_40k"] = {"ms": t * 1e3, "points": 800_000, "nnz": int(ci.shape[0])}
    res = {}

    def solve():
        x, rel, it, st = ctx.solve(rp, ci, vals, b, rtol=1e-10, max_iter=10, inner="f64")
        res.update(rel=rel[0], it=it)

    t = timed(solve)
    out["a9_solve_40k"] = {"ms": t * 1e3, "centers": g40.N, "relres": res["rel"],
                           "refine_sweeps": res["it"], "inner": "f64", "method": "banded"}
    # the same solve by nested dissection: the pattern analysed once (host),
    # then factor + solves + refinement per call
    t0 = time.perf_counter()
    plan = ctx.solve_plan(rp, ci)
    t_plan = time.perf_counter() - t0
    for inner in ("f64",):
        def solve_nd():
            x, rel, it, st = plan.run(vals, b, rtol=1e-10, max_iter=20, inner=inner)
            res.update(rel=rel[0], it=it)

        t = timed(solve_nd)
        out[f"a9_solve_40k_nd_{inner}"] = {
            "ms": t * 1e3, "centers": g40.N, "relres": res["rel"], "refine_sweeps": res["it"],
            "inner": inner, "method": "nested dissection", "plan_ms": t_plan * 1e3,
            **plan.info()}
    plan.close()
    g40.close()
    return out


def _host_cpu():
    """Host CPU model name and the number of cores the process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:  # pragma: no cover
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        nproc = os.cpu_count() or 1
    return model, nproc


def cpu_baseline(od, centers_np, p, first, pcols, frame0, batches=3, eval_pts=2000):
    """The FP64 oracle, as it stands, on a bounded sample of one frame:
    `batches` Kalman batches of the update and `eval_pts` evaluation points,
    scaled to one frame (20k update points, 200k evaluation points), with
    all host threads and again with one thread (one batch, a quarter of the
    points). The same leg checks the GPU state after the first frame (from
    the prior) against the oracle: the batch ridge solution of that frame
    (w = calH^{-1} b, P = R calH^{-1} on sampled columns) by a sparse solve,
    and the heights it implies at 2000 of the frame's scan points."""
    import numpy as np
    import oracle as O
    from threadpoolctl import threadpool_info, threadpool_limits
    cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    model, nproc = _host_cpu()
    B = 1024
    xy, z = od.ground(0)
    N = centers_np.shape[0]

    def sample(nb, ne):
        w0, P0 = O.initial_state(N, p.lam, p.R)
        m = nb * B
        t0 = time.perf_counter()
        O.kalman_update(w0, P0, xy[:m], z[:m], centers_np, p.sigma, p.cutoff, 0.0, p.R,
                        batch=B)
        t_upd = time.perf_counter() - t0
        pts, R, t = od.scan(0, n=ne)
        t0 = time.perf_counter()
        O.eval_pose(pts, R, t, 0.0, centers_np, w0 + 0.1, p.sigma, p.cutoff)
        t_ev = time.perf_counter() - t0
        per_frame = t_upd * (od.GROUND_PER_FRAME / m) + t_ev * (od.SCAN_PER_FRAME / ne)
        return per_frame, t_upd, t_ev

    per_frame, t_upd, t_ev = sample(batches, eval_pts)
    with threadpool_limits(limits=1):
        per_frame1, t_upd1, t_ev1 = sample(1, eval_pts // 4)
    out = {
        "value": 1.0 / per_frame, "unit": "scan updates/s", "cores": int(cores),
        "kind": "oracle",
        "sample": (f"frame 0: {batches} of {math.ceil(od.GROUND_PER_FRAME / B)} Kalman "
                   f"batches ({batches * B} of {od.GROUND_PER_FRAME} points, dense P "
                   f"{N}x{N}) in {t_upd:.1f} s and {eval_pts} of {od.SCAN_PER_FRAME} scan "
                   f"points (f, grad, r, J) in {t_ev:.1f} s, scaled to one frame; one "
                   f"thread: 1 batch in {t_upd1:.1f} s and {eval_pts // 4} points in "
                   f"{t_ev1:.1f} s"),
        "eval_mpts_s": eval_pts / t_ev / 1e6,
        "value_1thread": 1.0 / per_frame1,
        "host_cpu": model,
        "nproc": nproc,
    }
    # ---- the GPU's first frame against the oracle's batch ridge solution
    xy0, z0 = xy, z
    H, b = O.gram(xy0, z0, centers_np, p.sigma, p.cutoff, 0.0, p.lam, sparse=True)
    E = np.zeros((N, pcols.shape[0] + 1))
    E[pcols, np.arange(pcols.shape[0])] = 1.0
    E[:, -1] = b
    X = O.spd_solve(H, E)
    Pref, wref = p.R * X[:, :-1], X[:, -1]
    spts = frame0[2][:2000].double().cpu().numpy()
    R0, t0_ = frame0[3]
    qxy = O.to_world(spts, R0, t0_)[:, :2]
    f_ref = O.eval_height_grad(qxy, centers_np, wref, p.sigma, p.cutoff)[0]
    err = {"reference": ("first frame from the prior (20k points): oracle batch ridge "
                         "solution by sparse LU; P on 16 sampled columns; heights at 2000 "
                         "scan points from the oracle's evaluation of each w")}
    for prec, st in first.items():
        wg = st["w"].cpu().numpy()
        Pg = st["P"].cpu().numpy()
        e = {"w_rel": float(np.linalg.norm(wg - wref) / np.linalg.norm(wref)),
             "P_cols_max_abs": float(np.abs(Pg - Pref).max()),
             "P_cols_rel": float(np.linalg.norm(Pg - Pref) / np.linalg.norm(Pref)),
             "height_max_m": float(np.abs(O.eval_height_grad(qxy, centers_np, wg, p.sigma,
                                                             p.cutoff)[0] - f_ref).max())}
        if "w_refined" in st:
            wr = st["w_refined"].cpu().numpy()
            e["w_rel_refined"] = float(np.linalg.norm(wr - wref) / np.linalg.norm(wref))
            e["height_max_m_refined"] = float(np.abs(
                O.eval_height_grad(qxy, centers_np, wr, p.sigma, p.cutoff)[0] - f_ref).max())
        err[prec] = e
    out["err"] = err
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the multi-GPU "
                                   "sharding of the path is a design note, not built"}))
        sys.exit(2)
    if args.copy_calibrate:
        copy_calibrate(args.copy_calibrate)
        return
    import numpy as np
    import torch

    from paper_2509_26222_amd import _lib as L
    from paper_2509_26222_amd import api, synth

    torch.cuda.init()
    ctx = api.Context(0)
    p = api.Params()
    od = synth.OdometryCase()
    dev = torch.device("cuda:0")

    # ---- setup (untimed): centers by voxel selection over all frames
    allxy = np.concatenate([od.ground_xy(k) for k in range(od.N_FRAMES)])
    centers = ctx.select_centers(torch.from_numpy(allxy).to(dev), od.roi, 0.5, 0.5, 4,
                                 L.SELECT_VOXEL)
    N = centers.shape[0]
    grid = ctx.grid(p, centers.contiguous())
    # the selected centers are nodes of the 0.5 m candidate mesh: the
    # evaluations run in the mesh form (the binned form is timed beside it)
    grid.set_mesh_roi(od.roi, 0.5)
    nfr = args.frames if args.frames > 0 else args.steps + args.warmup
    nfr = max(1, min(nfr, args.steps + args.warmup))
    frames = []
    for k in range(nfr):
        xy, z = od.ground(k)
        pts, R, t = od.scan(k)
        frames.append((torch.from_numpy(xy).to(dev), torch.from_numpy(z).to(dev),
                       torch.from_numpy(pts).to(dev), (R, t)))
    w = torch.zeros(N, dtype=torch.float64, device=dev)
    P = torch.empty((N, N), dtype=torch.float64, device=dev)
    log(f"setup done: {N} centers, {nfr} frames")

    # information form (center-pair pattern) for the refinement of the
    # mixed-precision legs; depends only on the centers
    rowptr, colidx = ctx.gram_pattern(p, grid)
    hvals = torch.zeros(colidx.shape[0], dtype=torch.float64, device=dev)
    hb = torch.zeros(N, dtype=torch.float64, device=dev)
    refine_log = {}
    n_act = []
    # state after the first frame from the prior, for the oracle comparison
    # of the cpu_baseline leg: w (before refinement in the mixed legs), w
    # after refinement, and sampled columns of P
    pcols = torch.as_tensor(np.sort(np.random.default_rng(5).choice(N, 16, replace=False)),
                            device=dev)
    first = {}
    step_ms = {}

    def run_sequence(gemm_prec, streams=args.streams, active=False, joseph=False):
        """Warmup + timed frames from the prior (w = 0, P = (R/lambda) I).
        Low-precision covariance products are followed by the FP64
        refinement of w against the accumulated information form. With
        active=True each frame is absorbed by the active-rows form; with
        joseph=True (FP32 products) the covariance update takes the Joseph
        form."""
        label = gemm_prec + ("_joseph" if joseph else "")
        ctx.set_update_streams(streams)
        ctx.set_update_joseph(joseph)
        w.zero_()
        P.zero_()
        P.diagonal().fill_(p.R / p.lam)
        hvals.zero_()
        hb.zero_()
        sweeps = []
        n_act.clear()

        def step(k):
            xy, z, pts, pose = frames[k % nfr]
            xs, zs, _ = ctx.sort_points(grid, xy, z)
            if active:
                n_act.append(ctx.update_active(p, grid, w, P, xs, zs, batch=args.batch,
                                               gemm_prec=gemm_prec)[1])
            else:
                ctx.update(p, grid, w, P, xs, zs, batch=args.batch, gemm_prec=gemm_prec,
                           sync=False)
            if k == 0 and not active:
                first[label] = {"w": w.clone(), "P": P[:, pcols].clone()}
            if gemm_prec != "f64":
                ctx.assemble_gram(p, grid, xs, zs, rowptr, colidx, hvals, hb,
                                  add_lambda=(k == 0))
                rel, it, _ = ctx.refine(p, rowptr, colidx, hvals, hb, P, w, rtol=1e-10,
                                        max_iter=30)
                sweeps.append(it)
                if k == 0 and not active:
                    first[label]["w_refined"] = w.clone()
            return ctx.eval(p, grid, w, pts, pose=pose)

        for k in range(args.warmup):
            step(k)
        torch.cuda.synchronize()
        ctx.sync_status()
        ctx.profile(True)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        t0 = time.perf_counter()
        for k in range(args.steps):
            evs[k][0].record()
            step(args.warmup + k)
            evs[k][1].record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.set_update_joseph(False)
        ms = np.array([a.elapsed_time(b) for a, b in evs])
        step_ms[(label, streams, active)] = {
            "median": float(np.median(ms)), "p10": float(np.percentile(ms, 10)),
            "p90": float(np.percentile(ms, 90))}
        ctx.sync_status()
        prof = {name: ctx.profile_read(kind) for name, kind in
                (("syrk", L.PROF_SYRK), ("trsm", L.PROF_TRSM), ("chol", L.PROF_CHOL),
                 ("gather", L.PROF_GATHER), ("eval", L.PROF_EVAL))}
        ctx.profile(False)
        refine_log[label] = sweeps
        return t1 - t0, prof

    # mixed-precision covariance products first, FP64 last (its w is kept)
    mixed = {}
    last = frames[(args.warmup + args.steps - 1) % nfr]
    for mp in (() if args.no_mixed else ("bf16", "f32", "f32_joseph")):
        dtm, profm = run_sequence(mp.split("_")[0], joseph=mp.endswith("joseph"))
        log(f"{mp} covariance-product leg: {dtm / args.steps * 1e3:.1f} ms/step")
        fm = ctx.eval(p, grid, w, last[2], pose=last[3])["f"].clone()
        mixed[mp] = {"value": args.steps / dtm, "ms_per_step": dtm / args.steps * 1e3,
                     "step_ms": step_ms[(mp, args.streams, False)],
                     "syrk_ms_per_step": profm["syrk"][0] / args.steps,
                     "refine_sweeps_per_step": refine_log[mp][args.warmup:], "_f": fm}
    other = 3 - args.streams
    other_schedule = None
    if not args.no_other_schedule:
        dt_o, prof_o = run_sequence("f64", streams=other)
        log(f"f64 leg, {other} stream(s): {dt_o / args.steps * 1e3:.1f} ms/step")
        other_schedule = {"update_streams": other, "value": args.steps / dt_o,
                          "ms_per_step": dt_o / args.steps * 1e3,
                          "kernel_ms_per_step": {k: v[0] / args.steps
                                                 for k, v in prof_o.items()}}
    active_rows = None
    if not args.no_active:
        dt_a, prof_a = run_sequence("f64", active=True)
        log(f"active-rows leg: {dt_a / args.steps * 1e3:.1f} ms/step")
        fa = ctx.eval(p, grid, w, last[2], pose=last[3])["f"].clone()
        wa = w.clone()
        active_rows = {"value": args.steps / dt_a, "ms_per_step": dt_a / args.steps * 1e3,
                       "step_ms": step_ms[("f64", args.streams, True)],
                       "active_centers_per_step": n_act[args.warmup:],
                       "kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof_a.items()}}
    dt, prof = run_sequence("f64")
    log(f"f64 leg, {args.streams} stream(s): {dt / args.steps * 1e3:.1f} ms/step")
    f64 = ctx.eval(p, grid, w, last[2], pose=last[3])["f"]
    if active_rows is not None:
        dh = (fa - f64).abs()
        active_rows["speedup_vs_dense"] = active_rows["value"] / (args.steps / dt)
        active_rows["max_height_dev_vs_dense_m"] = float(dh.max())
        active_rows["mean_height_dev_vs_dense_m"] = float(dh.mean())
        active_rows["w_rel_dev_vs_dense"] = float((wa - w).norm() / w.norm())
    for mp in mixed:
        mixed[mp]["max_height_dev_vs_f64_m"] = float((mixed[mp].pop("_f") - f64).abs().max())
        mixed[mp]["speedup_vs_f64"] = mixed[mp]["value"] / (args.steps / dt)
    pts_per_frame = od.GROUND_PER_FRAME
    syrk_ms, syrk_n = prof["syrk"]
    # algorithmic work of P -= V V^T with symmetry: N(N+1)/2 entries, 2 flops
    # per absorbed point each
    syrk_flops = N * (N + 1) * pts_per_frame * args.steps
    syrk_tfs = syrk_flops / (syrk_ms * 1e-3) / 1e12 if syrk_ms > 0 else 0.0

    # ---- rbf_eval throughput: 500 launches of 200k points (1e8) per timed
    # region, each launch timed by its own event pair; then launches of 20M
    # points (the frame's scan points repeated), which fill the GPU
    ev = {}
    grid_b = ctx.grid(p, centers.contiguous())  # the same centers, binned form
    xy0, z0, pts0, pose0 = frames[0]
    big = pts0.repeat(args.eval_fill // pts0.shape[0], 1) if args.eval_fill else None

    def launches(fn, reps):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in range(reps)]
        ta = time.perf_counter()
        for a, b in pairs:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - ta) / reps
        us = np.array([a.elapsed_time(b) for a, b in pairs]) * 1e3
        return wall, {"median": float(np.median(us)), "p10": float(np.percentile(us, 10)),
                      "p90": float(np.percentile(us, 90))}

    for name, dt_ in (("f64", torch.float64), ("f32", torch.float32)):
        pts = pts0.to(dt_).contiguous()
        q = pts.shape[0]
        # the binding's own host time (argument checks, ctypes) bounds the
        # wall rate of a 200k-point call; the kernel rate is in mpts_s_kernel
        outs = {"f": torch.empty(q, dtype=dt_, device=dev),
                "grad": torch.empty((q, 2), dtype=dt_, device=dev),
                "resid": torch.empty(q, dtype=dt_, device=dev),
                "jac": torch.empty((q, 6), dtype=dt_, device=dev)}
        ctx.profile(True)
        wall, call_us = launches(lambda: ctx.eval(p, grid, w, pts, pose=pose0, out=outs),
                                 args.eval_reps)
        ems, en = ctx.profile_read(L.PROF_EVAL)
        ctx.profile(False)
        gn_wall, gn_us = launches(lambda: ctx.eval_gn(p, grid, w, pts, pose=pose0),
                                  args.eval_reps)
        ctx.profile(True)
        launches(lambda: ctx.eval(p, grid_b, w, pts, pose=pose0, out=outs), args.eval_reps)
        bms_, bn_ = ctx.profile_read(L.PROF_EVAL)
        ctx.profile(False)
        gnb_wall, gnb_us = launches(lambda: ctx.eval_gn(p, grid_b, w, pts, pose=pose0),
                                    args.eval_reps)
        esz = pts.element_size()
        bytes_pt = 3 * esz + 10 * esz  # read xyz, write f, grad(2), r, J(6)
        kern_s = ems * 1e-3 / en
        ev[name] = {
            "mpts_s_wall": q / wall / 1e6,
            "mpts_s_kernel": q / kern_s / 1e6,
            "kernel_us": kern_s * 1e6,
            "call_us": call_us,
            "points": q,
            "hbm_gbs": q * bytes_pt / kern_s / 1e9,
            "hbm_frac": q * bytes_pt / kern_s / 1e9 / PEAK_HBM_GBS,
            "gauss_newton_mpts_s_wall": q / gn_wall / 1e6,
            "gauss_newton_call_us": gn_us,
            "binned": {"kernel_us": bms_ * 1e3 / bn_,
                       "mpts_s_kernel": q / (bms_ * 1e-3 / bn_) / 1e6,
                       "gauss_newton_call_us": gnb_us},
        }
        if big is not None:
            bp = big.to(dt_).contiguous()
            ctx.profile(True)
            bwall, bus = launches(lambda: ctx.eval(p, grid, w, bp, pose=pose0), 5)
            bms, bn = ctx.profile_read(L.PROF_EVAL)
            ctx.profile(False)
            bk = bms * 1e-3 / bn
            ev[name]["fill"] = {"points": int(bp.shape[0]), "kernel_us": bk * 1e6,
                                "mpts_s_kernel": bp.shape[0] / bk / 1e6,
                                "mpts_s_wall": bp.shape[0] / bwall / 1e6,
                                "hbm_frac": bp.shape[0] * bytes_pt / bk / 1e9 / PEAK_HBM_GBS}
            del bp
    del big

    if not args.no_rows:
        out_rows = rows_leg(ctx, api, synth, L, od, torch.from_numpy(allxy).to(dev), centers,
                            grid, frames[0], w, p)
        log("rows leg done")
    else:
        out_rows = None
    out = {
        "metric": METRIC,
        "value": args.steps / dt,
        "unit": "scan updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "step_ms": step_ms[("f64", args.streams, False)],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": ("odometry frame: 50x50 m map, 10,000 centers (voxel selection "
                         "0.5 m), 20k ground points absorbed by the FP64 Kalman-form "
                         "update of w and dense P (10k x 10k), then f, grad f, residual "
                         "and 6-DoF Jacobian at 200k scan points (FP64)"),
            "centers": N,
            "update_points": pts_per_frame,
            "eval_points": int(pts0.shape[0]),
            "batch": args.batch,
            "sigma": p.sigma, "cutoff": p.cutoff, "lambda": p.lam, "R": p.R,
        },
        "roofline": {
            "kernel": "k_syrk_f64 + k_syrk_f64_tail (P -= V V^T, FP64 MFMA)",
            "bound": "mfma",
            "achieved": syrk_tfs,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": syrk_tfs / PEAK_FP64_TFLOPS,
            "traffic": (SYRK_F64_TRAFFIC.get((N, args.batch)) if args.streams == 1 else None),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE)",
            "launches": syrk_n,
            "avg_launch_ms": syrk_ms / max(syrk_n, 1),
            "flops_per_launch": syrk_flops / max(syrk_n, 1),
            "launches_note": ("one launch = one batch's product: k_syrk_f64 over the whole "
                              "rounds of 128x128 tiles, then k_syrk_f64_tail over the "
                              "leftover tiles as 32x64 sub-tiles, timed together by one "
                              "event pair; achieved = all product flops / all product time"),
        },
        "update_streams": args.streams,
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof.items()},
        "other_schedule": other_schedule,
        "mixed_precision": mixed,
        "active_rows": active_rows,
        "eval": ev,
        "rows": out_rows,
    }
    log("eval leg done")
    frame0_keep = frames[0]
    if args.patches > 0:
        del P, frames
        torch.cuda.empty_cache()
        log(f"batched leg: {args.patches} patches ...")
        out["batched"] = batched_leg(ctx, api, synth, args.patches, not args.no_tune)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cb = cpu_baseline(od, centers.cpu().numpy(), p, first, pcols.cpu().numpy(),
                          frame0_keep)
        out["err"] = cb.pop("err")
        out["cpu_baseline"] = cb
    else:
        out["err"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
