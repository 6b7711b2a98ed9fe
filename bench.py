#!/usr/bin/env python
"""Throughput of the patch-graph Gauss-Newton BA on one MI355X.

Workload (default): sliding-window local BA -- 22-frame window x 96
patches/frame, every patch linked to the frames within +-13 of its source
inside the window (37,440 edges per call), last 12 poses free, 2 Gauss-Newton
iterations per call, 1000 calls with the window advancing one frame.  One
"step" is the whole 1000-call sequence, every call starting from its own
seeded initial estimate; all inputs are resident in device memory before the
timed region.  value = edge-iterations per second (edges x GN iterations /
wall time).

Prints one JSON line.  The dominant kernel's average duration comes from
hipEvent pairs the library records on the launch stream during the timed
region (every `--trace-every`-th launch of each phase); the CPU baseline is
the float64 oracle on a bounded sample of the same windows.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BA edges/s & GN iters/s (fwd, fwd+adjoint) at oracle tolerance; % HBM peak"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE
# (each scaled by what the counter reads for a plain 256 MiB copy: x2.000 and
# x1.000) for the kernels as they are in this tree; the commands and counts
# are in profiles/tile_assembly_traffic.md.  Re-measure when either kernel
# changes.
TRAFFIC_WINDOW_LAUNCH = 4.887e6       # small_solve_kernel<float>, one 22-frame window solve
TRAFFIC_GLOBAL_ASSEMBLY = 131.65e6    # tile_iterate_kernel<float>, global BA, per launch


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_windows(n_calls):
    from scenes import make_window
    t0 = time.time()
    ws = [make_window(c, n_calls=n_calls) for c in range(n_calls)]
    log(f"[bench] generated {n_calls} windows in {time.time() - t0:.1f}s "
        f"(E={ws[0].n_edges}, P={ws[0].n_patches}, N={ws[0].n_frames})")
    for w in ws[1:]:
        assert np.array_equal(w.ii, ws[0].ii) and np.array_equal(w.jj, ws[0].jj) and np.array_equal(w.kk, ws[0].kk)
    return ws


def cpu_baseline(windows, budget_s=12.0, max_windows=80):
    """The float64 oracle, as it stands, on the first windows of the sequence."""
    from threadpoolctl import threadpool_limits
    from oracle import ba64
    done = 0
    edges_iters = 0
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        for w in windows[:max_windows]:
            ba64.solve_scene(w)
            done += 1
            edges_iters += w.n_edges * w.n_iters
            if time.perf_counter() - t0 > budget_s:
                break
    dt = time.perf_counter() - t0
    return {"value": edges_iters / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} windows of the sliding-window sequence (calls 0..{done - 1}), "
                      f"{windows[0].n_iters} GN iterations each, float64 numpy/scipy, 1 BLAS thread",
            "seconds": dt}


def tile_launch_bytes(info, E, P, N, first, tsize=4):
    """Algorithmic HBM bytes of one tile-assembly launch over the whole edge set:
    reads -- per cell of the (patch, slot) grid its edge id (4 B), per edge target
    and weight (16 B), per patch its centre and inverse depth (first iteration:
    8 + 4 B) or its stored ray, depth and 1/sqrt(C~), w/sqrt(C~) (later: 8 + 4 + 8 B)
    plus its stored Schur row (later), per pose 28 B, the previous pose step;
    writes -- the tiles' shares of S and of (s, Diag(B)), the Schur rows, and per
    patch the stored ray (first), depth and the two scales."""
    n = 6 * info["n_free"]
    reads = info["grid_cells"] * 4 + E * 16 + N * 28
    writes = tsize * (info["part_S_elems"] + info["part_vec_elems"] + info["u_elems"]) + P * (4 + 2 * tsize)
    if first:
        reads += P * 12
        writes += P * 2 * tsize
    else:
        reads += P * (2 * tsize + 4 + 2 * tsize) + tsize * info["u_elems"] + tsize * n
    return reads + writes


def bench_global(steps, precision=None):
    """Global BA after loop closure: 1000 keyframes x 96 patches, 1,505,568
    edges, 5 GN iterations (float32 or mixed).  Returns throughput, per-phase
    average launch durations, the edge-assembly roofline and the error
    against the stored float64 oracle result."""
    import torch
    import paper_2408_01654_amd as dp
    from scenes import make_config
    precision = dp.FP32 if precision is None else precision
    s = make_config(2)
    g = dp.GraphTensors.from_scene(s)
    ctx = dp.Context(0)
    t0 = time.perf_counter()
    ctx.analyze(g)
    t_an = time.perf_counter() - t0
    info = ctx.analysis_info()
    poses0 = torch.as_tensor(s.poses).cuda().contiguous()
    depth0 = torch.as_tensor(s.inv_depth).cuda().contiguous()
    poses, depth = poses0.clone(), depth0.clone()
    kw = dict(n_iters=s.n_iters, lam=s.lam, z_min=s.z_min, precision=precision)
    ctx.solve(g, poses, depth, report=False, **kw)
    torch.cuda.synchronize()
    ctx.trace_begin(sample_every=1, max_pairs=1 << 16)
    t0 = time.perf_counter()
    for _ in range(steps):
        poses.copy_(poses0)
        depth.copy_(depth0)
        ctx.solve(g, poses, depth, report=False, **kw)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    ph = ctx.trace_end()
    rep = ctx.solve(g, poses.copy_(poses0), depth.copy_(depth0), **kw)
    gold = np.load(os.path.join(ROOT, "tests", "golden", "global_ba_oracle.npz"))
    from oracle import ba64
    dtr, drr = ba64.pose_errors(poses.double().cpu().numpy(), gold["poses"])
    drel = np.abs(depth.double().cpu().numpy() - gold["inv_depth"]) / np.abs(gold["inv_depth"])
    err = max(float(dtr.max()), float(drr.max()), float(drel.max()))
    ctx.close()
    avg = {k: (v[0] / v[1] * 1e3 if v[1] else 0.0) for k, v in ph.items()}
    E, P, N = s.n_edges, s.n_patches, s.n_frames
    # per launch of the assembly: edge records (grid cell 4 B + target 8 B + weight 8 B), patch centre and
    # inverse depth, poses, and the outputs: tile shares of S and s, stored Schur rows (4 B per element)
    # average over the iterations of one solve (the first launch reads the caller's arrays)
    alg = (tile_launch_bytes(info, E, P, N, True)
           + (s.n_iters - 1) * tile_launch_bytes(info, E, P, N, False)) / s.n_iters
    ach = alg / (avg["assemble"] * 1e-6) / 1e9 if avg["assemble"] else 0.0
    name = "mixed (float64-refined camera solve)" if precision == dp.MIXED else "float32"
    out = {"workload": "global BA after loop closure: 1000 keyframes x 96 patches, 1,505,568 edges, "
                       f"5 GN iterations, {name}",
           "max_err_vs_oracle": err, "refine_resid": rep["refine_resid"], "fp64_fallback": rep["fp64_fallback"],
           "min_pivot": rep["min_pivot"],
           "edges_per_s": E * s.n_iters * steps / sec, "gn_iters_per_s": s.n_iters * steps / sec,
           "ms_per_solve": 1e3 * sec / steps, "analysis_s": t_an, "phases_avg_us": avg,
           "phases_launches": {k: v[2] for k, v in ph.items()},
           "assembly_roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": ach / HBM_PEAK_GBS, "alg_bytes_per_launch": alg,
                                 "kernel": "tile_iterate_kernel", "avg_launch_us": avg["assemble"],
                                 "traffic": TRAFFIC_GLOBAL_ASSEMBLY if precision == dp.FP32 else None},
           "cost": rep["cost"], "status": rep["status"]}
    log(f"[bench] global BA {name}: {out['ms_per_solve']:.2f} ms/solve, {out['edges_per_s']:.4g} edge-iters/s, "
        f"assembly {avg['assemble']:.1f} us ({ach:.0f} GB/s), analysis {t_an:.2f}s, err {err:.2e}")
    return out


def _parity(P_list, D_list, scenes):
    """Worst pose / depth error of GPU results against the oracle."""
    from oracle import ba64
    worst = 0.0
    for P, D, s in zip(P_list, D_list, scenes):
        Po, Do, _ = ba64.solve_scene(s)
        dt, dr = ba64.pose_errors(P, Po)
        rel = np.abs(D - Do) / np.abs(Do)
        worst = max(worst, float(dt.max()), float(dr.max()), float(rel.max()))
    return worst


def bench_window_mixed(windows, calls, steps):
    """The sliding-window sequence in DPVBA_MIXED (float64-refined camera
    solve; one stream synchronisation per GN iteration for the fallback
    decision), on the first `calls` windows."""
    import torch
    import paper_2408_01654_amd as dp
    ws = windows[:calls]
    w0 = ws[0]
    ctx = dp.Context(0)
    gs = [dp.GraphTensors.from_scene(w) for w in ws]
    # one analysis serves every call (same index arrays)
    for g in gs[1:]:
        g.ii, g.jj, g.kk = gs[0].ii, gs[0].jj, gs[0].kk
    ctx.analyze(gs[0])
    p0 = [torch.as_tensor(w.poses).cuda() for w in ws]
    d0 = [torch.as_tensor(w.inv_depth).cuda() for w in ws]
    ps = [p.clone() for p in p0]
    ds = [d.clone() for d in d0]

    def step():
        for c in range(calls):
            ps[c].copy_(p0[c])
            ds[c].copy_(d0[c])
            ctx.solve(gs[c], ps[c], ds[c], n_iters=w0.n_iters, lam=w0.lam, z_min=w0.z_min, precision=dp.MIXED,
                      report=False)
    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    rep = ctx.solve(gs[0], ps[0].copy_(p0[0]), ds[0].copy_(d0[0]), n_iters=w0.n_iters, lam=w0.lam, z_min=w0.z_min,
                    precision=dp.MIXED)
    idx = [0, calls - 1]
    err = _parity([ps[c].double().cpu().numpy() for c in idx], [ds[c].double().cpu().numpy() for c in idx],
                  [ws[c] for c in idx])
    ctx.close()
    out = {"workload": f"sliding-window local BA, first {calls} calls, DPVBA_MIXED",
           "edges_per_s": w0.n_edges * w0.n_iters * calls * steps / sec,
           "gn_iters_per_s": w0.n_iters * calls * steps / sec, "us_per_call": 1e6 * sec / (calls * steps),
           "max_err_vs_oracle": err, "refine_resid": rep["refine_resid"], "fp64_fallback": rep["fp64_fallback"]}
    log(f"[bench] window mixed: {out['us_per_call']:.1f} us/call, err {err:.2e}")
    return out


def bench_batch(precision, graph, steps, tuner_cache=None):
    """256 uneven windows (8-40 frames x 48-128 patches, radius 4-13, 2 GN
    iterations) solved as one batch; tile shapes from the autotuner."""
    import torch
    import paper_2408_01654_amd as dp
    from paper_2408_01654_amd.autotune import TileTuner
    from scenes import make_config
    scenes = [make_config(4, i) for i in range(256)]
    t0 = time.perf_counter()
    tuner = TileTuner(tuner_cache)
    tp = tuner.tile_patches(scenes, dp.FP32 if precision != dp.FP64 else dp.FP64)
    t_tune = time.perf_counter() - t0
    b = dp.BatchTensors.from_scenes(scenes)
    ctx = dp.Context(0)
    ctx.analyze_batch(b, tp)
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    E = int(b.edge_off[-1])
    nit = scenes[0].n_iters
    with torch.cuda.stream(st):
        p0, d0 = b.poses.clone(), b.inv_depth.clone()
        poses, depth = p0.clone(), d0.clone()

        def step():
            poses.copy_(p0)
            depth.copy_(d0)
            ctx.solve_batch(b, poses, depth, n_iters=nit, lam=scenes[0].lam, z_min=scenes[0].z_min,
                            precision=precision, report=False, graph=graph, stream=st)
        step()
        st.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(st)
        for _ in range(steps):
            step()
        ev1.record(st)
        ev1.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        reps = ctx.solve_batch(b, poses.copy_(p0), depth.copy_(d0), n_iters=nit, lam=scenes[0].lam,
                               z_min=scenes[0].z_min, precision=precision, report=True, graph=False, stream=st)
    P = poses.double().cpu().numpy()
    D = depth.double().cpu().numpy()
    check = [0, 1, int(np.argmax([s.n_frames for s in scenes]))]
    err = _parity([P[b.frame_off[q]:b.frame_off[q + 1]] for q in check],
                  [D[b.patch_off[q]:b.patch_off[q + 1]] for q in check], [scenes[q] for q in check])
    ctx.close()
    name = {dp.FP32: "float32", dp.MIXED: "mixed", dp.FP64: "float64"}[precision]
    out = {"workload": f"256 uneven windows in one batch, {name}, graph={graph}", "edges_total": E,
           "ms_per_batch": ms, "edges_per_s": E * nit / (ms * 1e-3), "gn_iters_per_s": 256 * nit / (ms * 1e-3),
           "max_err_vs_oracle_sampled": err, "checked_problems": check, "tune_s": t_tune,
           "status_ok": all(r["status"] == 0 for r in reps),
           "fp64_fallbacks": int(sum(sum(r["fp64_fallback"]) for r in reps))}
    log(f"[bench] batch {name}: {ms:.3f} ms/batch, {out['edges_per_s']:.4g} edge-iters/s, err {err:.2e}")
    return out


def bench_adjoint(steps):
    """Forward + adjoint of 16 windows (12-22 frames x 64-96 patches, 2 GN
    iterations), loss on the poses and depths: GN iterations per second of
    the forward and of forward + backward, and the gradient error of one
    window against the float64 gradient oracle."""
    import torch
    import paper_2408_01654_amd as dp
    from oracle import grad64
    from scenes import make_config
    scenes = [make_config(3, i) for i in range(16)]
    ctx = [dp.Context(0) for _ in scenes]
    gs = [dp.GraphTensors.from_scene(s) for s in scenes]
    for c, g in zip(ctx, gs):
        c.analyze(g)
    refs = [(torch.as_tensor(s.poses_gt, dtype=torch.float32).cuda(),
             torch.as_tensor(s.inv_depth_gt, dtype=torch.float32).cuda()) for s in scenes]
    p0 = [torch.as_tensor(s.poses).cuda() for s in scenes]
    d0 = [torch.as_tensor(s.inv_depth).cuda() for s in scenes]
    tg = [g.target.clone().requires_grad_(True) for g in gs]
    wg = [g.weight.clone().requires_grad_(True) for g in gs]

    def fwd(backward):
        for q, s in enumerate(scenes):
            poses, d = dp.bundle_adjust(ctx[q], gs[q], p0[q], d0[q], tg[q], wg[q], n_iters=s.n_iters, lam=s.lam,
                                        z_min=s.z_min)
            if backward:
                grad64.pose_depth_loss(poses, d, refs[q][0], refs[q][1], s.n_fixed).backward()
    out = {}
    for name, bw in (("forward", False), ("forward_adjoint", True)):
        fwd(bw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fwd(bw)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out[name] = {"gn_iters_per_s": sum(s.n_iters for s in scenes) * steps / sec,
                     "edges_per_s": sum(s.n_edges * s.n_iters for s in scenes) * steps / sec,
                     "ms_per_batch": 1e3 * sec / steps}
    for x in tg + wg:
        x.grad = None
    fwd(True)
    L, gt_o, gw_o, _, _ = grad64.loss_and_grads(scenes[0])
    rel = lambda a, b: float(np.abs(a - b).max() / np.abs(b).max())
    out["grad_rel_err_window0"] = {"target": rel(tg[0].grad.double().cpu().numpy(), gt_o),
                                   "weight": rel(wg[0].grad.double().cpu().numpy(), gw_o)}
    out["workload"] = "16 windows (12-22 frames x 64-96 patches), 2 unrolled GN iterations, float32"
    for c in ctx:
        c.close()
    log(f"[bench] adjoint: fwd {out['forward']['ms_per_batch']:.2f} ms, fwd+adj "
        f"{out['forward_adjoint']['ms_per_batch']:.2f} ms per 16 windows, grad err {out['grad_rel_err_window0']}")
    return out



def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--calls", type=int, default=1000)
    ap.add_argument("--trace-every", type=int, default=7)
    ap.add_argument("--check", type=int, default=4, help="windows checked against the oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--global-steps", type=int, default=3,
                    help="timed solves of the 1000-keyframe global BA reported beside the main line (0: skip)")
    ap.add_argument("--variants", default="mixed,batch,adjoint",
                    help="comma list of side workloads reported beside the main line: mixed (window and global "
                         "BA in DPVBA_MIXED), batch (256 uneven windows), adjoint (16 windows forward+adjoint); "
                         "empty: none")
    ap.add_argument("--tile-patches", type=int, default=0,
                    help="patches per tile of the float32 plan of the window workload (0: library default)")
    ap.add_argument("--global-only", action="store_true",
                    help="only time the 1000-keyframe global BA (--global-steps solves) and print its record")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="only run 5 plain device copies of this many MiB and exit (calibrates HBM byte "
                         "counters of a profiler against a kernel of known traffic)")
    args = ap.parse_args()
    if args.copy_probe_mb > 0:
        import torch
        n = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "launches": 5}))
        return
    if args.global_only:
        import paper_2408_01654_amd as dp
        print(json.dumps({"global_ba": bench_global(max(1, args.global_steps))}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the BA path here is "
              f"single-GPU and has no multi-GPU mode", file=sys.stderr)
        sys.exit(2)

    import ctypes
    import torch
    import paper_2408_01654_amd as dp
    from paper_2408_01654_amd import binding

    windows = build_windows(args.calls)
    w0 = windows[0]
    dev = torch.device("cuda:0")
    st = lambda a, dt=torch.float32: torch.as_tensor(np.stack(a), dtype=dt).to(dev).contiguous()
    patches = st([w.patches for w in windows])
    target = st([w.target for w in windows])
    weight = st([w.weight for w in windows])
    poses0 = st([w.poses for w in windows])
    depth0 = st([w.inv_depth for w in windows])
    poses = poses0.clone()
    depth = depth0.clone()
    ii = torch.as_tensor(w0.ii).to(dev).contiguous()
    jj = torch.as_tensor(w0.jj).to(dev).contiguous()
    kk = torch.as_tensor(w0.kk).to(dev).contiguous()

    ctx = dp.Context(0)
    g0 = dp.GraphTensors(w0.n_frames, w0.n_fixed, patches[0], ii, jj, kk, target[0], weight[0],
                         tuple(float(x) for x in w0.intrinsics))
    ctx.analyze(g0, tile_patches_fp32=args.tile_patches)
    info = ctx.analysis_info()
    L = binding.lib()
    graphs = []
    for c in range(args.calls):
        g = dp.GraphTensors(w0.n_frames, w0.n_fixed, patches[c], ii, jj, kk, target[c], weight[c], g0.intrinsics)
        graphs.append(g.struct())
    opts = binding.Opts(w0.n_iters, binding.FP32, float(w0.lam), float(w0.z_min), 0)
    stream = torch.cuda.current_stream(dev)
    sptr = ctypes.c_void_p(stream.cuda_stream)
    hctx = ctx._h
    pose_ptr = [ctypes.c_void_p(poses[c].data_ptr()) for c in range(args.calls)]
    depth_ptr = [ctypes.c_void_p(depth[c].data_ptr()) for c in range(args.calls)]
    solve = L.dpvba_solve
    gref = [ctypes.byref(g) for g in graphs]
    oref = ctypes.byref(opts)

    def step():
        poses.copy_(poses0)
        depth.copy_(depth0)
        for c in range(args.calls):
            rc = solve(hctx, gref[c], pose_ptr[c], depth_ptr[c], oref, None, sptr)
            if rc:
                raise dp.DpvbaError(rc, "dpvba_solve")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} steps)")

    ctx.trace_begin(sample_every=args.trace_every, max_pairs=1 << 18)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases = ctx.trace_end()
    sec = t1 - t0
    ms_per_step = 1e3 * sec / args.steps
    edges_iters = w0.n_edges * w0.n_iters * args.calls * args.steps
    value = edges_iters / sec
    gn_iters = w0.n_iters * args.calls * args.steps / sec
    log(f"[bench] timed {args.steps} steps: {ms_per_step:.2f} ms/step, {value:.4g} edge-iters/s, "
        f"{1e6 * sec / (args.steps * args.calls):.1f} us/call")

    # parity of the timed outputs with the oracle on a sample of windows
    from oracle import ba64
    P = poses.double().cpu().numpy()
    D = depth.double().cpu().numpy()
    idx = sorted(set(int(x) for x in np.linspace(0, args.calls - 1, max(1, args.check))))
    worst = {"dt": 0.0, "dr": 0.0, "depth_rel": 0.0}
    for c in idx:
        Po, Do, _ = ba64.solve_scene(windows[c])
        dtr, drr = ba64.pose_errors(P[c], Po)
        rel = np.abs(D[c] - Do) / np.abs(Do)
        worst = {"dt": max(worst["dt"], float(dtr.max())), "dr": max(worst["dr"], float(drr.max())),
                 "depth_rel": max(worst["depth_rel"], float(rel.max()))}
    parity_ok = max(worst.values()) < 1e-4
    log(f"[bench] parity vs oracle on calls {idx}: {worst} ok={parity_ok}")

    # roofline of the dominant kernel (largest summed sampled time)
    E, Pn, N = w0.n_edges, w0.n_patches, w0.n_frames
    avg = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in phases.items()}
    share = {k: avg[k] * v[2] for k, v in phases.items()}
    dom = max(share, key=share.get)
    n = 6 * info["n_free"]
    # One timed launch is one whole window solve (a single kernel for systems of
    # this size): two tile passes, two gathers of the tile shares into
    # the packed reduced system (written, then read by the factorisation), the
    # pose updates and the final depth write-back.
    n = 6 * info["n_free"]
    shares = 4 * (info["part_S_elems"] + info["part_vec_elems"])
    packed = 4 * (n * (n + 1) // 2 + 3 * n)
    it = w0.n_iters
    fused = (tile_launch_bytes(info, E, Pn, N, True) + (it - 1) * tile_launch_bytes(info, E, Pn, N, False)
             + it * (shares + 2 * packed + N * 28 * 2 + 4 * n)
             + 4 * info["u_elems"] + Pn * 12 + 4 * n + Pn * 4 + N * 28)
    achieved = fused / (avg[dom] * 1e-3) / 1e9 if avg[dom] > 0 else 0.0
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": TRAFFIC_WINDOW_LAUNCH,
                "kernel": "small_solve_kernel<float> (one fused window solve per launch)", "phase": dom,
                "avg_launch_us": avg[dom] * 1e3, "alg_bytes_per_launch": fused}

    global_ba = bench_global(args.global_steps) if args.global_steps > 0 else None
    wanted = [v for v in args.variants.split(",") if v]
    variants = {}
    if "mixed" in wanted:
        variants["window_mixed"] = bench_window_mixed(windows, calls=100, steps=1)
        if args.global_steps > 0:
            variants["global_mixed"] = bench_global(args.global_steps, dp.MIXED)
    if "batch" in wanted:
        variants["batch_fp32"] = bench_batch(dp.FP32, graph=True, steps=5)
        variants["batch_mixed"] = bench_batch(dp.MIXED, graph=True, steps=5)
    if "adjoint" in wanted:
        variants["adjoint"] = bench_adjoint(steps=3)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(windows)
        log(f"[bench] cpu baseline (oracle) {cpu['value']:.4g} edges/s over {cpu['seconds']:.1f}s")

    out = {
        "metric": METRIC, "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "sliding-window local BA: 22-frame window x 96 patches, edges within +-13 "
                               "frames (37,440 per call), last 12 poses free, 2 GN iterations per call, "
                               f"{args.calls} calls advancing one frame",
                   "global_batch": args.calls, "edges_per_call": E, "gn_iters_per_call": w0.n_iters,
                   "parallelism": "single GPU"},
        "gn_iters_per_s": gn_iters, "us_per_call": 1e6 * sec / (args.steps * args.calls),
        "parity": {"checked_calls": idx, "max_pose_t": worst["dt"], "max_pose_r": worst["dr"],
                   "max_depth_rel": worst["depth_rel"], "tol": 1e-4, "ok": parity_ok},
        "phases_avg_us": {k: avg[k] * 1e3 for k in avg},
        "phases_launches": {k: v[2] for k, v in phases.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "global_ba": global_ba,
        "variants": variants,
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    if not parity_ok:
        sys.exit(1)


if __name__ == "__main__":
    main()
