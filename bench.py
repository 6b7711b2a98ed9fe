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


def bench_global(steps):
    """Global BA after loop closure: 1000 keyframes x 96 patches, 1,505,568
    edges, 5 GN iterations (float32).  Returns throughput, per-phase average
    launch durations and the edge-assembly roofline."""
    import torch
    import paper_2408_01654_amd as dp
    from scenes import make_config
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
    ctx.solve(g, poses, depth, n_iters=s.n_iters, lam=s.lam, z_min=s.z_min, report=False)
    torch.cuda.synchronize()
    ctx.trace_begin(sample_every=1, max_pairs=1 << 16)
    t0 = time.perf_counter()
    for _ in range(steps):
        poses.copy_(poses0)
        depth.copy_(depth0)
        ctx.solve(g, poses, depth, n_iters=s.n_iters, lam=s.lam, z_min=s.z_min, report=False)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    ph = ctx.trace_end()
    rep = ctx.solve(g, poses.copy_(poses0), depth.copy_(depth0), n_iters=s.n_iters, lam=s.lam, z_min=s.z_min)
    ctx.close()
    avg = {k: (v[0] / v[1] * 1e3 if v[1] else 0.0) for k, v in ph.items()}
    E, P, N = s.n_edges, s.n_patches, s.n_frames
    # per launch of the assembly: edge records (grid cell 4 B + target 8 B + weight 8 B), patch centre and
    # inverse depth, poses, and the outputs: tile shares of S and s, stored Schur rows (4 B per element)
    alg = (info["grid_cells"] * 4 + E * 16 + P * 12 + N * 28
           + 4 * (info["part_S_elems"] + info["part_vec_elems"] + info["u_elems"]) + P * 8)
    ach = alg / (avg["assemble"] * 1e-6) / 1e9 if avg["assemble"] else 0.0
    out = {"workload": "global BA after loop closure: 1000 keyframes x 96 patches, 1,505,568 edges, "
                       "5 GN iterations, float32",
           "edges_per_s": E * s.n_iters * steps / sec, "gn_iters_per_s": s.n_iters * steps / sec,
           "ms_per_solve": 1e3 * sec / steps, "analysis_s": t_an, "phases_avg_us": avg,
           "phases_launches": {k: v[2] for k, v in ph.items()},
           "assembly_roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": ach / HBM_PEAK_GBS, "alg_bytes_per_launch": alg},
           "cost": rep["cost"], "status": rep["status"]}
    log(f"[bench] global BA: {out['ms_per_solve']:.2f} ms/solve, {out['edges_per_s']:.4g} edge-iters/s, "
        f"assembly {avg['assemble']:.1f} us ({ach:.0f} GB/s), analysis {t_an:.2f}s")
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
    args = ap.parse_args()
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
    ctx.analyze(g0)
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
    alg_bytes = {
        # per edge: grid cell (edge id, 4 B) + target (8 B) + weight (8 B); per patch: centre (8 B) +
        # inverse depth (4 B); per pose 28 B; outputs: the tiles' partial systems and vectors (4 B each)
        "assemble": info["grid_cells"] * 4 + E * 16 + Pn * 12 + N * 28
                    + 4 * (info["part_S_elems"] + info["part_vec_elems"]),
        "gather": 4 * (info["part_S_elems"] + info["part_vec_elems"]) + 4 * (n * (n + 1) // 2 + 3 * n),
        "factor": 4 * (n * (n + 1) // 2 + 3 * n),
        "backsub": info["grid_cells"] * 4 + E * 16 + Pn * 16 + N * 28 + 4 * n,
        "retract": N * 28 * 2 + 4 * n,
        "cost": E * (12 + 16) + Pn * 12 + N * 28,
    }
    achieved = alg_bytes[dom] / (avg[dom] * 1e-3) / 1e9 if avg[dom] > 0 else 0.0
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": dom,
                "avg_launch_us": avg[dom] * 1e3, "alg_bytes_per_launch": alg_bytes[dom]}

    global_ba = bench_global(args.global_steps) if args.global_steps > 0 else None

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
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    if not parity_ok:
        sys.exit(1)


if __name__ == "__main__":
    main()
