#!/usr/bin/env python3
"""Throughput of the ray-MRF belief-propagation hot path on one MI355X.

One step is the whole path over one synthetic batch already resident in HBM:
graph build (ray clipping, 3D-DDA traversal, CSR incidence by radix sort),
potentials, K batched BP sweeps (hipGraph), marginals, and (for the
differentiable workload) the reverse pass through the K sweeps to the
per-voxel prior log-odds and the 64-bin sigma table.

value = E * K / step time: ray-voxel message updates per second, one update
being one edge's voxel->ray and ray->voxel messages in one sweep.

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ray-voxel msg updates/s per BP sweep (% HBM peak); batched fwd+bwd vs plain BP"
UNIT = "ray-voxel msg updates/s"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c4": ("30 keyframes of 640x480 along a loop in a 5x5x3 m room with 20 boxes, 250x250x150 grid "
           "at 0.02 m, 64-bin sigma table, 8 sweeps forward + reverse pass (BCE vs ground truth)",
           8, True),
    "c3": ("30 keyframes of 640x480 along a loop in a 5x5x3 m room, 250x250x150 grid at 0.02 m, "
           "10 sweeps forward", 10, False),
    "c2": ("one 640x480 frame in a 5x5x3 m room, 100x100x60 grid at 0.05 m, 10 sweeps forward",
           10, False),
    "c1": ("one 64x48 frame, 64^3 grid at 0.05 m, 5 sweeps forward", 5, False),
    "c5": ("8 independent rooms (grids 64^3 .. 400x400x150 at 0.05 .. 0.0125 m, 120, 20 and 6 x 10 frames) "
           "batched in one launch sequence, 10 sweeps forward + reverse pass; the count pass trims frames of "
           "the rooms with the most edges until the step fits --mem-frac of the GPU's memory", 10, True),
}


# HBM traffic per launch (read, written bytes) of the kernels that can be the
# dominant one on c4 (the top kernels by time per step, and every launch shape
# the autotuner may pick for their ray classes), from two rocprofv3 --pmc runs
# of this script (FETCH_SIZE, then WRITE_SIZE; each run also times one plain
# copy through --calib-copy-mib, which calibrates the counter: FETCH_SIZE read
# 0.5 x the bytes the copy reads, WRITE_SIZE 1.0 x the bytes it writes).  Valid
# only while the kernel sources hash to `src_sha256`; otherwise traffic is
# reported as null.
TRAFFIC = {"workload": "c4",
           "sources": ['adjoint_kernels.hip', 'sweep_kernels.hip', 'dev_common.hpp', 'tile_lds.hpp',
                       'mrf_internal.hpp'],
           "src_sha256": "db49eb0cdb9d65dec414cea544507680eaa67cd133d7450c7efb25f990c72a25",
           "kernels": {
                       "ray_adj_lds_k<32,10,1>": [1.2761e+10, 4.666e+09],
                       "ray_adj_lds_k<32,10,2>": [1.2234e+10, 4.666e+09],
                       "ray_adj_lds_k<32,8,1>": [7.1532e+09, 2.7667e+09],
                       "ray_adj_lds_k<32,8,2>": [7.3984e+09, 2.7676e+09],
                       "ray_adj_lds_k<64,4,1>": [7.3932e+09, 2.7666e+09],
                       "ray_adj_lds_k<64,4,2>": [7.4075e+09, 2.7666e+09],
                       "ray_adj_lds_k<64,5,1>": [1.2765e+10, 4.666e+09],
                       "ray_adj_lds_k<64,5,2>": [1.2776e+10, 4.6661e+09],
                       "voxel_k<4,16,1>": [8.8416e+09, 8.0598e+06]}}


def src_sha256(files):
    import hashlib
    d = os.path.join(ROOT, "paper_2006_03512_amd", "csrc")
    h = hashlib.sha256()
    for f in files:
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def trim_to_memory(m, scs, K, backward, mem_frac, keyframe_average=False):
    """The count pass decides: with B bytes per edge slot (the ten per-edge arrays of
    the build and sweeps, 37 bytes, the radix sort's tile histograms and offsets,
    under one byte, plus K - 1 checkpointed ray messages of 4 bytes for the reverse
    pass) and the per-voxel and per-ray arrays, drop the last frame of the room
    holding the most slots until the whole step fits mem_frac of the GPU's memory.
    With per-keyframe averaged messages the checkpoints are per (keyframe, voxel)
    pair instead (counted as 2 bytes per slot) and three per-edge arrays are
    added (chord length, weight share in list and in slot order, 12 bytes), and
    the batch must stay under 2^32 slots (one group).
    Returns the trimmed scenes and a record of what was done."""
    import dataclasses

    import numpy as np
    import torch
    slots, edges = m.count(scs)
    if keyframe_average:
        per_slot = 38 + 12 + (2 if backward else 0)
    else:
        per_slot = 38 + (4 * (K - 1) if backward else 0)
    max_slots = (1 << 32) - 1 if keyframe_average else None
    V = sum(x.grid.n_voxels for x in scs)
    per_voxel = 4 * 3 + 8 + 24 + 8 + (8 * (K - 1) if backward else 8)
    total_mem = torch.cuda.get_device_properties(0).total_memory
    budget = mem_frac * total_mem
    off = np.cumsum([0] + [x.n_frames for x in scs])
    F = [x.n_frames for x in scs]

    def need():
        S = sum(int(slots[off[i]: off[i] + F[i]].sum()) for i in range(len(scs)))
        R = sum(F[i] * x.depth[0].size for i, x in enumerate(scs))
        return per_slot * S + per_voxel * V + 12 * R, S
    while need()[0] > budget or (max_slots is not None and need()[1] > max_slots):
        big = max(range(len(scs)), key=lambda i: (int(slots[off[i]: off[i] + F[i]].sum()) if F[i] > 1 else -1))
        if F[big] <= 1:
            break
        F[big] -= 1
    out = []
    for x, f in zip(scs, F):
        if f < x.n_frames:
            ex = dict(x.extra)
            if "clean_depth" in ex:
                ex["clean_depth"] = ex["clean_depth"][:f].copy()
            x = dataclasses.replace(x, depth=x.depth[:f].copy(), T_wc=x.T_wc[:f].copy(), extra=ex)
        out.append(x)
    nb, S = need()
    rec = {"stated_frames": [int(x.n_frames) for x in scs], "frames": [int(f) for f in F],
           "stated_slots": int(slots.sum()), "stated_edges": int(edges.sum()),
           "slots": int(S), "edges": int(sum(int(edges[off[i]: off[i] + F[i]].sum()) for i in range(len(scs)))),
           "bytes_per_slot": per_slot, "memory_budget_gb": round(budget / 1e9, 1),
           "estimated_gb": round(nb / 1e9, 1), "stated_estimated_gb": round(
               (per_slot * int(slots.sum()) + per_voxel * V + 12 * sum(x.depth.size for x in scs)) / 1e9, 1)}
    return out, rec


def make_scene(name, frames=None, c5_scale=1.0):
    """List of scenes of the workload (one scene except c5)."""
    from paper_2006_03512_amd import scenes
    if name in ("c3", "c4"):
        return [getattr(scenes, f"make_{name}")(n_frames=frames or 30)]
    if name == "c5":
        return scenes.make_c5(frame_scale=c5_scale)
    return [scenes.make(name)]


def cpu_baseline(name, sc, sweeps, backward, row_frac, nf=1, single_rows=10, runs=5):
    """The FP64 oracle on a bounded sample of the same workload: the first nf
    frames of the batch, restricted to a band of their pixel rows (the other
    pixels carry no measurement), on every thread; then on one thread over a
    band of single_rows rows of frame 0.  Each figure is the median of `runs`
    timed runs after one untimed run."""
    import numpy as np

    from oracle import oracle
    from paper_2006_03512_amd import scenes as S

    def band(frames, rows):
        depth = sc.depth[:frames].copy()
        H = depth.shape[1]
        keep = max(1, min(H, rows))
        r0 = (H - keep) // 2
        depth[:, :r0] = 0.0
        depth[:, r0 + keep:] = 0.0
        sub = S.Scene(sc.name, depth, sc.T_wc[:frames].copy(), sc.intr, sc.grid, sc.solids,
                      sc.params, sc.sigma_table, sc.prior, sc.sweeps)
        return sub, f"rows {r0}..{r0 + keep - 1} of frames 0..{frames - 1}"

    def run(sub):
        y = sub.occupancy().astype(np.float64) if backward else None   # labels: not timed
        t0 = time.perf_counter()
        G = oracle.build_graph(sub)
        th = sub.prior_logit().astype(np.float64)
        res = oracle.infer(G, th, sub.sigma_table, sweeps, keep_history=backward)
        if backward:
            oracle.backward(G, res, oracle.bce_logit_grad(res.L, y), sub.sigma_table)
        return G.n_edges, time.perf_counter() - t0

    def median_run(sub):
        run(sub)   # untimed: pages in the oracle library and the sample's memory
        ts = []
        for _ in range(runs):
            E, dt = run(sub)
            ts.append(dt)
        return E, sorted(ts)[len(ts) // 2], ts

    what = "build + %d sweeps%s" % (sweeps, " + reverse pass" if backward else "")
    nf = max(1, min(nf, sc.n_frames))
    sub, where = band(nf, int(round(sc.depth.shape[1] * row_frac)))
    E, dt, ts = median_run(sub)
    threads = oracle.num_threads()
    sub1, where1 = band(1, single_rows)
    oracle.set_threads(1)
    try:
        E1, dt1, ts1 = median_run(sub1)
    finally:
        oracle.set_threads(threads)
    spread = lambda t: ", ".join(f"{x:.2f}" for x in t)
    return {"value": E * sweeps / dt, "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": f"{where} of the {sc.n_frames}-frame {name} batch ({E} edges), {what}, FP64, "
                      f"median of {runs} runs: {dt:.2f} s ({spread(ts)} s)",
            "single_thread": {"value": E1 * sweeps / dt1, "unit": UNIT, "cores": 1,
                              "sample": f"{where1} ({E1} edges), {what}, FP64, median of {runs} runs: "
                                        f"{dt1:.2f} s ({spread(ts1)} s)"}}


def copy_bandwidth(nbytes: int, reps: int = 5) -> float:
    """GB/s (bytes read + written) of torch's device-to-device copy, best of reps."""
    import torch
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    del src, dst
    return 2.0 * n * 4 / (best / 1e3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--frames", type=int, default=None, help="override the batch size (c3/c4)")
    ap.add_argument("--profile-reps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=float, default=0.4, help="fraction of the sampled frames' rows the oracle runs on")
    ap.add_argument("--cpu-frames", type=int, default=1, help="frames of the batch the oracle runs on")
    ap.add_argument("--c5-scale", type=float, default=1.0,
                    help="frame-count scale of the c5 rooms before the count pass trims them")
    ap.add_argument("--mem-frac", type=float, default=0.8,
                    help="c5: fraction of the GPU's memory the step may use (the count pass trims frames to fit)")
    ap.add_argument("--sparse-bricks", type=int, default=-1,
                    help="brick radius of a sparse grid (bricks around the measured points); -1: dense")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in launch shapes instead of timing the candidates after warmup")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="time one plain device copy of this many MiB first (HBM counter calibration)")
    ap.add_argument("--quick", action="store_true",
                    help="skip the sections outside the step and its roofline (bias table, accuracy by sweep "
                         "count, keyframe averaging, depth messages): for counter runs")
    ap.add_argument("--forward-only", action="store_true",
                    help="time build + K sweeps + marginals without checkpoints or the reverse pass")
    ap.add_argument("--keyframe-average", action="store_true",
                    help="time per-keyframe averaged messages (Sec. IV-A) as the step: build + K sweeps + "
                         "marginals, no reverse pass")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the ray-MRF path runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2006_03512_amd.mrf import RayMRF

    torch.cuda.set_device(0)
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {n * 4} bytes read, {n * 4} bytes written")
        del src, dst
    desc, K, backward = WORKLOADS[args.workload]
    kf_step = args.keyframe_average
    if args.forward_only and backward:
        backward = False
        desc = desc.replace(" + reverse pass (BCE vs ground truth)", "").replace(" + reverse pass", "")
        desc += "; forward sweeps only (no checkpoints, no reverse pass)"
    if kf_step:
        desc += "; per-keyframe averaged messages (one chord-length-weighted average per keyframe and voxel)"
    t = time.perf_counter()
    scs = make_scene(args.workload, args.frames, args.c5_scale)
    sc = scs[0]
    if args.sparse_bricks >= 0:   # sparse grid: bricks around the measured points only
        import dataclasses
        sc.params = dataclasses.replace(sc.params, sparse_bricks=1, brick_radius=args.sparse_bricks)
    for other in scs[1:]:
        other.params, other.sigma_table = sc.params, sc.sigma_table
    n_frames = sum(x.n_frames for x in scs)
    log(f"scene {args.workload}: {len(scs)} scene(s), {n_frames} frames "
        f"({time.perf_counter() - t:.1f} s to generate)")

    m = RayMRF(0)
    trim = None
    if args.workload == "c5":
        scs, trim = trim_to_memory(m, scs, K, backward, args.mem_frac, kf_step)
        n_frames = sum(x.n_frames for x in scs)
        log(f"count pass: stated frames {trim['stated_frames']} ({trim['stated_slots']} slots, "
            f"~{trim['stated_estimated_gb']} GB), run with {trim['frames']} ({trim['slots']} slots, "
            f"~{trim['estimated_gb']} GB of {trim['memory_budget_gb']} GB)")
    m.upload(scs)
    theta = torch.from_numpy(np.concatenate([x.prior_logit() for x in scs])).cuda()
    sigma = torch.from_numpy(sc.sigma_table.astype(np.float32)).cuda()
    y = torch.from_numpy(np.concatenate([x.occupancy() for x in scs])).cuda() if backward else None

    def step():
        if kf_step:
            m.build_resident(keyframe_average=True)
            m.infer_keyframe_avg(theta, sigma, K, keep_checkpoints=backward)
            p, _ = m.marginals()
            if backward:
                m.backward((p - y) / p.numel())
            return
        m.build_resident()
        m.infer(theta, sigma, K, keep_checkpoints=backward)
        p, logit = m.marginals()
        if backward:
            m.backward((p - y) / p.numel())   # d BCE-with-logits / d logit

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done (E = {m.n_edges})")
    if not args.no_autotune:
        if args.warmup == 0:
            step()
        tun = m.autotune(reps=2)
        step()   # captures the graph with the chosen shapes
        torch.cuda.synchronize()
        log(f"autotuned: lanes {tun['fwd_lanes'][:8]} reverse {tun['adj_lanes'][:8]} x {tun['adj_rays'][:8]}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1e3 * dt / args.steps
    E = m.n_edges
    value = E * K / (ms / 1e3)
    log(f"timed {args.steps} steps: {ms:.2f} ms/step")

    # ---- breakdown (outside the timed region)
    def timed(fn, n=2):
        fn()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - a) / n

    st = m.stats()
    kf_pairs = st.n_keyframe_pairs
    if kf_step:   # the step's own scheme: per-keyframe averaged messages on the kept build
        def fwd():
            m.infer_keyframe_avg(theta, sigma, K)

        build_ms = timed(lambda: m.build_resident(keyframe_average=True), 1)
    else:
        def fwd():
            m.infer(theta, sigma, K)

        build_ms = timed(lambda: m.build_resident(), 1)
    m.set_schedule("graph")
    fwd_graph_ms = timed(fwd)
    m.set_schedule("plain")
    fwd_plain_ms = timed(fwd)
    m.set_schedule("graph")
    bwd_ms = None
    if backward:
        if kf_step:
            m.infer_keyframe_avg(theta, sigma, K, keep_checkpoints=True)
        else:
            m.infer(theta, sigma, K, keep_checkpoints=True)
        p, _ = m.marginals()
        gl = (p - y) / p.numel()
        bwd_ms = timed(lambda: m.backward(gl))
    log(f"build {build_ms:.1f} ms, forward graph {fwd_graph_ms:.1f} ms, plain {fwd_plain_ms:.1f} ms, "
        f"backward {bwd_ms}")
    fwd_bias_ms = bwd_bias_ms = acc_ms = dd_ms = fwd_cell_ms = bwd_cell_ms = None
    acc_counts, acc_clean, acc_by_k, clean_by_k = [0, 0], None, {}, {}
    kf_build_ms = kf_fwd_ms = kf_plain_ms = kf_clean = kf_bwd_ms = None
    kf_acc, kf_by_k, kf_clean_by_k, kf_prof = [0, 0], {}, {}, []
    if not args.quick:
        # the same sweeps with a learnt depth-bias table in the sensor model, and the
        # reverse pass that also returns its gradient
        from paper_2006_03512_amd import scenes as S
        bias = torch.from_numpy(S.bias_table(sc.sigma_table, 7).astype(np.float32)).cuda()
        fwd_bias_ms = timed(lambda: m.infer(theta, sigma, K, bias_table=bias))
        bwd_bias_ms = None
        if backward:
            m.infer(theta, sigma, K, keep_checkpoints=True, bias_table=bias)
            p, _ = m.marginals()
            gl = (p - y) / p.numel()
            bwd_bias_ms = timed(lambda: m.backward(gl, want_bias=True))
        log(f"with a bias table: forward graph {fwd_bias_ms:.1f} ms, backward {bwd_bias_ms}")
        # the same with sigma and bias tables per 20x20-pixel region (Sec. IV-C)
        ncell = m.set_sensor_cells(20)
        sig_c = sigma.reshape(1, -1).repeat(ncell, 1).contiguous()
        bias_c = bias.reshape(1, -1).repeat(ncell, 1).contiguous()
        fwd_cell_ms = timed(lambda: m.infer(theta, sig_c, K, bias_table=bias_c))
        bwd_cell_ms = None
        if backward:
            m.infer(theta, sig_c, K, keep_checkpoints=True, bias_table=bias_c)
            p, _ = m.marginals()
            gl = (p - y) / p.numel()
            bwd_cell_ms = timed(lambda: m.backward(gl, want_bias=True))
        m.set_sensor_cells(0)
        log(f"with tables per 20x20-pixel region ({ncell}): forward graph {fwd_cell_ms:.1f} ms, "
            f"backward {bwd_cell_ms}")
        # the accuracy metric of the inferred map over every pixel of the batch
        m.infer(theta, sigma, K)
        acc_ms = timed(lambda: m.accuracy())
        acc = m.accuracy()
        acc_counts = acc["counts"].cpu().numpy().sum(0).tolist()
        log(f"accuracy metric: {acc_ms:.1f} ms, {acc_counts[1]} of {acc_counts[0]} rays accurate")
        # the paper's evaluation rule (Sec. V): the most likely surface within 1.5 sigma(Z) of
        # the noise-free depth rendered from the same poses
        clean = torch.from_numpy(np.concatenate([x.extra["clean_depth"].reshape(-1) for x in scs])).cuda()

        def frac_clean():
            c = m.accuracy(ref_depth=clean, tol_nsigma=1.5)["counts"].cpu().numpy().sum(0)
            return round(float(c[1]) / max(float(c[0]), 1.0), 6)

        acc_clean = frac_clean()
        # the same metrics after 1..9 sweeps: flooding BP can cycle, and the map's quality
        # then depends on the phase the stated K lands in
        acc_by_k, clean_by_k = {}, {}
        for k in range(1, 10):
            m.infer(theta, sigma, k)
            c = m.accuracy()["counts"].cpu().numpy().sum(0)
            acc_by_k[str(k)] = round(float(c[1]) / max(float(c[0]), 1.0), 6)
            clean_by_k[str(k)] = frac_clean()
        log(f"accurate fraction by sweeps: {acc_by_k}; 1.5 sigma of noise-free depth: {clean_by_k}")
        # the ray factors' messages to their depth variables after K sweeps (Eq. depth_message)
        m.infer(theta, sigma, K)
        dd_ms = timed(lambda: m.depth_distribution())

        # per-keyframe averaged messages (Sec. IV-A) on the same batch: build, K sweeps,
        # and the accuracy metric after 1..9 sweeps
        kf_build_ms = timed(lambda: m.build_resident(keyframe_average=True), 1)
        kf_pairs = m.stats().n_keyframe_pairs
        kf_fwd_ms = timed(lambda: m.infer_keyframe_avg(theta, sigma, K))
        kf_plain_ms = None
        m.set_schedule("plain")
        kf_plain_ms = timed(lambda: m.infer_keyframe_avg(theta, sigma, K))
        m.set_schedule("graph")
        m.infer_keyframe_avg(theta, sigma, K)
        kf_acc = m.accuracy()["counts"].cpu().numpy().sum(0).tolist()
        kf_clean = frac_clean()
        kf_by_k, kf_clean_by_k = {}, {}
        for k in range(1, 10):
            m.infer_keyframe_avg(theta, sigma, k)
            c = m.accuracy()["counts"].cpu().numpy().sum(0)
            kf_by_k[str(k)] = round(float(c[1]) / max(float(c[0]), 1.0), 6)
            kf_clean_by_k[str(k)] = frac_clean()
        kf_bwd_ms = None
        if backward:   # the reverse pass through the keyframe-averaged sweeps
            m.infer_keyframe_avg(theta, sigma, K, keep_checkpoints=True)
            p, _ = m.marginals()
            gl = (p - y) / p.numel()
            kf_bwd_ms = timed(lambda: m.backward(gl))
        m.infer_keyframe_avg(theta, sigma, K)
        kf_prof = m.profile_sweeps(args.profile_reps, include_backward=False)
        log(f"keyframe average: build {kf_build_ms:.1f} ms ({kf_pairs} pairs), {K} sweeps {kf_fwd_ms:.1f} ms "
            f"(plain {kf_plain_ms:.1f}), reverse {kf_bwd_ms}, accurate fraction by sweeps {kf_by_k}")
        if not kf_step:
            m.build_resident()   # back to the plain graph for the profile below

    # ---- roofline of the dominant kernel (HIP events around each launch)
    if kf_step and kf_fwd_ms is None:   # --quick: the breakdown above timed the keyframe-average scheme
        kf_build_ms, kf_fwd_ms, kf_plain_ms, kf_bwd_ms = build_ms, fwd_graph_ms, fwd_plain_ms, bwd_ms
    if kf_step:
        m.infer_keyframe_avg(theta, sigma, K)
    else:
        m.infer(theta, sigma, K)
    prof = m.profile_sweeps(args.profile_reps, include_backward=backward)
    dom = max(prof, key=lambda k: k["avg_ms"] * k["launches"] / args.profile_reps)
    ach = dom["bytes_per_launch"] / (dom["avg_ms"] / 1e3) / 1e9
    sweep_ms = fwd_graph_ms / K   # one forward sweep in the captured graph (potentials and marginals included)
    fwd_bytes = st.fwd_bytes_per_sweep
    traffic = None
    if (TRAFFIC["workload"] == args.workload and dom["name"] in TRAFFIC["kernels"] and args.frames is None
            and TRAFFIC["src_sha256"] == src_sha256(TRAFFIC["sources"])):
        traffic = sum(TRAFFIC["kernels"][dom["name"]])
    # the same kernel and the sweeps at the per-edge bytes of the hot-path scope table
    # (ray phase 12, voxel phase 12, ray adjoint 16; a forward sweep 24, forward +
    # reverse 68 per edge and sweep), which leave out the builder's extra per-edge arrays
    nm = dom["name"]
    survey_b = 16.0 if nm.startswith("ray_adj") else 12.0
    dom_edges = dom.get("edges_per_launch", 0)
    ach_survey = survey_b * dom_edges / (dom["avg_ms"] / 1e3) / 1e9
    fwd_ms_step = kf_fwd_ms if kf_step else fwd_graph_ms
    survey = {"kernel_bytes_per_edge": survey_b, "kernel_GBs": round(ach_survey, 1),
              "forward_24B_GBs": round(24.0 * E * K / (fwd_ms_step / 1e3) / 1e9, 1)}
    survey["forward_frac"] = round(survey["forward_24B_GBs"] / HBM_PEAK_GBS, 4)
    if backward:
        survey["fwd_bwd_68B_GBs"] = round(68.0 * E * K / ((fwd_graph_ms + bwd_ms) / 1e3) / 1e9, 1)
        survey["fwd_bwd_frac"] = round(survey["fwd_bwd_68B_GBs"] / HBM_PEAK_GBS, 4)
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "frac_survey": round(ach_survey / HBM_PEAK_GBS, 4),
                "survey_bytes": survey, "traffic": traffic, "kernel": dom["name"],
                "kernel_avg_ms": round(dom["avg_ms"], 4),
                "bytes_per_launch": dom["bytes_per_launch"],
                "forward_sweep_ms": round(sweep_ms, 3),
                "forward_sweep_algorithmic_GBs": round(fwd_bytes / (sweep_ms / 1e3) / 1e9, 1),
                "forward_sweep_frac": round(fwd_bytes / (sweep_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    kernels = [{"name": k["name"], "avg_ms": round(k["avg_ms"], 4), "launches": k["launches"],
                "GBs": round(k["bytes_per_launch"] / max(k["avg_ms"], 1e-9) / 1e6, 1)} for k in prof]
    # achievable HBM bandwidth on this part: a plain 2 GiB device copy (read + write), HIP events
    copy_gbs = copy_bandwidth(2 << 30)
    roofline["copy_GBs"] = round(copy_gbs, 1)
    roofline["frac_of_copy"] = round(ach / copy_gbs, 4)
    log(f"device copy: {copy_gbs:.0f} GB/s; dominant kernel at {ach / copy_gbs:.1%} of it")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(args.workload, sc, K, backward, args.cpu_rows, args.cpu_frames)
        log(f"cpu baseline: {cpu['value']:.3e} {UNIT} on {cpu['cores']} threads")

    def r2(x):
        return None if x is None else round(x, 2)

    line = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (f64 traversal)", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "scenes": len(scs), "frames": n_frames,
                   "grid": [[x.grid.nx, x.grid.ny, x.grid.nz] for x in scs],
                   "voxel_m": [x.grid.voxel for x in scs],
                   "sweeps": K, "rays": st.n_rays, "edges": E, "voxels": st.n_voxels,
                   "edge_slots": st.n_slots, "tiles": st.n_tiles, "slot_groups": st.n_slot_groups,
                   "touched_voxels": st.n_touched_voxels, "max_ray_len": st.max_ray_len,
                   "max_voxel_degree": st.max_voxel_degree, "parallelism": "single GPU",
                   "grid_storage": ("dense" if args.sparse_bricks < 0
                                    else f"sparse bricks, radius {args.sparse_bricks}"),
                   "frames_per_scene": [int(x.n_frames) for x in scs],
                   "count_pass": trim,
                   "ray_len_log2_hist": st.ray_len_hist[:12],
                   "voxel_degree_log2_hist": st.voxel_degree_hist[:20]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "breakdown_ms": {"build": round(build_ms, 2), "forward_graph": round(fwd_graph_ms, 2),
                         "forward_plain_per_frame": round(fwd_plain_ms, 2),
                         "backward": None if bwd_ms is None else round(bwd_ms, 2),
                         "forward_graph_with_bias": None if fwd_bias_ms is None else round(fwd_bias_ms, 2),
                         "backward_with_bias_grad": None if bwd_bias_ms is None else round(bwd_bias_ms, 2),
                         "forward_graph_with_20px_region_tables": (None if fwd_cell_ms is None
                                                                   else round(fwd_cell_ms, 2)),
                         "backward_with_20px_region_table_grads": (None if bwd_cell_ms is None
                                                                   else round(bwd_cell_ms, 2)),
                         "accuracy_metric": None if acc_ms is None else round(acc_ms, 2),
                         "depth_messages": None if dd_ms is None else round(dd_ms, 2)},
        "map_accuracy": {"rule": "measurement inside the chord of the most likely surface's voxel (Sec. III-D)",
                         "evaluated_rays": acc_counts[0], "accurate_rays": acc_counts[1],
                         "fraction": acc_counts[1] / max(acc_counts[0], 1), "vis_min": 0.5,
                         "fraction_by_sweeps": acc_by_k,
                         "rule_1p5sigma": "most likely surface within 1.5 sigma(Z) of the noise-free depth (Sec. V)",
                         "fraction_1p5sigma_noise_free": acc_clean,
                         "fraction_1p5sigma_noise_free_by_sweeps": clean_by_k},
        "forward_updates_per_s": {"batched_graph": E * K / (fwd_graph_ms / 1e3),
                                  "plain_per_frame": E * K / (fwd_plain_ms / 1e3),
                                  "plain_schedule": "eager launches, one per frame and ray class, "
                                                    "untuned one-wave-per-ray shapes, no graph"},
        "keyframe_average": None if kf_fwd_ms is None else {
                             "pairs": kf_pairs, "build_ms": r2(kf_build_ms),
                             "forward_graph_ms": r2(kf_fwd_ms),
                             "forward_plain_per_frame_ms": r2(kf_plain_ms),
                             "backward_ms": r2(kf_bwd_ms),
                             "updates_per_s": E * K / (kf_fwd_ms / 1e3),
                             "map_accuracy": {"evaluated_rays": kf_acc[0], "accurate_rays": kf_acc[1],
                                              "fraction": kf_acc[1] / max(kf_acc[0], 1), "vis_min": 0.5,
                                              "fraction_by_sweeps": kf_by_k,
                                              "fraction_1p5sigma_noise_free": kf_clean,
                                              "fraction_1p5sigma_noise_free_by_sweeps": kf_clean_by_k},
                             "kernels": [{"name": k["name"], "avg_ms": round(k["avg_ms"], 4),
                                          "launches": k["launches"],
                                          "GBs": round(k["bytes_per_launch"] / max(k["avg_ms"], 1e-9) / 1e6, 1)}
                                         for k in kf_prof]},
        "kernels": kernels,
        "tuning": {k: v for k, v in m.tuning().items() if k in ("cap", "fwd_lanes", "adj_lanes", "adj_rays")},
        "autotuned": not args.no_autotune,
    }
    if backward:
        line["fwd_bwd_edge_sweeps_per_s"] = E * K / ((fwd_graph_ms + bwd_ms) / 1e3)
    print(json.dumps(line), flush=True)
    m.close()


if __name__ == "__main__":
    main()
