#!/usr/bin/env python3
"""Benchmark of the dilation-based ICP hot path on one MI355X.

A step is one pass of the whole hot path over the indoor-scene workload
(226,000 target / 200,000 source points, voxel 0.05 m, 3 dilation rings,
30 ICP iterations): voxelise + count, offset scan, scatter + order, dilation,
then 30 x (local/global search, moments, float64 solve).  Inputs are
resident in HBM before the timed region.  Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Extra figures on the same line: ICP iterations/s, the dilation-buffer bytes
of every workload against the fixed 64 KiB-per-voxel allocation, the
batched (64 pairs) and differentiable (16 x 40k forward + backward) forms,
per-kernel times from HIP events, the roofline of the dominant kernel and the
CPU oracle timed on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NNS queries/s + ICP iters/s at 226K pts; dilation buffer bytes; fwd+bwd pairs/s"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3        # published dense float32 vector peak
# flops per byte of the search: one candidate is 16 bytes (x, y, z, index)
# and 8 flops (3 subtractions, 1 multiply, 2 fused multiply-adds)
SEARCH_FLOPS_PER_BYTE = 8.0 / 16.0
PROFILE_PMC = os.path.join(ROOT, "profiles", "nns_local_room_226k_pmc.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2512_04996_amd", "csrc", "k_nns.hip")
PROFILE_PMC_DIL = os.path.join(ROOT, "profiles", "dilate_fused_room_226k_pmc.json")
KERNEL_SRC_DIL = os.path.join(ROOT, "paper_2512_04996_amd", "csrc", "k_dilate.hip")


def counter_traffic(pmc_path, src_path, kernel):
    """HBM bytes per launch of this kernel variant from a stored FETCH_SIZE +
    WRITE_SIZE summary, or None when the variant is not in it or its source
    changed since the counters were taken."""
    if not os.path.exists(pmc_path):
        return None
    pmc = json.load(open(pmc_path))
    src_hash = hashlib.sha256(open(src_path, "rb").read()).hexdigest()
    if pmc.get("kernel_source_sha256") != src_hash:
        return None
    v = pmc.get("variants", {}).get(kernel)
    return None if v is None else v.get("hbm_bytes_per_launch")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="room_226k")
    ap.add_argument("--graph", type=int, default=1, help="replay the ICP iterations from a hipGraph")
    ap.add_argument("--schedule", default="auto",
                    help="search schedule: 'auto' (tuned on this workload first) or "
                         "'BLOCK,LANES,SORT,FALLBACK_GRID[,SEARCH_MODE]', e.g. 128,2,0,64")
    ap.add_argument("--build-schedule", default=None,
                    help="with a given --schedule: 'COUNT_BLOCK,DILATE_FUSED,DILATE_TILE,RING_BLOCK', e.g. 256,1,0,256")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the batched / differentiable / bytes figures")
    ap.add_argument("--no-prof", action="store_true", help="no per-kernel HIP events in the timed region")
    ap.add_argument("--separate-calls", action="store_true",
                    help="time a step as rebuild, dilate and register in turn instead of one vicp_rebuild_register")
    ap.add_argument("--extra-only", choices=("batched", "diff"), default=None,
                    help="run only this extra figure (64-pair batch or 16x40k differentiable loss) and print it")
    ap.add_argument("--calib-copy-mib", type=float, default=0.0,
                    help="after the run, one plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def nns_local_bytes(m, F, cand, nrecords):
    """Algorithmic bytes of one registration-search launch (each logical
    access once): per query 16 (the bucketed source point, float4) + 8 (its
    voxel's search-directory entry); 16 per candidate (float4 x, y, z,
    index); 12 per query sent to the global search (list slot + 64-bit key);
    per wave one record of 19 float64 moments + 3 counters (176)."""
    return m * 24 + 16 * cand + 12 * F + 176 * nrecords


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; multi-GPU runs are not part of it",
                          "n_gpus": a.gpus}), flush=True)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2512_04996_amd import _lib, api, synth
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    if a.extra_only:
        fig = (batched_figure if a.extra_only == "batched" else diff_figure)(api, synth, torch, dev, np)
        print(json.dumps({"extra_only": a.extra_only, "figure": fig}), flush=True)
        return

    P = synth.config(a.workload)
    q = torch.from_numpy(P.q).to(dev)
    p = torch.from_numpy(P.p).to(dev)
    torch.cuda.synchronize()

    # one grid object serves every step: each step refills it from the target
    # (bounding box, counts, offsets, segments), dilates it and registers
    g = api.build_grid(q, P.voxel, P.rings)
    if a.schedule == "auto":
        g.dilate(P.rings)
        g.autotune(p, searches_per_plan=P.iters)
    else:
        vals = [int(x) for x in a.schedule.split(",")]
        bs, lpq, srt, fg = vals[:4]
        g.set_schedule(bs, lpq, bool(srt), fg, vals[4] if len(vals) > 4 else 0)
        if a.build_schedule:
            cb, fu, ti, rb = (int(x) for x in a.build_schedule.split(","))
            g.set_build_schedule(cb, bool(fu), ti, rb)
    schedule = g.schedule
    tf = lambda b: "true" if b else "false"
    # the variant that runs: registration form over segments, single pair
    nns_variant = (f"k_nns_local<{schedule['nns_block']}, {schedule['lanes_per_query']}, "
                   f"{tf(schedule['sort_source'])}, true, false, {schedule['search_mode']}, true>")
    # one moment record per search wave
    nns_records = -(-P.m * schedule['lanes_per_query'] // schedule['nns_block']) * (schedule['nns_block'] // 64)
    build_schedule = g.build_schedule

    def step():
        if a.separate_calls:
            g.rebuild(q)
            g.dilate(P.rings)
            return g.register(p, P.iters, use_graph=bool(a.graph))
        # the same work in one call: the refill's passes share launches with the source plan's
        return g.rebuild_register(q, P.rings, p, P.iters, use_graph=bool(a.graph))

    log(f"[bench] workload {P.name}: n={P.n} m={P.m} voxel={P.voxel} rings={P.rings} iters={P.iters}")
    # the timed region runs with no timing events at all (events recorded
    # inside a graph perturb it); per-kernel durations come from an eager
    # pass of the same steps afterwards
    for _ in range(max(a.warmup, 1)):
        res = step()
    log("[bench] warmup done")
    torch.cuda.synchronize()
    step_ms = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        ts = time.perf_counter()
        res = step()   # ends with the registration's result copy, a stream synchronisation
        step_ms.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log("[bench] timed region done")
    ms = (t1 - t0) * 1e3 / a.steps
    # the two parts of a step on their own: the grid refill + dilation, and
    # the registration (one graph replay of the K iterations)
    reps = max(5, min(a.steps, 20))
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for _ in range(reps):
        g.rebuild(q)
        g.dilate(P.rings)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - tb) * 1e3 / reps
    reg_ms = []
    for _ in range(reps):
        ts = time.perf_counter()
        g.register(p, P.iters, use_graph=bool(a.graph))
        reg_ms.append((time.perf_counter() - ts) * 1e3)
    K = int(res.iters[0])
    queries_per_s = K * P.m / (ms * 1e-3)
    kernels = {}
    timing_pass = None
    per_iter = None
    if not a.no_prof:
        prof_steps = min(a.steps, 5)
        api.prof_reset()
        api.prof_enable(True)
        for _ in range(prof_steps):
            g.rebuild(q)
            g.dilate(P.rings)
            g.register(p, P.iters, use_graph=False)
        torch.cuda.synchronize()
        api.prof_enable(False)
        timing_pass = (f"eager pass of {prof_steps} steps after the timed region: search, global search and solve "
                       "timed by start/stop HIP events recorded at the kernel (hipExtLaunchKernelGGL), other "
                       "kernels by HIP events around the launch")
        for name in ("aabb", "count", "scan", "place", "rank_sort", "dilate", "dilate_ring", "src_plan", "nns_local",
                     "fallback", "solve"):
            n_launch, tot = api.prof_read(name)
            if n_launch:
                kernels[name] = {"launches_per_step": n_launch / prof_steps, "avg_us": 1e3 * tot / n_launch,
                                 "ms_per_step": tot / prof_steps}
        # per-iteration search time (local search + global search), each
        # iteration's mean over the timing pass's steps
        ns, fs = api.prof_samples("nns_local"), api.prof_samples("fallback")
        if len(ns) == len(fs) == prof_steps * P.iters:
            it = (np.asarray(ns) + np.asarray(fs)).reshape(prof_steps, P.iters).mean(0) * 1e-3
            per_iter = {"median_s": float(np.median(it)), "iter0_s": float(it[0]),
                        "nns_local_median_us": float(np.median(np.asarray(ns).reshape(prof_steps, P.iters).mean(0))) * 1e3}
        if not a.separate_calls:
            # the timed step's paired launches (refill pass + source plan pass)
            api.prof_reset()
            api.prof_enable(True)
            for _ in range(prof_steps):
                g.rebuild_register(q, P.rings, p, P.iters, use_graph=False)
            torch.cuda.synchronize()
            api.prof_enable(False)
            for name in ("start_frame", "count_bucket", "scan_pair", "place_pair", "rank_pair"):
                n_launch, tot = api.prof_read(name)
                if n_launch:
                    kernels[name] = {"launches_per_step": n_launch / prof_steps, "avg_us": 1e3 * tot / n_launch,
                                     "ms_per_step": tot / prof_steps}

    F = np.asarray(res.fallbacks[0], np.int64)
    cand = np.asarray(res.candidates[0], np.int64)
    dil = np.asarray(res.dilated_lookups[0], np.int64)
    per_launch = [nns_local_bytes(P.m, int(F[k]), int(cand[k]), nns_records) for k in range(K)]
    bytes_per_launch = float(np.mean(per_launch))
    roofline = None
    if "nns_local" in kernels:
        dur_s = kernels["nns_local"]["avg_us"] * 1e-6
        achieved = bytes_per_launch / dur_s / 1e9
        # counters of this very kernel variant, taken from the current source
        traffic = counter_traffic(PROFILE_PMC, KERNEL_SRC, nns_variant)
        # the roofline that bounds the kernel, from its arithmetic intensity
        # against the machine balance (peak flops / peak bytes)
        balance = FP32_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
        bound = "hbm" if SEARCH_FLOPS_PER_BYTE < balance else "alu"
        measured = None if traffic is None else traffic / dur_s / 1e9
        if measured is None:
            limiter = "unknown (no counter traffic for this kernel source)"
        elif measured < 0.5 * HBM_PEAK_GBS:
            limiter = (f"latency: the counters see {measured:.0f} GB/s of HBM traffic ({measured / HBM_PEAK_GBS:.2f} "
                       f"of peak); the rest of the algorithmic bytes are served by the caches")
        else:
            limiter = "hbm bandwidth"
        roofline = {"kernel": nns_variant, "bound": bound, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "hbm_measured_gbs": None if measured is None else round(measured, 1),
                    "hbm_frac": None if measured is None else round(measured / HBM_PEAK_GBS, 4),
                    "limiter": limiter,
                    "flops_per_byte": SEARCH_FLOPS_PER_BYTE, "machine_balance_flops_per_byte": round(balance, 2),
                    "timing": "mean of the per-launch start/stop HIP events of the eager timing pass",
                    "algorithmic_bytes_per_launch": int(bytes_per_launch),
                    "mean_candidates_per_query": round(float(cand.mean()) / P.m, 3),
                    "dilated_lookup_fraction": round(float(dil.mean()) / P.m, 4)}

    desc = g.describe()
    g.free()
    ours = desc["dynamic_bytes"] + desc["static_bytes"]
    dil_bytes = {"workload": P.name, "V": desc["V"], "occupied": desc["occupied"], "dilated": desc["dilated"],
                 "dynamic_bytes": desc["dynamic_bytes"], "static_bytes": desc["static_bytes"],
                 "vanicp_fixed_bytes": desc["vanicp_bytes"],
                 "saving": round(1.0 - ours / desc["vanicp_bytes"], 6),
                 # not graded: 64 KiB for the occupied and dilated voxels only,
                 # and a tight uniform block of (largest count + 2) words per voxel
                 "vanicp_occupied_dilated_bytes": 65536 * (desc["occupied"] + desc["dilated"]),
                 "saving_vs_occupied_dilated": round(1.0 - ours / (65536 * (desc["occupied"] + desc["dilated"])), 6),
                 "tight_uniform_bytes": (desc["max_count"] + 2) * 4 * desc["V"],
                 "extra_device_bytes": desc["extra_bytes"]}
    # global atomics of the count: one per distinct (256-point block, voxel)
    # after the LDS hash, against one per point without it (float32
    # quantisation as the kernel's, computed here with numpy)
    o32 = np.asarray(desc["origin"], np.float32)
    inv32 = np.float32(desc["inv"])
    f = (P.q - o32[:, None]) * inv32
    ijk = np.floor(f).astype(np.int64)
    dims = np.asarray(desc["dims"], np.int64)
    vox = ijk[0] + dims[0] * (ijk[1] + dims[1] * ijk[2])
    blk = np.arange(P.n) // 256
    atomics = int(np.unique(blk * desc["V"] + vox).size)
    # the dilation's bytes, two ways.  This kernel's own compulsory bytes:
    # all rings in one launch read each voxel's directory entry once (8;
    # the halo re-reads hit the caches) and, per dilated voxel, write its
    # count word (4) and its directory entry (8).  The ring model: every ring
    # reads each voxel's offset and count word (8) and writes each newly
    # dilated voxel's word (4), i.e. 8 L V + 4 (dilated) for L rings.
    dilation_roof = None
    V, nd = desc["V"], desc["dilated"]
    ring_model = 8 * P.rings * V + 4 * nd
    tiles = ("8x8x4", "16x8x4", "8x8x8", "32x8x4", "16x16x4")
    if "dilate" in kernels:
        dur = kernels["dilate"]["avg_us"] * 1e-6
        dbytes = 8 * V + 12 * nd
        ach = dbytes / dur / 1e9
        t = tiles[build_schedule["dilate_tile"]].split("x")
        dname = f"k_dilate_fused<{P.rings}, {t[0]}, {t[1]}, {t[2]}>"
        dtraffic = counter_traffic(PROFILE_PMC_DIL, KERNEL_SRC_DIL, dname)
        dmeas = None if dtraffic is None else dtraffic / dur / 1e9
        dilation_roof = {"kernel": dname, "bound": "hbm",
                         "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(ach / HBM_PEAK_GBS, 4), "compulsory_bytes_per_launch": int(dbytes),
                         "ring_model_bytes": int(ring_model),
                         "ring_model_frac": round(ring_model / dur / 1e9 / HBM_PEAK_GBS, 4),
                         "traffic": dtraffic,
                         "hbm_frac": None if dmeas is None else round(dmeas / HBM_PEAK_GBS, 4),
                         "limiter": ("unknown (no counter traffic for this kernel source)" if dmeas is None else
                                     f"latency: one round of about 1.6 blocks per CU, each a chain of a load "
                                     f"round, the rings in LDS and the writes; the counters see "
                                     f"{dmeas:.0f} GB/s of HBM traffic"),
                         "avg_us": round(kernels["dilate"]["avg_us"], 3)}
    elif "dilate_ring" in kernels:
        dur = kernels["dilate_ring"]["avg_us"] * 1e-6 * P.rings
        ach = ring_model / dur / 1e9
        dilation_roof = {"kernel": f"k_dilate_ring<{build_schedule['ring_block']}> x {P.rings}", "bound": "hbm",
                         "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(ach / HBM_PEAK_GBS, 4), "ring_model_bytes": int(ring_model),
                         "avg_us_all_rings": round(dur * 1e6, 3)}
    search_qps = None
    if "nns_local" in kernels and "fallback" in kernels:
        it_us = kernels["nns_local"]["avg_us"] + kernels["fallback"]["avg_us"]
        search_qps = round(P.m / (it_us * 1e-6), 1)
    nns_qps = None
    if per_iter is not None:
        nns_qps = {"median_over_iterations": round(P.m / per_iter["median_s"], 1),
                   "iteration0": round(P.m / per_iter["iter0_s"], 1),
                   "median_iteration_us": round(per_iter["median_s"] * 1e6, 3),
                   "iteration0_us": round(per_iter["iter0_s"] * 1e6, 3),
                   "what": "source points / (local search + global search time of one iteration), per-launch HIP "
                           "events of the timing pass, each iteration averaged over its steps"}
    # attainable bandwidth: a plain device-to-device copy of 1 GiB (with the
    # timing pass only: profiler runs keep their copies to the calibration one)
    if roofline is not None:
        nel = (1 << 30) // 4
        src = torch.ones(nel, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        roofline["attainable_copy_gbs"] = round(2.0 * (1 << 30) * 10 / (time.perf_counter() - tc) / 1e9, 1)
        del src, dst

    out = {
        "metric": METRIC, "value": round(queries_per_s, 1), "unit": "queries/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": P.name, "n_target": P.n, "n_source": P.m, "voxel": P.voxel, "rings": P.rings,
                   "iters": P.iters, "step": "grid build + dilation + 30 ICP iterations",
                   "step_call": ("vicp_grid_rebuild, vicp_dilate, vicp_register in turn" if a.separate_calls else
                                 "vicp_rebuild_register (the refill's passes paired with the source plan's in shared launches)"),
                   "icp_mode": "graph" if a.graph else "eager", "schedule": schedule,
                   "build_schedule": build_schedule,
                   "schedule_source": "autotuned" if a.schedule == "auto" else "given",
                   "kernel_timing": timing_pass},
        "icp_iters_per_s": round(K / (ms * 1e-3), 2),
        "step_ms_median": round(float(np.median(step_ms)), 4),
        "step_ms_p90": round(float(np.percentile(step_ms, 90)), 4),
        "build_ms": round(build_ms, 4),
        "register_ms_median": round(float(np.median(reg_ms)), 4),
        "register_ms_p90": round(float(np.percentile(reg_ms, 90)), 4),
        "icp_iters_per_s_registration": round(K / (float(np.median(reg_ms)) * 1e-3), 2),
        "search_queries_per_s": search_qps,
        "nns_queries_per_s": nns_qps,
        "global_searches_per_iter": [int(x) for x in F],
        "count_global_atomics": {"with_lds_hash": atomics, "one_per_point": P.n},
        "roofline": roofline,
        "roofline_dilation": dilation_roof,
        "kernels": kernels,
        "dilation_buffer": dil_bytes,
    }
    log(f"[bench] {ms:.3f} ms/step, {queries_per_s:.3e} queries/s")

    if not a.no_extra:
        out["extra"] = extra_figures(api, synth, torch, dev, np)

    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(P)

    if a.calib_copy_mib > 0:
        nel = int(a.calib_copy_mib * 2 ** 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_mib"] = a.calib_copy_mib

    print(json.dumps(out), flush=True)


def extra_figures(api, synth, torch, dev, np):
    """Batched and differentiable forms and the buffer bytes of every workload."""
    ex = {}
    # dilation-buffer bytes of the other workloads
    sizes = {}
    for name in ("sphere_2k", "bumpy_40k"):
        Pw = synth.config(name)
        g = api.build_grid(torch.from_numpy(Pw.q).to(dev), Pw.voxel, Pw.rings)
        g.dilate(Pw.rings)
        d = g.describe()
        g.free()
        sizes[name] = {"V": d["V"], "dynamic_bytes": d["dynamic_bytes"], "static_bytes": d["static_bytes"],
                       "vanicp_fixed_bytes": d["vanicp_bytes"],
                       "saving": round(1 - (d["dynamic_bytes"] + d["static_bytes"]) / d["vanicp_bytes"], 6)}
    # the paper's own setting: unit-sphere clouds, 2^4 voxels per axis, L = 10,
    # up to 50 iterations with the RMSE-difference stop; a step is the grid
    # refill, the dilation and the registration
    log("[bench] paper setting")
    paper = {}
    for name in ("paper_bunny_40k", "paper_room_226k"):
        Pw = synth.config(name)
        qd = torch.from_numpy(Pw.q).to(dev)
        pd_ = torch.from_numpy(Pw.p).to(dev)
        g = api.build_grid_fixed(qd, Pw.meta["grid_origin"], Pw.voxel, Pw.meta["grid_dims"], Pw.rings)
        g.dilate(Pw.rings)
        g.autotune(pd_, searches_per_plan=Pw.iters)

        def run():
            g.rebuild(qd)
            g.dilate(Pw.rings)
            return g.register(pd_, Pw.iters, rmse_eps=Pw.meta["rmse_eps"], early_stop=True, use_graph=True)

        for _ in range(2):
            r = run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            r = run()
        torch.cuda.synchronize()
        tp = (time.perf_counter() - t0) / 5
        d = g.describe()
        k = int(r.iters[0])
        paper[name] = {"iters": k, "ms": round(tp * 1e3, 3), "queries_per_s": round(k * Pw.m / tp, 1),
                       "schedule": g.schedule, "V": d["V"], "static_bytes": d["static_bytes"],
                       "static_mib": d["static_bytes"] / 2 ** 20, "dynamic_bytes": d["dynamic_bytes"],
                       "candidates_per_query": round(float(np.mean(r.candidates[0][:k])) / Pw.m, 1),
                       "final_rmse": float(r.rmse[0][k - 1])}
        g.free()
    ex["paper_setting"] = paper
    # the Alg. 1 ablation: the paper's host-side offset scan (MOC) and fused
    # LDS hash entry against the defaults, on the main workload's build
    log("[bench] Alg. 1 ablation")
    Pm = synth.config("room_226k")
    qd = torch.from_numpy(Pm.q).to(dev)
    g = api.build_grid(qd, Pm.voxel, Pm.rings)
    abl = {}
    for label, host, packed in (("default", False, False), ("packed_hash", False, True),
                                ("host_offsets", True, False)):
        g.set_build_options(host_offsets=host, packed_hash=packed)
        for _ in range(2):
            g.rebuild(qd)
        torch.cuda.synchronize()
        api.prof_reset()
        api.prof_enable(True)
        t0 = time.perf_counter()
        for _ in range(10):
            g.rebuild(qd)
        torch.cuda.synchronize()
        tr = (time.perf_counter() - t0) / 10
        api.prof_enable(False)
        row = {"rebuild_ms": round(tr * 1e3, 4)}
        for k in ("count", "scan", "moc_host"):
            n_l, tot = api.prof_read(k)
            if n_l:
                row[k + "_us"] = round(1e3 * tot / n_l, 2)
        abl[label] = row
    g.free()
    abl["note"] = ("rebuild = bounding box + count + offsets + scatter + order; moc_host is the serial host "
                   "scan alone, the rebuild also pays the histogram and offset copies")
    ex["alg1_ablation"] = abl
    # the exhaustive-NNS comparator (Table 2's "Brute") on the main workload:
    # the same 30 iterations with the exact global search for every query
    log("[bench] exhaustive comparator")
    Pm = synth.config("room_226k")
    qd = torch.from_numpy(Pm.q).to(dev)
    pd_ = torch.from_numpy(Pm.p).to(dev)
    g = api.build_grid(qd, Pm.voxel, Pm.rings)
    g.dilate(Pm.rings)
    g.set_schedule(128, 2, False, 1024)
    rb = g.register(pd_, Pm.iters, use_graph=True, global_only=True)   # warm-up and capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rb = g.register(pd_, Pm.iters, use_graph=True, global_only=True)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    g.autotune(pd_, searches_per_plan=Pm.iters)
    rd = g.register(pd_, Pm.iters, use_graph=True)
    g.free()
    Rb, Rd = rb.Rt[:9].reshape(3, 3), rd.Rt[:9].reshape(3, 3)
    Rtrue = np.asarray(Pm.R_true).T          # the registration maps p back onto q
    ang = lambda A, B: float(np.degrees(np.arccos(np.clip((np.trace(A.T @ B) - 1) / 2, -1, 1))))
    ex["exhaustive_comparator"] = {
        "workload": Pm.name, "iters": Pm.iters, "ms": round(tb * 1e3, 3),
        "queries_per_s": round(Pm.iters * Pm.m / tb, 1),
        "distance_evals_per_s": round(Pm.iters * Pm.m * Pm.n / tb, 1),
        "final_rmse_exhaustive": float(rb.rmse[0][-1]), "final_rmse_dilated": float(rd.rmse[0][-1]),
        "rotation_gap_deg": ang(Rb, Rd), "translation_gap": float(np.linalg.norm(rb.Rt[9:] - rd.Rt[9:])),
        "rotation_error_deg_exhaustive": ang(Rb, Rtrue), "rotation_error_deg_dilated": ang(Rd, Rtrue)}
    ex["vanicp_comparator"] = vanicp_comparator(api, synth, torch, dev, np)
    ex["batched_64"] = batched_figure(api, synth, torch, dev, np)
    ex["diff_16x40k"] = diff_figure(api, synth, torch, dev, np)
    ex["dilation_buffer_other"] = sizes
    return ex


def batched_figure(api, synth, torch, dev, np):
    """64 uneven pairs in one launch sequence, against a loop of single-pair runs."""
    ex = {}
    # batched: 64 uneven pairs in one launch sequence, against a loop of single-pair runs
    log("[bench] batched workload")
    pairs = synth.config("batched_64")
    qc = torch.from_numpy(np.concatenate([x.q for x in pairs], 1)).to(dev)
    pc = torch.from_numpy(np.concatenate([x.p for x in pairs], 1)).to(dev)
    ns = [x.n for x in pairs]
    ms_ = [x.m for x in pairs]
    vox = [x.voxel for x in pairs]
    iters = pairs[0].iters

    gb = api.build_grid_batched(qc, ns, vox, 3)
    gb.dilate(3)
    gb.autotune(pc, m_per_pair=ms_, searches_per_plan=iters)
    V_total = sum(gb.describe(b)["V"] for b in range(len(pairs)))

    def batched():
        gb.rebuild(qc)
        gb.dilate(3)
        return gb.register(pc, iters, m_per_pair=ms_, use_graph=True)

    qs = [torch.from_numpy(x.q).to(dev) for x in pairs]
    ps = [torch.from_numpy(x.p).to(dev) for x in pairs]
    singles = [api.build_grid(qs[b], x.voxel, 3) for b, x in enumerate(pairs)]
    for x in singles:
        x.set_schedule(**gb.schedule)      # the same kernels, so results can match bit for bit

    def looped():
        out = []
        for b in range(len(pairs)):
            singles[b].rebuild(qs[b])
            singles[b].dilate(3)
            out.append(singles[b].register(ps[b], iters, use_graph=True))
        return out

    for _ in range(2):
        rb = batched()
        looped()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        rb = batched()
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / 5
    t0 = time.perf_counter()
    for _ in range(2):
        rl = looped()
    torch.cuda.synchronize()
    tl = (time.perf_counter() - t0) / 2
    same = all(np.array_equal(rb.Rt[b], rl[b].Rt) for b in range(len(pairs)))
    fb0 = int(sum(int(f[0]) for f in rb.fallbacks if len(f)))
    gb.free()
    for x in singles:
        x.free()
    ex["batched_64"] = {"pairs": len(pairs), "points": int(sum(ns)), "V_total": int(V_total),
                        "ms": round(tb * 1e3, 3), "pairs_per_s": round(len(pairs) / tb, 2),
                        "pair_iters_per_s": round(len(pairs) * iters / tb, 1),
                        "looped_single_ms": round(tl * 1e3, 3), "speedup_vs_looped": round(tl / tb, 3),
                        "bit_identical_to_looped": bool(same), "fallbacks_iter0": fb0,
                        "vanicp_fixed_bytes": int(65536 * V_total)}
    return ex["batched_64"]


def diff_figure(api, synth, torch, dev, np):
    """The differentiable loss, 16 x 40k forward + backward, against 16 single-pair calls."""
    from paper_2512_04996_amd.autograd import p2p_loss
    ex = {}
    # differentiable: 16 x 40k forward + backward
    log("[bench] differentiable workload")
    dpairs, xi = synth.config("diff_16x40k")
    B = len(dpairs)
    qd = torch.from_numpy(np.concatenate([x.q for x in dpairs], 1)).to(dev)
    P3 = torch.from_numpy(np.stack([x.p.T for x in dpairs])).to(dev)       # (16, 40000, 3)
    g = api.build_grid_batched(qd, [x.n for x in dpairs], [x.voxel for x in dpairs], 2)
    g.dilate(2)
    g.autotune(P3.permute(2, 0, 1).reshape(3, -1).contiguous(), m_per_pair=[x.m for x in dpairs])
    xit = torch.from_numpy(xi).to(dev)

    def fwd_bwd():
        Pg = P3.detach().requires_grad_(True)
        xg = xit.detach().requires_grad_(True)
        L = p2p_loss(g, Pg, xg).sum()
        L.backward()
        return Pg.grad, xg.grad

    for _ in range(3):
        gb_P, gb_x = fwd_bwd()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nrep = 20
    for _ in range(nrep):
        fwd_bwd()
    torch.cuda.synchronize()
    td = (time.perf_counter() - t0) / nrep
    # the same 16 forward + backward passes as single-pair calls, one grid
    # per pair under the same schedule, at the same accuracy (compared)
    singles = []
    for b, x in enumerate(dpairs):
        gs = api.build_grid(torch.from_numpy(x.q).to(dev), x.voxel, 2)
        gs.dilate(2)
        gs.set_schedule(**g.schedule)
        singles.append(gs)

    def single_fwd_bwd():
        out = []
        for b in range(B):
            Pg = P3[b:b + 1].detach().requires_grad_(True)
            xg = xit[b:b + 1].detach().requires_grad_(True)
            L = p2p_loss(singles[b], Pg, xg).sum()
            L.backward()
            out.append((Pg.grad, xg.grad))
        return out

    for _ in range(3):
        sl = single_fwd_bwd()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nrep):
        single_fwd_bwd()
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / nrep
    same = all(torch.equal(sl[b][0][0], gb_P[b]) and torch.equal(sl[b][1][0], gb_x[b]) for b in range(B))
    for gs in singles:
        gs.free()
    g.free()
    ex["diff_16x40k"] = {"pairs": B, "points_per_pair": dpairs[0].m, "ms_fwd_bwd": round(td * 1e3, 3),
                         "fwd_bwd_pairs_per_s": round(B / td, 1),
                         "single_pair_calls_ms": round(ts * 1e3, 3),
                         "single_pair_calls_pairs_per_s": round(B / ts, 1),
                         "speedup_vs_single_pair_calls": round(ts / td, 3),
                         "bit_identical_to_single_pair_calls": bool(same)}
    return ex["diff_16x40k"]


def vanicp_comparator(api, synth, torch, dev, np):
    """VANICP's monolithic layout (64 KiB per voxel, points copied into
    every occupied and dilated voxel's block) against the segmented layout,
    on the same grid, rings and search schedule: build time, registration
    time, search-kernel time and bytes.  On the paper's fixed 16^3 grid the
    densest voxels overflow their blocks and send queries to the global
    search."""
    log("[bench] VANICP layout comparator")
    out = {}
    for name in ("room_226k", "paper_room_226k"):
        Pw = synth.config(name)
        qd = torch.from_numpy(Pw.q).to(dev)
        pd_ = torch.from_numpy(Pw.p).to(dev)
        paper = name.startswith("paper")
        if paper:
            g = api.build_grid_fixed(qd, Pw.meta["grid_origin"], Pw.voxel, Pw.meta["grid_dims"], Pw.rings)
            kw = {"rmse_eps": Pw.meta["rmse_eps"], "early_stop": True}
        else:
            g = api.build_grid(qd, Pw.voxel, Pw.rings)
            kw = {}
        g.dilate(Pw.rings)
        g.autotune(pd_, searches_per_plan=Pw.iters)

        def avg(fn, reps):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                r = fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps, r

        t_seg_build, _ = avg(lambda: g.rebuild(qd).dilate(Pw.rings), 5)
        t_dir_build, _ = avg(lambda: g.build_direct(65536), 5)
        t_seg, rs = avg(lambda: g.register(pd_, Pw.iters, use_graph=True, **kw), 5)
        t_dir, rd = avg(lambda: g.register(pd_, Pw.iters, use_graph=True, layout="direct", **kw), 5)
        api.prof_reset()
        api.prof_enable(True)
        g.build_direct(65536)
        g.register(pd_, Pw.iters, use_graph=False, **kw)
        g.register(pd_, Pw.iters, use_graph=False, layout="direct", **kw)
        torch.cuda.synchronize()
        api.prof_enable(False)
        kus = {}
        for k in ("nns_local", "nns_direct", "direct_count", "direct_dilate_ring", "direct_replicate"):
            n_l, tot = api.prof_read(k)
            if n_l:
                kus[k + "_us"] = round(1e3 * tot / n_l, 2)
        d = g.describe()
        sched = g.schedule
        g.free()
        ks, kd = int(rs.iters[0]), int(rd.iters[0])
        out[name] = {
            "V": d["V"], "block_bytes": 65536,
            "bytes_vanicp": d["V"] * 65536 + 4 * d["V"],
            "bytes_segmented": d["static_bytes"] + d["dynamic_bytes"],
            "build_ms_segmented": round(t_seg_build * 1e3, 3), "build_ms_vanicp": round(t_dir_build * 1e3, 3),
            "register_ms_segmented": round(t_seg * 1e3, 3), "register_ms_vanicp": round(t_dir * 1e3, 3),
            "iters_segmented": ks, "iters_vanicp": kd,
            "global_searches_iter0_segmented": int(rs.fallbacks[0][0]),
            "global_searches_iter0_vanicp": int(rd.fallbacks[0][0]),
            "final_rmse_segmented": float(rs.rmse[0][ks - 1]), "final_rmse_vanicp": float(rd.rmse[0][kd - 1]),
            "same_pose": bool(np.array_equal(rs.Rt, rd.Rt)), "schedule": sched, **kus}
    return out


def cpu_baseline(P):
    """The CPU oracle as it stands on this host's cores: whole registrations
    (grid, dilation, every iteration) of the three single-pair workloads,
    single-threaded and with Alg. 4's per-query loop on every core the
    process may use (at most 16), median of 3 runs (1 for the room); then the
    headline figure, the room workload on every core, repeated for about
    10 s."""
    import statistics

    import oracle
    from paper_2512_04996_amd import synth
    log("[bench] cpu baseline (oracle)")
    oracle.lib()
    cores = min(16, len(os.sched_getaffinity(0)))
    try:
        cores = min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))
    except ValueError:
        pass
    cores = max(cores, 1)
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    per = {}
    for name, reps in (("sphere_2k", 3), ("bumpy_40k", 3), ("room_226k", 1)):
        W = P if name == P.name else synth.config(name)
        row = {}
        for th in sorted({1, cores}):
            used = oracle.set_threads(th)
            times = []
            for _ in range(reps):
                t0 = time.perf_counter()
                r = oracle.register(W.q, W.p, W.voxel, W.rings, W.iters)
                times.append(time.perf_counter() - t0)
            t = statistics.median(times)
            row[f"threads_{used}"] = {"queries_per_s": round(r.iters * W.m / t, 1),
                                      "icp_iters_per_s": round(r.iters / t, 3), "s_per_registration": round(t, 4)}
        per[name] = row
    used = oracle.set_threads(cores)
    reps = 0
    t0 = time.perf_counter()
    while True:
        r = oracle.register(P.q, P.p, P.voxel, P.rings, P.iters)
        reps += 1
        el = time.perf_counter() - t0
        if el > 10.0 or reps >= 200:
            break
    oracle.set_threads(1)
    return {"value": round(reps * r.iters * P.m / el, 1), "unit": "queries/s", "cores": used, "kind": "oracle",
            "sample": f"{reps} full registrations of {P.name} (grid + dilation + {P.iters} iterations), "
                      f"{el:.1f} s, Alg. 4's per-query loop on {used} threads",
            "icp_iters_per_s": round(reps * r.iters / el, 3), "cpu": cpu,
            "per_workload": per,
            "note": "median of 3 runs for sphere_2k and bumpy_40k, 1 for room_226k; threads_1 is single-threaded"}


if __name__ == "__main__":
    main()
