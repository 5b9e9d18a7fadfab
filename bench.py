"""Benchmark: resident 3DGS training steps on one MI355X.

Workload (one step = the whole hot path over one batch): the aerial scene of
1,000,000 Gaussians (200 blobs, sigma 5 m, over 500 x 500 m), 4 views of
1920x1080 per batch on a 250 m-radius orbit at 150 m altitude; per step
preprocess -> bin/sort -> composite -> loss (0.8 L1 + 0.2 D-SSIM) ->
adjoint with the masked Adam update fused in, all through libtide.so.  Inputs are seeded and
synthetic; targets are rendered once (untimed) from perturbed parameters and
kept in HBM.

Prints one JSON line.  Besides iters/s it reports Gaussian-pixel visits/s
(forward and backward), per-kernel times, the roofline of the dominant kernel
(measured live with HIP events armed through the library's timing hook on
every timed step; the other kernels' times come from a separate untimed pass
with all events armed, since each armed event pair idles the GPU briefly) and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "train iters/s & Gaussian-pixel visits/s fwd+bwd; HBM GB/s vs peak; stall s/iter"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3

# Algorithmic work per visit of the compositing kernels, the byte/flop model
# of the method's per-pixel formulas: about 20 arithmetic operations and one
# exponential per forward visit (offset 2, exponent 8, exp 1, alpha 1,
# transmittance 2, weight 1, colour 6), about 50 and two transcendentals
# (exponential, reciprocal) per backward visit; a transcendental counts as one.
FLOPS_PER_FWD_VISIT = 21
FLOPS_PER_BWD_VISIT = 52
# Kernels bound by HBM: their algorithmic GB/s is reported as a fraction of
# the 8 TB/s peak as well.
HBM_BOUND = ("preprocess", "reduce_pairs", "adjoint", "adam", "adjoint_adam", "loss_fwd", "loss_bwd")
# HBM traffic per launch of the dominant kernel from two rocprofv3 counter
# passes (FETCH_SIZE, WRITE_SIZE) of this benchmark, each scaled by what the
# counter reads for a plain 1 GiB device copy (x1.9999 and x1.0000), and the
# hash of the kernel's sources when they were taken: the figure is reported
# only while the sources are unchanged.
TRAFFIC = {"render_bwd": {"bytes": 3957.3e6, "sources": ["raster_bwd.hip", "raster.h"],
                          "sha256_16": "1620c5990e6483b0"}}
# Executed-instruction view of the dominant kernel from one SQ counter pass
# of this benchmark (profiles/render_aerial1M_sq_instructions.md): VALU
# wave-instructions per launch and the busy cycles per VALU instruction of a
# SIMD (4 cycles is one wave64 instruction back to back on a 16-lane SIMD),
# reported while the kernel's sources are those the counters were taken on.
ISSUE = {"render_bwd": {"valu_wave_instr": 705.6e6, "cycles_per_valu_per_simd": 3.82,
                        "sources": ["raster_bwd.hip", "raster.h"], "sha256_16": TRAFFIC["render_bwd"]["sha256_16"]}}
# The step runs the backward's last stage and the masked Adam update as one
# kernel (adjoint_adam); adjoint and adam are the same two stages as separate
# kernels (gradient stored in between), timed in a pass of their own.
KERNELS = ["preprocess", "compact_vis", "emit", "render_fwd", "loss_fwd", "loss_bwd", "render_bwd",
           "reduce_pairs", "adjoint_adam"]
UNFUSED = ["adjoint", "adam"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="OpenMP threads of the oracle in the CPU baseline (0 = all cores)")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="time only the oracle's iteration (no GPU), e.g. at --cpu-threads 1")
    ap.add_argument("--n-blobs", type=int, default=200)
    ap.add_argument("--per-blob", type=int, default=5000)
    ap.add_argument("--workload", choices=["aerial", "street50m", "city", "city-ablation", "city-budget", "city-order",
                                           "layout"],
                    default="aerial",
                    help="aerial: resident training (default); city: out-of-core street city, exact-only "
                         "streaming against predictor-hinted streaming; city-ablation: the same city "
                         "without differential streaming, without overlap and without the Morton layout; "
                         "city-budget: a binding block budget with persisted and with cold-restarted moments; "
                         "city-order: one pass over a fixed street view set in capture, shuffled and clustered "
                         "travelling-salesperson order; layout: the out-of-core Morton layout build of a "
                         "street city from a table file")
    ap.add_argument("--layout-blocks", type=int, default=477, help="blocks of 65536 for --workload layout")
    ap.add_argument("--layout-run-rows", type=int, default=1 << 22, help="rows per sorted run")
    ap.add_argument("--budget-blocks", type=int, default=160, help="C for --workload city-budget")
    ap.add_argument("--budget-zfar", type=float, default=1000.0, help="z_far for --workload city-budget")
    ap.add_argument("--city-blocks", type=int, default=954, help="blocks of 65536 Gaussians (954 = 1 km^2)")
    ap.add_argument("--city-iters", type=int, default=150)
    ap.add_argument("--city-dir", default="/tmp/tide_city_store")
    ap.add_argument("--city-host-blocks", type=int, default=200)
    ap.add_argument("--city-zfar", type=float, default=150.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, one plain 1 GiB device-to-device copy (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    return ap.parse_args()


def algorithmic_bytes(kernel, n_pidx, n_kept, n_vis, n_inst, n_active, pixels, V):
    """HBM bytes each kernel must move at minimum (one launch)."""
    if kernel == "preprocess":
        return n_pidx * (12 + 4) + n_kept * 224 + n_vis * 64 + (V * n_pidx - n_vis) * 4
    if kernel == "render_fwd":
        return n_inst * (4 + 4 + 48) + pixels * 20
    if kernel == "render_bwd":
        return n_inst * (4 + 4 + 48 + 36) + pixels * 20
    if kernel == "reduce_pairs":
        return n_vis * (4 + 8 + 36) + n_inst * 36
    if kernel == "adjoint":
        return n_active * (236 + 236 + 8) + n_vis * 36
    if kernel == "adam":   # p, m, v read and written, g read
        return n_active * (7 * 236)
    if kernel == "adjoint_adam":   # p, m, v read and written, step read and written, flags
        return n_active * (6 * 236 + 8 + 8) + n_vis * 36
    if kernel in ("loss_fwd",):
        return pixels * 3 * (4 + 4 + 12)
    if kernel in ("loss_bwd",):
        return pixels * 3 * (12 + 8 + 4)
    return 0


def sources_unchanged(t):
    import hashlib
    h = hashlib.sha256()
    for f in t["sources"]:
        with open(os.path.join(ROOT, "paper_2605_20150_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16] == t["sha256_16"]


def measured_traffic(kernel):
    """Counter-measured bytes per launch, or None if the kernel's sources have
    changed since the counters were taken."""
    t = TRAFFIC.get(kernel)
    if t is None:
        return None
    return t["bytes"] if sources_unchanged(t) else None


def measured_issue(kernel):
    """The executed-instruction figures of ISSUE, or None (as for traffic)."""
    t = ISSUE.get(kernel)
    if t is None or not sources_unchanged(t):
        return None
    return {"valu_wave_instr_per_launch": t["valu_wave_instr"],
            "cycles_per_valu_per_simd": t["cycles_per_valu_per_simd"],
            "note": "rocprofv3 SQ_INSTS_VALU and GRBM_GUI_ACTIVE / 8 over 1024 SIMDs; 4 cycles per wave64 "
                    "VALU instruction is back-to-back issue"}


def _oracle_iteration(oracle, th, cm, targets):
    """One whole training iteration of the FP64 oracle; per-stage seconds and
    the forward's visit count."""
    import numpy as np
    t = [time.perf_counter()]
    p = oracle.project(th, cm)
    t.append(time.perf_counter())
    radius = np.where(p["keep"], p["radius"], 0)
    gid, ranges = oracle.bin_sort(p["u"], p["v"], np.float32(p["depth"]).astype(np.float64), radius, p["keep"], cm)
    t.append(time.perf_counter())
    rec = np.concatenate([p["u"][..., None], p["v"][..., None], p["conic"], p["opacity"][..., None], p["rgb"]], -1)
    r = oracle.composite(gid, ranges, rec, cm)
    t.append(time.perf_counter())
    _, dimg = oracle.loss(r["image"], targets)
    t.append(time.perf_counter())
    g = oracle.backward(th, cm, dimg)
    t.append(time.perf_counter())
    z = np.zeros_like(th)
    oracle.adam(th, z, z, np.zeros(th.shape[0], dtype=np.int64), g, p["keep"].any(0).astype(np.uint8))
    t.append(time.perf_counter())
    names = ["project", "bin_sort", "composite", "loss", "backward", "adam"]
    return {k: round(t[i + 1] - t[i], 4) for i, k in enumerate(names)}, float(r["visits"].sum())


def cpu_baseline(theta, cams, targets, threads=0):
    """The FP64 oracle (as it stands), built -O3 -march=native on this host,
    over one whole iteration of the timed workload: the 4 views of batch 0
    through projection, binning, compositing, loss, backward and masked
    Adam, each stage timed.  threads = 0 uses every core the OpenMP runtime
    offers.  Beside it: one thread on a bounded sample (the forward of view
    0), and the tiny scene (1000 Gaussians, one 64x64 view) for a whole
    iteration on all threads and on one."""
    import tempfile

    import numpy as np

    import oracle
    from paper_2605_20150_amd import synth
    from paper_2605_20150_amd.synth import cams_array
    so = os.path.join(tempfile.gettempdir(), f"liboracle_native_{os.getpid()}.so")
    oracle.build(force=True, so=so, native=True)
    oracle.use(so)
    used = oracle.set_threads(threads)
    th = theta.astype(np.float64)
    cm = cams_array(cams)
    stages, visits = _oracle_iteration(oracle, th, cm, targets)
    total = sum(stages.values())
    # one thread: the forward of view 0
    oracle.set_threads(1)
    t0 = time.perf_counter()
    p = oracle.project(th, cm[:1])
    radius = np.where(p["keep"], p["radius"], 0)
    gid, ranges = oracle.bin_sort(p["u"], p["v"], np.float32(p["depth"]).astype(np.float64), radius, p["keep"],
                                  cm[:1])
    rec = np.concatenate([p["u"][..., None], p["v"][..., None], p["conic"], p["opacity"][..., None], p["rgb"]], -1)
    r1 = oracle.composite(gid, ranges, rec, cm[:1])
    t1 = time.perf_counter() - t0
    single = {"cores": 1, "s": round(t1, 3),
              "sample": "the forward (projection, binning, compositing) of view 0 of batch 0",
              "visits_per_s_fwd": float(r1["visits"].sum()) / t1}
    # the tiny scene, all threads and one
    tth, tcams, ttgt = synth.tiny_workload()
    tcm = cams_array(tcams)
    ttarget = oracle.render(ttgt.astype(np.float64), tcm)["image"]
    tiny = {}
    for name, n in (("all_threads", used), ("one_thread", 1)):
        oracle.set_threads(n)
        st, _ = _oracle_iteration(oracle, tth.astype(np.float64), tcm, ttarget)
        tiny[name] = {"iters_per_s": 1.0 / sum(st.values()), "stage_s": st}
    oracle.set_threads(used)
    os.remove(so)
    return {"value": 1.0 / total, "unit": "iters/s", "cores": used, "kind": "oracle", "cpu": cpu_model(),
            "build": "g++ -O3 -march=native -fopenmp -ffp-contract=off (no fast-math)",
            "sample": (f"one whole iteration: the FP64 oracle over all {th.shape[0]} Gaussians and the 4 "
                       f"1920x1080 views of batch 0, {total:.1f} s; the backward recomputes its forward"),
            "stage_s": stages,
            "visits_per_s_fwd": visits / (stages["composite"] + stages["bin_sort"] + stages["project"]),
            "gaussians_per_s_project": th.shape[0] * len(cams) / stages["project"],
            "single_thread": single, "tiny_scene": tiny}


def cpu_model():
    """The host CPU's model name and socket count (from /proc/cpuinfo)."""
    name, sockets = "unknown", set()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name") and name == "unknown":
                    name = line.split(":", 1)[1].strip()
                elif line.startswith("physical id"):
                    sockets.add(line.split(":", 1)[1].strip())
    except OSError:
        pass
    return f"{name}, {max(len(sockets), 1)} socket(s)"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def city_size(args, rec):
    from paper_2605_20150_amd import city as CT
    import math
    free = CT.free_bytes(args.city_dir)
    n_blocks = min(args.city_blocks, int(0.6 * free // rec))
    extent = 1000.0 * math.sqrt(n_blocks / 954.0)
    return n_blocks, extent, free


def ablation_main(args):
    """Sec. 4.4's component ablations on the out-of-core street city, one
    walk, exact culling only: the full method (Alg. 1, transfers overlapped
    with compute), without differential streaming (every block of K_{t+1}
    moves again), without overlap (transfers serialised with compute), and
    without the Morton layout (the same centres in random order, a store of
    its own)."""
    import shutil

    import numpy as np

    from paper_2605_20150_amd import city as CT
    from paper_2605_20150_amd import predictor as P

    B = 65536
    rec = B * (3 * 59 * 4 + 4)
    n_blocks, extent, free = city_size(args, rec)
    z_far = args.city_zfar
    T = args.city_iters
    H = args.city_host_blocks
    log(f"ablation city: {n_blocks} blocks of {B} over {extent:.0f} m, store {n_blocks * rec / 1e9:.1f} GB "
        f"({free / 1e9:.0f} GB free), {T} iterations, host cache {H} blocks")

    def sizes_of(spheres, batches):
        K = spheres.shape[0]
        words = (K + 31) // 32
        return [len(P.bits_to_ids(P.cull_bits(spheres, b, words), K)) for b in batches]

    shutil.rmtree(args.city_dir, ignore_errors=True)
    N, city, spheres, build_m = CT.build_store(args.city_dir, n_blocks, B, 30, extent, log=log)
    batches = CT.walk_batches(city, 34, T + 1, z_far, 1600, 900)
    sizes = sizes_of(spheres, batches)
    capacity = 2 * max(sizes) + 8
    targets = CT.targets_for(batches, 35, 900, 1600)
    runs, digests = {}, {}
    for name, kw in (("full", {}), ("no_tide", dict(no_tide=True)), ("no_overlap", dict(no_overlap=True))):
        log(f"run {name}: capacity {capacity}, |K_t| {min(sizes)}..{max(sizes)}")
        res, dig, _ = CT.run(args.city_dir, N, B, batches, targets, capacity, 8, H, None, log=log, **kw)
        log(f"{name}: {res}")
        runs[name], digests[name] = res, dig
    shutil.rmtree(args.city_dir, ignore_errors=True)

    _, _, spheres_r, build_r = CT.build_store(args.city_dir, n_blocks, B, 30, extent, layout="random", log=log)
    sizes_r = sizes_of(spheres_r, batches)
    cap_r = max(sizes_r) + 8
    log(f"run no_morton: |K_t| {min(sizes_r)}..{max(sizes_r)} of {n_blocks} blocks; at capacity {capacity} "
        f"{'feasible' if max(sizes_r) <= capacity else 'infeasible'}; run at capacity {cap_r}")
    res, dig_r, _ = CT.run(args.city_dir, N, B, batches, targets, cap_r, 8, H, None, log=log)
    log(f"no_morton: {res}")
    shutil.rmtree(args.city_dir, ignore_errors=True)
    res["feasible_at_full_capacity"] = bool(max(sizes_r) <= capacity)
    res["capacity_blocks"] = cap_r
    res["k_t_fraction_of_blocks"] = round(float(np.mean(sizes_r)) / n_blocks, 4)
    runs["no_morton"] = res

    def row(r):
        return dict(iter_ms=round(1e3 / r["iters_per_s"], 2), pcie_GB_per_iter=r["pcie_GB_per_iter"],
                    host_hit_rate=r["host_hit_rate"], stall_s_per_iter=r["stall_s_per_iter"])

    full = runs["full"]
    out = {
        "metric": METRIC, "value": full["iters_per_s"], "unit": "iters/s", "n_gpus": 1, "steps": T, "warmup": 0,
        "ms_per_step": round(1e3 / full["iters_per_s"], 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"component ablations, out-of-core street city, {n_blocks} blocks x {B} Gaussians "
                               f"({N}), batch 4 x 1600x900, {T}-iteration street walk, exact culling",
                   "gaussians": N, "blocks": n_blocks, "extent_m": round(extent, 1), "z_far_m": z_far,
                   "capacity_blocks": capacity, "host_cache_blocks": H, "o_direct": True,
                   "parallelism": "single GPU"},
        "table": {k: row(v) for k, v in runs.items()},
        "runs": runs,
        "identical_images": {k: digests[k] == digests["full"] for k in ("no_tide", "no_overlap")},
        "layout_build_s": {"morton": round(build_m, 1), "random": round(build_r, 1)},
    }
    print(json.dumps(out), flush=True)


def budget_main(args):
    """The paper's default operating point on the out-of-core street city
    (Sec. 3.5): a block budget C below |K_t| (camera-balanced Top-C decides
    what is rendered) with Adam moments persisted through the tiers and with
    moments that live only while a block is resident (cold restart); an
    unbounded run of the same walk for reference.  Reports iteration rate,
    traffic, the rendered fraction of K_t and the churn statistics."""
    import shutil

    import numpy as np

    from paper_2605_20150_amd import city as CT
    from paper_2605_20150_amd import predictor as P

    B = 65536
    rec = B * (3 * 59 * 4 + 4)
    n_blocks, extent, free = city_size(args, rec)
    z_far = args.budget_zfar
    T = args.city_iters
    H = args.city_host_blocks
    C_ = args.budget_blocks
    shutil.rmtree(args.city_dir, ignore_errors=True)
    N, city, spheres, build_s = CT.build_store(args.city_dir, n_blocks, B, 30, extent, log=log)
    batches = CT.walk_batches(city, 34, T + 1, z_far, 1600, 900)
    K = spheres.shape[0]
    words = (K + 31) // 32
    sizes = [len(P.bits_to_ids(P.cull_bits(spheres, b, words), K)) for b in batches]
    targets = CT.targets_for(batches, 35, 900, 1600)
    full_cap = 2 * max(sizes) + 8
    log(f"budget city: {n_blocks} blocks, z_far {z_far} m, |K_t| {min(sizes)}..{max(sizes)} "
        f"(mean {np.mean(sizes):.0f}); budget C = {C_}; unbounded capacity {full_cap}")
    runs = {}
    for name, cap, kw in (("unbounded_persisted", full_cap, {}),
                          ("bounded_persisted", C_, dict(bounded=True)),
                          ("bounded_cold_restart", C_, dict(bounded=True, cold_restart=True))):
        log(f"run {name}: capacity {cap}")
        res, _, losses = CT.run(args.city_dir, N, B, batches, targets, cap, 8, H, None, log=log, **kw)
        res["loss_first10"] = round(float(np.mean(losses[:10])), 5)
        res["loss_last10"] = round(float(np.mean(losses[-10:])), 5)
        log(f"{name}: {res}")
        runs[name] = res
    shutil.rmtree(args.city_dir, ignore_errors=True)
    main = runs["bounded_cold_restart"]
    out = {
        "metric": METRIC, "value": main["iters_per_s"], "unit": "iters/s", "n_gpus": 1, "steps": T, "warmup": 0,
        "ms_per_step": round(1e3 / main["iters_per_s"], 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"binding budget, out-of-core street city, {n_blocks} blocks x {B} Gaussians ({N}), "
                               f"batch 4 x 1600x900, {T}-iteration street walk, z_far {z_far:.0f} m, C = {C_}, "
                               f"cold-restarted moments",
                   "gaussians": N, "blocks": n_blocks, "extent_m": round(extent, 1), "z_far_m": z_far,
                   "capacity_blocks": C_, "host_cache_blocks": H, "o_direct": True, "parallelism": "single GPU"},
        "k_t": {"min": int(min(sizes)), "mean": round(float(np.mean(sizes)), 1), "max": int(max(sizes))},
        "runs": runs,
        "layout_build_s": round(build_s, 1),
    }
    print(json.dumps(out), flush=True)


def order_main(args):
    """View ordering (Sec. 3.5, App. A) on the out-of-core street city: a
    fixed set of 400 street views (ten walks, every fifth pose) trained for
    one pass in batches of 4, in the order the walks captured them, in a
    shuffled order and in the library's clustered travelling-salesperson
    order.  Every view keeps its own target, so the three runs optimise the
    same objective; only the schedule differs.  The capacity is the smallest
    all three orders can run with.  Blocks of 16384 Gaussians and a host
    cache that holds the whole store keep the shuffled run within a few
    minutes."""
    import shutil

    import numpy as np
    import torch

    from paper_2605_20150_amd import city as CT
    from paper_2605_20150_amd import predictor as P
    from paper_2605_20150_amd import synth
    from paper_2605_20150_amd.train import view_order

    B = 16384
    rec = B * (3 * 59 * 4 + 4)
    n_blocks, extent, free = city_size(args, rec)
    z_far = args.city_zfar
    shutil.rmtree(args.city_dir, ignore_errors=True)
    N, city, spheres, build_s = CT.build_store(args.city_dir, n_blocks, B, 30, extent, log=log)
    views = []
    for w in range(10):
        views += synth.street_walk(city, 200, 200 + w, width=1600, height=900, z_far=z_far)[::5]
    n = len(views)
    per_view = CT.targets_for([[v] for v in views], 36, 900, 1600)
    orders = {"capture": np.arange(n), "shuffle": np.random.Generator(np.random.PCG64(9)).permutation(n),
              "tsp": view_order(views, cluster_size=16, dir_weight=10.0)}
    K = spheres.shape[0]
    words = (K + 31) // 32
    batches, sizes = {}, {}
    for name, o in orders.items():
        b = [[views[i] for i in o[4 * t:4 * t + 4]] for t in range(n // 4)]
        batches[name] = (b + [b[0]], [torch.cat([per_view[i] for i in o[4 * t:4 * t + 4]]) for t in range(n // 4)]
                         + [torch.cat([per_view[i] for i in o[0:4]])])
        sizes[name] = [len(P.bits_to_ids(P.cull_bits(spheres, x, words), K)) for x in b]
    # the smallest capacity every order can run with: the shuffled order
    # then churns while the ordered ones keep their working sets
    capacity = max(max(v) for v in sizes.values()) + 8
    log(f"order city: {n_blocks} blocks of {B} over {extent:.0f} m, {n} views, capacity {capacity}, host cache "
        f"{n_blocks} blocks; |K_t| per order: " + ", ".join(f"{k} {np.mean(v):.0f}" for k, v in sizes.items()))
    runs = {}
    for name in ("capture", "shuffle", "tsp"):
        b, tg = batches[name]
        res, _, losses = CT.run(args.city_dir, N, B, b, tg, capacity, 8, n_blocks, None, log=log)
        res["loss_mean"] = round(float(np.mean(losses)), 5)
        res["loss_last_quarter"] = round(float(np.mean(losses[-len(losses) // 4:])), 5)
        res["consecutive_overlap"] = round(float(np.mean(
            [len(set(P.bits_to_ids(P.cull_bits(spheres, b[t], words), K)) &
                 set(P.bits_to_ids(P.cull_bits(spheres, b[t + 1], words), K))) / max(1, sizes[name][t + 1])
             for t in range(len(b) - 2)])), 4)
        log(f"{name}: {res}")
        runs[name] = res
    shutil.rmtree(args.city_dir, ignore_errors=True)
    tsp = runs["tsp"]
    out = {
        "metric": METRIC, "value": tsp["iters_per_s"], "unit": "iters/s", "n_gpus": 1, "steps": n // 4,
        "warmup": 0, "ms_per_step": round(1e3 / tsp["iters_per_s"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"view ordering, out-of-core street city, {n_blocks} blocks x {B} Gaussians ({N}), "
                               f"{n} street views 1600x900 in batches of 4, one pass, clustered TSP order",
                   "gaussians": N, "blocks": n_blocks, "extent_m": round(extent, 1), "z_far_m": z_far,
                   "capacity_blocks": capacity, "host_cache_blocks": n_blocks, "o_direct": True,
                   "parallelism": "single GPU"},
        "table": {k: dict(iter_ms=round(1e3 / v["iters_per_s"], 2), pcie_GB_per_iter=v["pcie_GB_per_iter"],
                          stall_s_per_iter=v["stall_s_per_iter"], consecutive_overlap=v["consecutive_overlap"],
                          loss_mean=v["loss_mean"]) for k, v in runs.items()},
        "runs": runs,
        "layout_build_s": round(build_s, 1),
    }
    print(json.dumps(out), flush=True)


def layout_main(args):
    """The layout build of Sec. 3.3 and 4.1 out of core: a street city's
    table (generation order) on disk, sorted runs of --layout-run-rows rows,
    a k-way merge into the base segment with the block spheres.  Checks two
    blocks against the in-memory Morton order of the same centres."""
    import shutil

    import numpy as np

    from paper_2605_20150_amd import city as CT
    from paper_2605_20150_amd import predictor as P
    from paper_2605_20150_amd.raster import Pool
    from paper_2605_20150_amd.tier import Tier

    B = 65536
    n_blocks = args.layout_blocks
    extent = 1000.0 * (n_blocks / 954.0) ** 0.5
    root = args.city_dir
    shutil.rmtree(root, ignore_errors=True)
    os.makedirs(root)
    table = os.path.join(root, "table.f32")
    N, _, t_table = CT.write_table(table, n_blocks, B, 30, extent, log=log)
    log(f"layout: table of {N} rows ({N * 236 / 1e9:.1f} GB) written in {t_table:.1f} s")
    tier = Tier(os.path.join(root, "store"), N, Pool.empty(1, B, "cpu"), 1, 4, io_threads=1, host_pool=True,
                odirect=True)
    t0 = time.perf_counter()
    tier.layout_build(table, root, args.layout_run_rows)
    t_build = time.perf_counter() - t0
    log(f"layout: built in {t_build:.1f} s")
    # the same order in memory, for two blocks
    th = np.memmap(table, dtype=np.float32, mode="r", shape=(N, 59))
    perm = P.morton_order(np.ascontiguousarray(th[:, :3]))
    same = all(np.array_equal(tier.read_block(k)["params"], th[perm[k * B:(k + 1) * B]].T) for k in (0, n_blocks - 1))
    tier.close()
    del th
    shutil.rmtree(root, ignore_errors=True)
    rate = N / t_build
    out = {
        "metric": METRIC, "value": round(rate / 1e6, 3), "unit": "M Gaussians/s laid out", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": round(1e3 * t_build, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"out-of-core Morton layout build, street city of {N} Gaussians ({n_blocks} blocks "
                               f"x {B}), runs of {args.layout_run_rows} rows, O_DIRECT base segment",
                   "gaussians": N, "blocks": n_blocks, "run_rows": args.layout_run_rows, "parallelism": "host"},
        "table_write_s": round(t_table, 1), "build_s": round(t_build, 1),
        "blocks_match_in_memory_order": bool(same),
    }
    print(json.dumps(out), flush=True)


def city_main(args):
    """Out-of-core street city: the same held-out walk trained from the same
    store with exact-culling-only streaming and with the predictor's hints."""
    import math
    import shutil

    import numpy as np
    import torch

    from paper_2605_20150_amd import city as CT
    from paper_2605_20150_amd import predictor as P

    B = 65536
    rec = B * (3 * 59 * 4 + 4)
    n_blocks, extent, free = city_size(args, rec)
    z_far = args.city_zfar
    log(f"city: {n_blocks} blocks of {B} over {extent:.0f} m, store {n_blocks * rec / 1e9:.1f} GB "
        f"({free / 1e9:.0f} GB free)")
    shutil.rmtree(args.city_dir, ignore_errors=True)
    N, city, spheres, build_s = CT.build_store(args.city_dir, n_blocks, B, 30, extent, log=log)
    predictor, pinfo = CT.train_predictor(spheres, city, z_far, range(100, 116), 400, log=log)
    T = args.city_iters
    batches = CT.walk_batches(city, 34, T + 1, z_far, 1600, 900)
    K = spheres.shape[0]
    words = predictor.words
    sizes = [len(P.bits_to_ids(P.cull_bits(spheres, b, words), K)) for b in batches]
    capacity = 2 * max(sizes) + 8
    # the predictor judged against exact culling on this walk
    X, Y = P.log_pairs(spheres, batches, words)
    mlp = predictor.mlp
    z = torch.cat([mlp.forward(torch.from_numpy(X[i:i + 256]).cuda()).clone() for i in range(0, X.shape[0], 256)])
    bits = mlp.predict_bits(z, predictor.thr).cpu().numpy().view(np.uint32) & P.valid_mask(K, words)[None, :]
    recall, precision = P.recall_precision(bits, Y)
    del z
    targets = CT.targets_for(batches, 35, 900, 1600)
    log(f"walk: {T} iterations, |K_t| {min(sizes)}..{max(sizes)}, capacity {capacity}, host cache "
        f"{args.city_host_blocks} blocks; predictor recall {recall:.4f} precision {precision:.4f}")
    exact, dig_e, loss_e = CT.run(args.city_dir, N, B, batches, targets, capacity, 8, args.city_host_blocks,
                                  None, log=log)
    log(f"exact-only: {exact}")
    pred, dig_p, loss_p = CT.run(args.city_dir, N, B, batches, targets, capacity, 8, args.city_host_blocks,
                                 predictor, log=log)
    log(f"with predictor: {pred}")
    shutil.rmtree(args.city_dir, ignore_errors=True)
    pred["hinted_blocks"] = predictor.hinted
    pred["wasted_prefetch_GB"] = round((pred["prefetch_issued"] - pred["prefetch_used"]) * rec / 1e9, 3)
    out = {
        "metric": METRIC, "value": pred["iters_per_s"], "unit": "iters/s", "n_gpus": 1, "steps": T, "warmup": 0,
        "ms_per_step": round(1e3 / pred["iters_per_s"], 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"out-of-core street city, {n_blocks} blocks x {B} Gaussians ({N}), "
                               f"batch 4 x 1600x900, {T}-iteration street walk, predictor-hinted streaming",
                   "gaussians": N, "blocks": n_blocks, "extent_m": round(extent, 1), "z_far_m": z_far,
                   "capacity_blocks": capacity, "host_cache_blocks": args.city_host_blocks, "o_direct": True,
                   "parallelism": "single GPU"},
        "stall_s_per_iter": pred["stall_s_per_iter"],
        "exact_only": exact, "with_predictor": pred,
        "predictor": dict(pinfo, walk_recall=round(recall, 4), walk_precision=round(precision, 4)),
        "identical_images": dig_e == dig_p, "identical_losses": loss_e == loss_p,
        "layout_build_s": round(build_s, 1),
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; the multi-GPU path is a design "
                          "(block ownership + all-to-all of projected records), not an executable"}))
        sys.exit(2)
    if args.workload == "city":
        return city_main(args)
    if args.workload == "city-ablation":
        return ablation_main(args)
    if args.workload == "city-budget":
        return budget_main(args)
    if args.workload == "city-order":
        return order_main(args)
    if args.workload == "layout":
        return layout_main(args)
    if args.workload == "street50m":
        return street_main(args)
    import numpy as np

    from paper_2605_20150_amd import synth

    theta, cams = synth.aerial_workload(n_blobs=args.n_blobs, per_blob=args.per_blob)
    V = 4
    if args.cpu_baseline_only:
        # the oracle's time does not depend on the target's content
        tg = np.zeros((V, 3, cams[0].height, cams[0].width))
        print(json.dumps({"cpu_baseline": cpu_baseline(theta, cams[:V], tg, args.cpu_threads)}), flush=True)
        return
    resident_run(args, theta, cams, 1920, 1080,
                 {"workload": f"aerial resident training, {theta.shape[0] // 1000000}M Gaussians, batch 4 x 1920x1080"},
                 with_cpu_baseline=not args.no_cpu_baseline)


def street_main(args):
    """The 50M-Gaussian scale case resident in HBM: the aerial blob recipe
    over 2 x 2 km (3200 blobs of 15 625 Gaussians, sigma 5 m, heights U(0, 40)
    m, seed 20), blobs laid out in the library's Morton order of their
    centres, trained from a street-level walk (1.7 m eye height along a
    street at y = 7 m, 1 m per pose, looking along the street, 1600x900,
    horizontal fov 60 deg, z_far 1000 m), batches of 4 consecutive poses."""
    import numpy as np

    from paper_2605_20150_amd import predictor as P
    from paper_2605_20150_amd import synth

    centres = synth.blob_centres(3200, 1000.0, (0.0, 40.0), 20)
    order = P.morton_order(centres.astype(np.float32))
    theta = synth.blob_scene_parallel(3200, 15625, 1000.0, (0.0, 40.0), 5.0, 20, order=order)
    f = synth.focal_for_hfov(1600, 60)
    n_poses = 4 * (args.warmup + args.steps)
    cams = [synth.look_at((-400.0 + p, 7.0, 1.7), (-300.0 + p, 7.0, 1.7), (0, 0, 1), 1600, 900, f, z_far=1000.0)
            for p in range(n_poses)]
    resident_run(args, theta, cams, 1600, 900,
                 {"workload": "street-level resident training, 50M Gaussians over 2 x 2 km, batch 4 x 1600x900"},
                 with_cpu_baseline=False)


def resident_run(args, theta, cams, W, H, workload, with_cpu_baseline):
    """Resident training steps (forward, loss, backward, masked Adam) over
    batches of 4 consecutive views; prints the JSON line."""
    import numpy as np
    import torch

    from paper_2605_20150_amd import synth
    from paper_2605_20150_amd import _lib as L
    from paper_2605_20150_amd.raster import LR59, Pool, Rasterizer, adam_cfg

    N = theta.shape[0]
    V = 4
    n_batches = len(cams) // V
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.device("cuda:0")
    rast = Rasterizer(dev)
    lib = L.load()
    B = 65536
    # targets: rendered once from perturbed parameters (seed 11), kept in HBM
    tpool = Pool.from_dense(torch.tensor(synth.perturbed(theta, 0.05, 11), device=dev), B)
    used = min(n_batches, args.warmup + args.steps)
    targets = []
    for b in range(used):
        _, _, fr = rast.forward(tpool, cams[V * b: V * b + V])
        targets.append(fr.image.clone())
    del tpool
    torch.cuda.synchronize()
    pool = Pool.from_dense(torch.tensor(theta, device=dev), B)
    cfg = adam_cfg(LR59, kappa=1.32)
    n_blocks = pool.n_slots
    spheres = torch.zeros((n_blocks, 4), dtype=torch.float32, device=dev)
    dirty = torch.zeros((n_blocks,), dtype=torch.uint8, device=dev)
    grad = torch.empty((59, pool.n_pidx), dtype=torch.float32, device=dev)
    cam_batches = [cams[V * (b % used): V * (b % used) + V] for b in range(used)]

    def step(b, stats=None, fused=True):
        cb = cam_batches[b % used]
        proj, bins, fr = rast.forward(pool, cb)
        loss, dimg = rast.loss(fr.image, targets[b % used])
        if fused:
            rast.backward_adam(pool, cb, proj, bins, fr, dimg, cfg, spheres, dirty)
        else:
            rast.backward(pool, cb, proj, bins, fr, dimg, grad=grad)
            rast.adam(pool, proj, grad, cfg, spheres, dirty)
        if stats is not None:
            # counters the kernels keep themselves: no extra reductions in the
            # timed region (the Gaussians kept by some camera are the active set)
            stats.append((bins.n_vis, bins.n_inst, proj.n_active.clone(), fr.visits, loss))

    # per-kernel HIP events armed on the launch stream; created (and
    # materialised by one record) before any measured pass
    P = min(args.steps, 10)
    ev = {k: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(P)] for k in KERNELS + UNFUSED}
    handles = {k: [(C_void(a), C_void(z)) for a, z in ev[k]] for k in KERNELS + UNFUSED}
    names = {k: k.encode() for k in KERNELS + UNFUSED}
    # warm-up steps run what the measured passes run (events armed, the
    # per-step statistics gathered), so first-use allocations happen here
    for b in range(args.warmup):
        for k in KERNELS:
            lib.tide_timer_arm(names[k], handles[k][0][0], handles[k][0][1])
        step(b, [])
    for k in UNFUSED:
        lib.tide_timer_arm(names[k], handles[k][0][0], handles[k][0][1])
    step(0, [], fused=False)
    torch.cuda.synchronize()

    # per-kernel times: P steps (the first P batches of the timed region)
    # with every kernel's events armed.  This pass is not timed: each armed
    # event pair leaves the GPU idle for a few microseconds, about 0.1 ms per
    # step over all ten kernels.
    for s in range(P):
        for k in KERNELS:
            lib.tide_timer_arm(names[k], handles[k][s][0], handles[k][s][1])
        step(args.warmup + s, [])
    # the same steps with the gradient stored between the backward and Adam
    for s in range(P):
        for k in UNFUSED:
            lib.tide_timer_arm(names[k], handles[k][s][0], handles[k][s][1])
        step(args.warmup + s, [], fused=False)
    torch.cuda.synchronize()
    lib.tide_timer_clear()
    kern_ms = {k: float(np.mean([a.elapsed_time(z) for a, z in ev[k]])) for k in KERNELS + UNFUSED}
    dominant = max(KERNELS, key=lambda k: kern_ms[k])
    ev_dom = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    h_dom = [(C_void(a), C_void(z)) for a, z in ev_dom]
    torch.cuda.synchronize()

    # step boundaries, for the median step time (one event record per step)
    ev_step = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    for e in ev_step:
        e.record()
    torch.cuda.synchronize()

    # timed region: K steps; only the dominant kernel's events are armed, and
    # its roofline is taken from them
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        lib.tide_timer_arm(names[dominant], h_dom[s][0], h_dom[s][1])
        ev_step[s].record()
        step(args.warmup + s, stats)
    ev_step[args.steps].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.tide_timer_clear()
    wall = t1 - t0
    dom_ms = float(np.mean([a.elapsed_time(z) for a, z in ev_dom]))
    kern_ms[dominant] = dom_ms
    step_ms = [ev_step[s].elapsed_time(ev_step[s + 1]) for s in range(args.steps)]

    n_vis = np.mean([s[0] for s in stats])
    n_inst = np.mean([s[1] for s in stats])
    n_active = np.mean([int(s[2].item()) for s in stats])
    fwd_visits = np.mean([int(s[3][0].sum().item()) for s in stats])
    bwd_visits = np.mean([int(s[3][1].sum().item()) for s in stats])
    n_kept = n_active
    pixels = V * W * H
    iters = args.steps / wall

    kernels = {}
    for k in KERNELS + UNFUSED:
        by = algorithmic_bytes(k, pool.n_pidx, n_kept, n_vis, n_inst, n_active, pixels, V)
        kernels[k] = {"ms": round(kern_ms[k], 4),
                      "alg_GBps": round(by / (kern_ms[k] * 1e-3) / 1e9, 1) if kern_ms[k] > 0 else None}
        if k in HBM_BOUND and kern_ms[k] > 0:
            kernels[k]["hbm_frac"] = round(by / (kern_ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)
    fwd_tflops = fwd_visits * FLOPS_PER_FWD_VISIT / (kern_ms["render_fwd"] * 1e-3) / 1e12
    bwd_tflops = bwd_visits * FLOPS_PER_BWD_VISIT / (kern_ms["render_bwd"] * 1e-3) / 1e12
    kernels["render_fwd"]["alg_TFLOPs"] = round(fwd_tflops, 2)
    kernels["render_bwd"]["alg_TFLOPs"] = round(bwd_tflops, 2)
    if dominant in ("render_fwd", "render_bwd"):
        ach = fwd_tflops if dominant == "render_fwd" else bwd_tflops
        roof = {"kernel": dominant, "bound": "alu", "achieved": round(ach, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / FP32_VECTOR_PEAK_TFLOPS, 4),
                "traffic": measured_traffic(dominant), "executed": measured_issue(dominant),
                "note": (f"algorithmic: {FLOPS_PER_BWD_VISIT if dominant == 'render_bwd' else FLOPS_PER_FWD_VISIT} "
                         f"operations per visit (entries up to each pixel's last contributor for the "
                         f"backward, entries evaluated for the forward) over the kernel's own launch time")}
    else:
        by = algorithmic_bytes(dominant, pool.n_pidx, n_kept, n_vis, n_inst, n_active, pixels, V)
        ach = by / (kern_ms[dominant] * 1e-3) / 1e9
        roof = {"kernel": dominant, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dominant)}

    out = {
        "metric": METRIC, "value": round(iters, 3), "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * wall / args.steps, 3),
        "iters_per_s_median": round(1e3 / float(np.median(step_ms)), 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": dict(workload, gaussians=N, views_per_step=V, width=W, height=H, block_rows=B,
                       parallelism="single GPU"),
        "visits_per_s": {"fwd": round(fwd_visits / (kern_ms["render_fwd"] * 1e-3), 1),
                         "bwd": round(bwd_visits / (kern_ms["render_bwd"] * 1e-3), 1),
                         "fwd_plus_bwd": round((fwd_visits + bwd_visits) /
                                               ((kern_ms["render_fwd"] + kern_ms["render_bwd"]) * 1e-3), 1)},
        "per_step": {"visible_pairs": int(n_vis), "instances": int(n_inst), "active_rows": int(n_active),
                     "fwd_visits": int(fwd_visits), "bwd_visits": int(bwd_visits)},
        "kernels": kernels,
        "kernels_note": f"ms of the dominant kernel from its events in the timed region; the others from an "
                        f"untimed pass of {P} steps with every kernel's events armed; adjoint and adam from "
                        f"{P} further steps that store the gradient between the backward and the update "
                        f"(the timed steps run them as one kernel, adjoint_adam)",
        "stall_s_per_iter": None,
        "roofline": roof,
    }
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if with_cpu_baseline:
        tg0 = targets[0].double().cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(theta, cams[:V], tg0, args.cpu_threads)
    print(json.dumps(out), flush=True)


def C_void(event):
    """Raw hipEvent_t of a torch event (recorded once so that it exists)."""
    import ctypes
    event.record()
    return ctypes.c_void_p(event.cuda_event)


if __name__ == "__main__":
    main()
