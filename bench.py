"""Benchmark of the photon-mapping hot path on one MI355X.

Default workload (the traversal-only configuration): 2^20 random triangles
(centroids uniform in the unit cube, lognormal(-5, 0.5) vertex offsets),
SAH-binned BVH (32 bins, <= 4 triangles per leaf), 1920x1080 coherent pinhole
rays plus 2^21 incoherent rays.  One step = closest-hit traversal of all
4,170,752 rays: two trace calls, inputs resident in HBM.  The camera batch is
traced as packets, one wavefront per 8x8 pixel tile (--coherent), the
incoherent batch after bucketing by (origin cell, link set) with postponed
leaf tests (--incoherent); every
option listed in KERNEL_VARIANTS gives identical results and is also timed.
The JSON line reports Mrays/s, the traversal's algorithmic-bytes roofline,
the CPU oracle timed on the host, the SPPM iteration on the 250k-triangle
procedural scene, the adjoint-to-forward time ratio and the batched renderer.

python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--no-sppm] [--no-adjoint] [--no-batch]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
TRACE_SOURCES = ["paper_1505_06022_amd/csrc/pm_device.h", "paper_1505_06022_amd/csrc/trace.hip",
                 "paper_1505_06022_amd/csrc/bvh_build.cpp"]


# Traversal options compared by the bench (names usable with --coherent/--incoherent)
KERNEL_VARIANTS = (
    ("per_ray", dict(kernel=1)), ("per_ray_reorder1", dict(kernel=1, reorder=1)),
    ("per_ray_reorder2", dict(kernel=1, reorder=2)), ("paired", dict(kernel=3)),
    ("paired_reorder1", dict(kernel=3, reorder=1)), ("persistent_refill16", dict(kernel=2, refill=16)),
    ("postponed_late0", dict(kernel=4, refill=0)), ("postponed_late4", dict(kernel=4, refill=4)),
    ("postponed_late16", dict(kernel=4, refill=16)), ("postponed_late0_reorder1", dict(kernel=4, reorder=1)),
    ("postponed_late4_reorder1", dict(kernel=4, refill=4, reorder=1)),
    ("postponed_late16_reorder1", dict(kernel=4, refill=16, reorder=1)),
    ("per_ray_block64", dict(kernel=1, block=64)), ("per_ray_block128", dict(kernel=1, block=128)),
    ("per_ray_reorder1_block64", dict(kernel=1, reorder=1, block=64)),
    ("per_ray_reorder1_block128", dict(kernel=1, reorder=1, block=128)),
    ("postponed_late16_block64", dict(kernel=4, refill=16, block=64)),
    ("postponed_late16_reorder1_block64", dict(kernel=4, refill=16, reorder=1, block=64)),
    ("paired_reorder1_block64", dict(kernel=3, reorder=1, block=64)),
    ("two_rays", dict(kernel=5)), ("two_rays_block64", dict(kernel=5, block=64)),
    ("two_rays_block128", dict(kernel=5, block=128)), ("two_rays_reorder1", dict(kernel=5, reorder=1)),
    ("two_rays_reorder1_block64", dict(kernel=5, reorder=1, block=64)),
    ("two_rays_reorder1_block128", dict(kernel=5, reorder=1, block=128)),
    ("two_rays_reorder2_block64", dict(kernel=5, reorder=2, block=64)),
    ("persistent_reorder1_refill4", dict(kernel=2, refill=4, reorder=1)),
    ("persistent_reorder1_refill16", dict(kernel=2, refill=16, reorder=1)),
    ("persistent_reorder1_refill32", dict(kernel=2, refill=32, reorder=1)),
    ("per_ray_tiles_block64", dict(kernel=1, block=64, tile_width="image")),
    ("packet_block64", dict(kernel=6, block=64)), ("packet_tiles", dict(kernel=6, tile_width="image")),
    ("packet_tiles_block64", dict(kernel=6, block=64, tile_width="image")),
    ("packet_reorder1_block64", dict(kernel=6, block=64, reorder=1)),
    ("postponed_late8_reorder1_block64", dict(kernel=4, refill=8, reorder=1, block=64)),
    ("postponed_late24_reorder1_block64", dict(kernel=4, refill=24, reorder=1, block=64)),
    ("postponed_late32_reorder1_block64", dict(kernel=4, refill=32, reorder=1, block=64)),
    ("postponed_late16_reorder2_block64", dict(kernel=4, refill=16, reorder=2, block=64)),
    ("postponed_late16_reorder1_block128", dict(kernel=4, refill=16, reorder=1, block=128)),
    ("slices_late32_reorder1_block64", dict(kernel=7, refill=32, reorder=1, block=64)),
    ("slices256_late32_reorder1_block64", dict(kernel=7, refill=32, reorder=1, block=64, slice_rays=256)))

IMAGE_WIDTH = 1920   # of the camera batch


def _kw_for(kw: dict, batch: int) -> dict:
    """Trace options for one batch: tile_width "image" takes the camera batch in
    8x8 pixel tiles and does not apply to the incoherent batch."""
    d = dict(kw)
    if d.get("tile_width") == "image":
        d["tile_width"] = IMAGE_WIDTH if batch == 0 else 0
    return d


def measured_traffic():
    """HBM bytes per traversal call (both batches) from the committed counter
    record, or None when the traversal sources changed since the counters were
    taken."""
    import hashlib
    h = hashlib.sha256()
    for f in TRACE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    try:
        with open(os.path.join(ROOT, "profiles", "k_trace_pmc_soup1M.md")) as fh:
            line = next(ln for ln in fh if ln.startswith("traffic-record:"))
    except (OSError, StopIteration):
        return None
    rec = json.loads(line.split(":", 1)[1])
    if rec["sources_sha256_16"] != h.hexdigest()[:16]:
        return None
    # the record lists each batch; one timed call traces all of them
    return 1024.0 * (rec["fetch_factor"] * sum(rec["fetch_kib"]) + rec["write_factor"] * sum(rec["write_kib"]))


def measured_sppm_traffic():
    """L2-to-memory bytes per SPPM stage (read + written, per iteration) from the
    committed counter record, or None when the SPPM sources changed since the
    counters were taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "sppm_pmc_procedural250k.md")) as fh:
            line = next(ln for ln in fh if ln.startswith("traffic-record:"))
    except (OSError, StopIteration):
        return None
    rec = json.loads(line.split(":", 1)[1])
    h = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if rec["sources_sha256_16"] != h.hexdigest()[:16]:
        return None
    return {st: 1024.0 * (rec["fetch_factor"] * rec["fetch_kib"][st] + rec["write_factor"] * rec["write_kib"][st])
            for st in rec["fetch_kib"]}


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sppm", action="store_true")
    ap.add_argument("--sppm-iters", type=int, default=16)
    ap.add_argument("--adjoint-iters", type=int, default=8)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--batch-iters", type=int, default=16)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the comparisons of traversal kernels and of SPPM schedules")
    ap.add_argument("--only-sppm", action="store_true",
                    help="run only the SPPM iteration leg and print it (profiling runs of its kernels)")
    names = [k for k, _ in KERNEL_VARIANTS]
    ap.add_argument("--coherent", default="packet_tiles_block64", choices=names,
                    help="traversal options of the camera batch")
    ap.add_argument("--incoherent", default="postponed_late32_reorder1_block64", choices=names,
                    help="traversal options of the incoherent batch")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run the library's 1 GiB stream copy (calibrates HBM byte counters)")
    ap.add_argument("--split-alpha", type=float, default=None,
                    help="spatial-split threshold of the traversal BVH (default: the soup's, 1e-4; 0 = none)")
    ap.add_argument("--trav-cost", type=float, default=None,
                    help="SAH node-visit cost of the traversal BVH (default: the soup's, 2)")
    return ap.parse_args()


def _cpu_threads() -> int:
    """Host threads for the oracle: the cores this process may run on, capped by
    OMP_NUM_THREADS where the machine sets it (a GPU host's share per GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS", "")
    if cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def _host_info() -> dict:
    """nproc, the cores this process may use, and the CPU model (lscpu, else /proc/cpuinfo)."""
    import subprocess
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        model = next((ln.split(":", 1)[1].strip() for ln in out.splitlines() if ln.startswith("Model name")), None)
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None:
        try:
            with open("/proc/cpuinfo") as fh:
                model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
        except OSError:
            pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = None
    return {"nproc": os.cpu_count(), "affinity_cores": aff, "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
            "cpu_model": model}


def _time_multi(torch, api, bvh, multi, reps=20):
    """Mean ms of one pm_trace_rays_multi call over `reps` calls after a short warm-up."""
    stream = torch.cuda.current_stream()
    for _ in range(5):
        api.trace_rays_multi(bvh, multi)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e[0].record(stream)
    for _ in range(reps):
        api.trace_rays_multi(bvh, multi)
    e[1].record(stream)
    torch.cuda.synchronize()
    return e[0].elapsed_time(e[1]) / reps


def traversal_bench(args, torch, api, scenes):
    sc, coh, inc = scenes.soup_workload()
    split_alpha = scenes.SOUP_SPLIT_ALPHA if args.split_alpha is None else args.split_alpha
    trav_cost = scenes.SOUP_TRAV_COST if args.trav_cost is None else args.trav_cost
    bvh = api.build_bvh(sc.verts, sc.tri_mat, split_alpha=split_alpha, trav_cost=trav_cost)
    info = bvh.info()
    dev = "cuda"
    rc = torch.from_numpy(coh).to(dev)
    ri = torch.from_numpy(inc).to(dev)
    batches = [rc, ri]
    # camera rays are traced in pixel order; the incoherent batch is first
    # bucketed by (origin cell, link set) -- an option of the trace call
    table = dict(KERNEL_VARIANTS)
    trace_kw = [_kw_for(table[args.coherent], 0), _kw_for(table[args.incoherent], 1)]
    outs = [(torch.empty(len(r), dtype=torch.int32, device=dev), torch.empty(len(r), dtype=torch.float32, device=dev))
            for r in batches]
    n_rays = sum(len(r) for r in batches)

    # traversal statistics (box and triangle tests per ray), outside the timed region
    per_batch = []
    for r in batches:
        cnt = torch.zeros((len(r), 2), dtype=torch.int32, device=dev)
        api.trace_rays(bvh, r, counters=cnt)
        c = cnt.to(torch.float64).sum(0).cpu().numpy()
        per_batch.append((c[0], c[1], len(r)))
    torch.cuda.synchronize()
    # per ray: 32 B ray + 8 B result + 16 B per node visited + 48 B per triangle tested
    alg_bytes = sum(40.0 * n + 16.0 * vn + 48.0 * vt for vn, vt, n in per_batch)

    # one step = one pm_trace_rays_multi call: the incoherent batch is bucketed, then one launch walks it
    # and, in its last workgroups, the camera batch's 8x8 pixel tiles
    stream = torch.cuda.current_stream()
    multi = [dict(rays=batches[b], hit=outs[b][0], t=outs[b][1], **trace_kw[b]) for b in (1, 0)]
    prewarm_steps = _prewarm(torch, lambda: api.trace_rays_multi(bvh, multi))
    for _ in range(args.warmup):
        api.trace_rays_multi(bvh, multi)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s in range(args.steps):
        ev[s][0].record(stream)
        api.trace_rays_multi(bvh, multi)
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = np.asarray([ev[s][0].elapsed_time(ev[s][1]) for s in range(args.steps)])
    step_ms = wall * 1e3 / args.steps
    # each batch alone, one call after the other (per-batch rates; not part of the timed steps)
    batch_ms = np.zeros(len(batches))
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2 * len(batches))]
    for rep in range(6):
        for b, (r, (h, t), kw) in enumerate(zip(batches, outs, trace_kw)):
            e[2 * b].record(stream)
            api.trace_rays(bvh, r, h, t, **kw)
            e[2 * b + 1].record(stream)
        torch.cuda.synchronize()
        if rep:
            batch_ms += [e[2 * b].elapsed_time(e[2 * b + 1]) for b in range(len(batches))]
    batch_ms /= 5
    # the other traversal kernels, for comparison (not part of the timed steps)
    variants = {}
    for name, kw in () if args.no_variants else KERNEL_VARIANTS:
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2 * len(batches))]
        ms = np.zeros(len(batches))
        for rep in range(4):
            for b, (r, (h, t)) in enumerate(zip(batches, outs)):
                e[2 * b].record(stream)
                api.trace_rays(bvh, r, h, t, **_kw_for(kw, b))
                e[2 * b + 1].record(stream)
            torch.cuda.synchronize()
            if rep:
                ms += [e[2 * b].elapsed_time(e[2 * b + 1]) for b in range(len(batches))]
        ms /= 3
        variants[name] = {"coherent_mrays_s": round(len(rc) / ms[0] / 1e3, 1),
                          "incoherent_mrays_s": round(len(ri) / ms[1] / 1e3, 1)}
    # the paper's TBVH comparison: every ray walks one link set (a single threaded BVH),
    # with the timed kernel options
    tbvh = {}
    if not args.no_variants:
        for ls in range(6):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(2 * len(batches))]
            ms = np.zeros(len(batches))
            for rep in range(4):
                for b, (r, (h, t), kw) in enumerate(zip(batches, outs, trace_kw)):
                    e[2 * b].record(stream)
                    api.trace_rays(bvh, r, h, t, link_set=ls, **kw)
                    e[2 * b + 1].record(stream)
                torch.cuda.synchronize()
                if rep:
                    ms += [e[2 * b].elapsed_time(e[2 * b + 1]) for b in range(len(batches))]
            ms /= 3
            tbvh[f"link_set_{ls}"] = {"coherent_mrays_s": round(len(rc) / ms[0] / 1e3, 1),
                                      "incoherent_mrays_s": round(len(ri) / ms[1] / 1e3, 1),
                                      "mrays_s": round((len(rc) + len(ri)) / ms.sum() / 1e3, 1)}
    # the GPU linear-BVH builder: build time and traversal rate with the timed options
    lbvh = None
    if not args.no_variants:
        for _ in range(2):   # the first build also loads the sort kernels
            t_b = time.perf_counter()
            lb = api.build_bvh(sc.verts, sc.tri_mat, builder=api.BUILD_GPU_LBVH)
            torch.cuda.synchronize()
            wall_ms = (time.perf_counter() - t_b) * 1e3
            if _ == 0:
                lb.destroy()
        linf = lb.info()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2 * len(batches))]
        ms = np.zeros(len(batches))
        for rep in range(4):
            for b, (r, (h, t), kw) in enumerate(zip(batches, outs, trace_kw)):
                e[2 * b].record(stream)
                api.trace_rays(lb, r, h, t, **kw)
                e[2 * b + 1].record(stream)
            torch.cuda.synchronize()
            if rep:
                ms += [e[2 * b].elapsed_time(e[2 * b + 1]) for b in range(len(batches))]
        ms /= 3
        lbvh = {"build_ms_wall": round(wall_ms, 1), "n_nodes": linf["n_nodes"], "depth": linf["depth"],
                "sah_cost": round(linf["sah_cost"], 1), "host_sah_build_ms": round(info["build_ms"], 1),
                "coherent_mrays_s": round(len(rc) / ms[0] / 1e3, 1),
                "incoherent_mrays_s": round(len(ri) / ms[1] / 1e3, 1),
                "mrays_s": round((len(rc) + len(ri)) / ms.sum() / 1e3, 1)}
        lb.destroy()
    if not args.no_variants:
        # spatial splits and node-visit cost: BVH size, build time and the timed call's rate
        spl = {}
        for a, tc in ((0.0, 1.0), (0.0, 2.0), (1e-3, 1.0), (1e-4, 1.0), (1e-3, 1.5)):
            if (a, tc) == (split_alpha, trav_cost):
                continue
            t_b = time.perf_counter()
            bv = api.build_bvh(sc.verts, sc.tri_mat, split_alpha=a, trav_cost=tc)
            wall_ms = (time.perf_counter() - t_b) * 1e3
            inf = bv.info()
            ms = _time_multi(torch, api, bv, multi)
            spl[f"split_alpha_{a:g}_trav_cost_{tc:g}"] = {"n_refs": inf["n_refs"], "n_nodes": inf["n_nodes"],
                                         "device_mb": round(inf["device_bytes"] / 1e6, 1),
                                         "sah_cost": round(inf["sah_cost"], 1), "build_ms_wall": round(wall_ms, 1),
                                         "step_ms": round(ms, 4), "mrays_s": round(n_rays / ms / 1e3, 1)}
            bv.destroy()
        variants["spatial_splits"] = spl
    avg_launch_ms = kern_ms.mean()
    per_launch_bytes = alg_bytes   # one call traces both batches
    achieved = per_launch_bytes / (avg_launch_ms * 1e-3) / 1e9
    hit_frac = float((outs[0][0] >= 0).float().mean().item())
    return dict(
        n_rays=n_rays, step_ms=step_ms, kern_ms=kern_ms, batch_ms=batch_ms, info=info, per_batch=per_batch,
        achieved=achieved, per_launch_bytes=per_launch_bytes, hit_frac=hit_frac, variants=variants, tbvh=tbvh,
        lbvh=lbvh, prewarm_steps=prewarm_steps, split_alpha=split_alpha, trav_cost=trav_cost,
        coherent_mrays=len(rc) / (batch_ms[0] * 1e-3) / 1e6,
        incoherent_mrays=len(ri) / (batch_ms[1] * 1e-3) / 1e6,
        scene=sc, rays=(coh, inc),
    )


def sppm_roofline(api, sc, p_kw, bvh, iters=4):
    """Per-stage algorithmic-bytes roofline of the SPPM iteration.  One handle
    counts the work (PM_PROFILE_COUNT: rays, box and triangle tests, stored
    photons, buckets and photons of the range query), another times the stages
    with HIP events on the streams they run on (PM_PROFILE_TIME); both run
    `iters` iterations after two warm-up ones.  Bytes per unit:
      eye pass + R_max  per eye ray 32 B ray + 8 B result + 16 B per box test
                        + 48 B per triangle test; per pixel 32 B hit point
                        written, 16 B of D read and written, 12 B for R_max
      photon pass       the same per photon ray, + 32 B per stored photon
      hashed grid       per stored photon: count 16 B read + 4 B atomic + 8 B
                        (bucket, rank) written; scatter 8 + 32 + 4 B read and
                        32 B written; per bucket 8 B (scan)
      range query       per pixel 16 B hit-point normal read + 12 B (M, flux)
                        written; per hit point 16 B position + 8 B radius; 8 B
                        per bucket visited; 16 B per photon examined and 16 B
                        more per photon accepted (a lower bound: a photon inside
                        the disc that faces away is read but not counted)
      update            per pixel 8 B (M, hit-point flag); per hit point 32 B
                        read and 24 B written (an upper bound: hit points with
                        M = 0 are skipped)"""
    res = {}
    for flag in (api.PROFILE_COUNT, api.PROFILE_TIME):
        h = api.Sppm(sc, api.sppm_params(profile=flag, **p_kw), bvh=bvh)
        h.iterate(2)
        h.stats(reset=True)
        h.iterate(iters)
        h.status()
        res[flag] = h.stats()
        h.destroy()
    c, t = res[api.PROFILE_COUNT], res[api.PROFILE_TIME]
    nc, nt = float(c["counted_iterations"]), float(t["timed_iterations"])
    P = sc.camera.width * sc.camera.height
    bits = 12
    while bits < 24 and (1 << bits) < 4 * p_kw["n_photons"]:
        bits += 1
    T = 1 << bits
    q = {k: v / nc for k, v in c.items() if k not in ("counted_iterations", "timed_iterations") and not k.startswith("ms_")}

    def rays(prefix):
        return 40.0 * q[prefix + "_rays"] + 16.0 * q[prefix + "_box_tests"] + 48.0 * q[prefix + "_tri_tests"]

    stages = {
        "eye": (rays("eye") + 60.0 * P, t["ms_eye"] / nt),
        "photon": (rays("photon") + 32.0 * q["photons_stored"], t["ms_photon"] / nt),
        "grid": (104.0 * q["photons_stored"] + 8.0 * T, t["ms_grid"] / nt),
        "gather": (28.0 * P + 24.0 * q["gather_hit_points"] + 8.0 * q["gather_buckets"] +
                   16.0 * q["gather_examined"] + 16.0 * q["gather_accepted"], t["ms_gather"] / nt),
        "update": (8.0 * P + 56.0 * q["gather_hit_points"], t["ms_update"] / nt),
    }
    traffic = measured_sppm_traffic()
    out = {}
    for name, (b, ms) in stages.items():
        gbs = b / (ms * 1e-3) / 1e9
        out[name] = {"bytes": round(b), "ms": round(ms, 4), "GBps": round(gbs, 1),
                     "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": round(traffic[name]) if traffic else None}
    counts = {k: round(v, 1) for k, v in q.items()}
    per_unit = {"eye_rays_per_pixel": round(q["eye_rays"] / P, 3),
                "boxes_per_photon_ray": round(q["photon_box_tests"] / q["photon_rays"], 2),
                "tris_per_photon_ray": round(q["photon_tri_tests"] / q["photon_rays"], 2),
                "rays_per_photon_path": round(q["photon_rays"] / q["photon_paths"], 3),
                "stored_per_photon_path": round(q["photons_stored"] / q["photon_paths"], 3),
                "examined_per_hit_point": round(q["gather_examined"] / q["gather_hit_points"], 1),
                "accepted_per_hit_point": round(q["gather_accepted"] / q["gather_hit_points"], 1),
                "buckets_per_hit_point": round(q["gather_buckets"] / q["gather_hit_points"], 2)}
    return {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s", "stages": out, "counts_per_iteration": counts,
            "per_unit": per_unit, "iteration_ms_timed": round(t["ms_iteration"] / nt, 4),
            "note": "stage times with a host wait after each iteration (PM_PROFILE_TIME); the eye pass runs beside "
                    "the photon pass on a second stream, so its time includes sharing the device"}


PREWARM_S = 0.5


def _prewarm(torch, step):
    """Untimed steps for at least PREWARM_S seconds before the W warm-up steps.
    A fresh process's first fraction of a second on the device shows transient
    slow steps (measured on the traversal step: one block of 20 steps at
    3.5 ms/step about 0.25 s after the first launch, against 2.52 ms/step
    before and after it), which would otherwise fall in a short timed
    window.  Returns the number of steps run."""
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < PREWARM_S:
        step()
        torch.cuda.synchronize()
        n += 1
    return n


def sppm_bench(args, torch, api, scenes):
    sc = scenes.procedural_scene()
    v = sc.verts.reshape(-1, 3)
    diag = float(np.linalg.norm(v.max(0) - v.min(0)))
    Np = 1 << 20
    p = api.sppm_params(Np, alpha=0.7, r0=0.05 * diag * 64 / 1280, seed=3)
    bvh = api.build_bvh(sc.verts, sc.tri_mat)
    warm = api.Sppm(sc, p, bvh=bvh)
    prewarm_iters = _prewarm(torch, lambda: warm.iterate(1))   # on a throwaway handle
    warm.destroy()
    s = api.Sppm(sc, p, bvh=bvh)
    s.iterate(2)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    s.iterate(args.sppm_iters)
    e1.record(st)
    torch.cuda.synchronize()
    it_ms = e0.elapsed_time(e1) / args.sppm_iters
    s.status()
    n_stored = int(s.views()["photon_count"][0].item())
    s.destroy()
    # the whole configuration: 64 iterations and the resolve, from a fresh handle (creation not timed)
    full = api.Sppm(sc, p, bvh=bvh)
    torch.cuda.synchronize()
    e0.record(st)
    full.iterate(64)
    full.resolve()
    e1.record(st)
    torch.cuda.synchronize()
    full.status()
    full.destroy()
    full_ms = e0.elapsed_time(e1)
    roof = sppm_roofline(api, sc, dict(n_photons=Np, alpha=0.7, r0=0.05 * diag * 64 / 1280, seed=3), bvh)
    variants, tbvh, schedule, sh = {}, {}, {}, {}
    if args.no_variants:
        bvh.destroy()
        return dict(iteration_ms=it_ms, photons_per_s=Np / (it_ms * 1e-3), n_stored=n_stored, variants=variants,
                    prewarm_iterations=prewarm_iters,
                    full_render={"iterations": 64, "ms": round(full_ms, 2),
                                 "photons_per_s": round(64 * Np / (full_ms * 1e-3), 1)},
                    roofline=roof, tbvh=tbvh, stochastic_hashing=sh, pass_schedule=schedule,
                    workload="procedural 250,094 triangles, 1280x720, 2^20 photons/iteration")
    runs = [("two_phase (default)", dict(photon_kernel=6)), ("two_phase_refill16", dict(photon_kernel=6, refill=16)),
            ("per_path", dict(photon_kernel=1)), ("regen_refill8", dict(photon_kernel=2, refill=8)),
            ("regen_refill16", dict(photon_kernel=2, refill=16)), ("regen_refill32", dict(photon_kernel=2, refill=32))]
    runs += [(f"ray_regen_refill{r}", dict(photon_kernel=4, refill=r)) for r in (4, 8, 16, 24, 32, 48)]
    runs += [("lds_queue", dict(photon_kernel=5))]
    # the paper's own schedule: one bounce per thread per launch (threads = pixels, then fixed pools)
    P = sc.camera.width * sc.camera.height
    runs += [("passes_threads_per_pixel", dict(photon_kernel=3)),
             ("passes_threads_2^18", dict(photon_kernel=3, pass_threads=1 << 18)),
             ("passes_threads_2^20_passes_24", dict(photon_kernel=3, pass_threads=1 << 20, passes=24))]
    # the paper's TBVH comparison: every ray walks one link set (a single threaded BVH)
    runs += [(f"single_link_set_{k}", dict(single_link_set=k + 1)) for k in range(6)]
    for name, kw in runs:
        sv = api.Sppm(sc, api.sppm_params(Np, alpha=0.7, r0=0.05 * diag * 64 / 1280, seed=3, **kw), bvh=bvh)
        sv.iterate(1)
        torch.cuda.synchronize()
        e0.record(st)
        sv.iterate(3)
        e1.record(st)
        torch.cuda.synchronize()
        (tbvh if name.startswith("single") else variants)[name] = round(e0.elapsed_time(e1) / 3, 3)
        if kw.get("photon_kernel") == 3:
            S = kw.get("pass_threads") or min(P, 1 << 26)
            schedule[name] = {"threads": S, "passes": kw.get("passes") or -(-Np // S) + 8,
                              "paths_left_to_drain": int(sv.views()["photon_count"][3].item())}
        sv.destroy()
    # stochastic spatial hashing (Sec. 3.4) against the exact gather: time per
    # iteration, and RMSE after 8 iterations against a 64-iteration exact render
    r0 = 0.05 * diag * 64 / 1280
    ref = api.Sppm(sc, api.sppm_params(Np, alpha=0.7, r0=r0, seed=101), bvh=bvh)
    ref.iterate(64)
    ref_img = ref.resolve().double()
    ref.destroy()
    for name, mode in (("exact", 0), ("stochastic", 1)):
        sv = api.Sppm(sc, api.sppm_params(Np, alpha=0.7, r0=r0, seed=3, gather_mode=mode), bvh=bvh)
        torch.cuda.synchronize()
        e0.record(st)
        sv.iterate(8)
        e1.record(st)
        torch.cuda.synchronize()
        img = sv.resolve().double()
        rmse = float(((img - ref_img) ** 2).mean().sqrt() / ref_img.mean())
        sh[name] = {"iteration_ms": round(e0.elapsed_time(e1) / 8, 3), "relative_rmse_after_8": round(rmse, 4)}
        sv.destroy()
    bvh.destroy()
    return dict(iteration_ms=it_ms, photons_per_s=Np / (it_ms * 1e-3), n_stored=n_stored, variants=variants,
                prewarm_iterations=prewarm_iters, full_render={"iterations": 64, "ms": round(full_ms, 2),
                             "photons_per_s": round(64 * Np / (full_ms * 1e-3), 1)},
                roofline=roof, tbvh=tbvh, stochastic_hashing=sh, pass_schedule=schedule,
                workload="procedural 250,094 triangles, 1280x720, 2^20 photons/iteration")


def adjoint_bench(args, torch, api, scenes):
    """The adjoint workload on the 250k-triangle scene at full size: 16 diffuse
    albedos and Le as parameters, L2 image loss against a target rendered at
    albedos perturbed by U[-0.1, 0.1] (same seed and K), gradient through the
    torch.autograd.Function.  Forward and forward+adjoint use the same K and
    photon count with common random numbers, so the forward image and its RMSE
    are identical by construction.  Two ratios: the autograd route end to end
    (its forward also creates the handle), and the device work of direct calls
    (K iterations + resolve against the replay adjoint)."""
    sc = scenes.procedural_scene()
    v = sc.verts.reshape(-1, 3)
    diag = float(np.linalg.norm(v.max(0) - v.min(0)))
    Np, K = 1 << 20, args.adjoint_iters
    r0 = 0.05 * diag * 64 / 1280
    p = api.sppm_params(Np, alpha=0.7, r0=r0, seed=3)
    pm = sc.albedo_params
    bvh = api.build_bvh(sc.verts, sc.tri_mat)
    rng = np.random.default_rng(11)
    rho_t = sc.mat_rho.copy()
    rho_t[pm] = np.clip(rho_t[pm] + rng.uniform(-0.1, 0.1, len(pm)).astype(np.float32), 0.01, 0.99)
    target = api.render(sc.with_rho(rho_t), p, K, bvh=bvh).double()
    light = int(np.nonzero(sc.mat_Le > 0)[0][0])
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def autograd_step():
        rho = torch.tensor(sc.mat_rho[pm].astype(np.float64), requires_grad=True)
        Le = torch.tensor(float(sc.mat_Le[light]), dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        ev[0].record(st)
        img = api.sppm_render_diff(rho, Le, sc, pm, p, K, bvh=bvh)
        loss = ((img.double() - target) ** 2).mean()
        ev[1].record(st)
        ev[2].record(st)
        loss.backward()
        ev[3].record(st)
        torch.cuda.synchronize()
        return (ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3]), img.detach(),
                np.concatenate([rho.grad.cpu().numpy(), [Le.grad.item()]]), float(loss.item()))

    autograd_step()                      # loads every kernel outside the timing
    f_ms, b_ms, img, grad, loss = autograd_step()
    # the device work alone, direct calls on one handle
    s = api.Sppm(sc, api.sppm_params(Np, alpha=0.7, r0=r0, seed=3, record_iterations=K), bvh=bvh)
    g = (2.0 * (img.double() - target) / img.numel()).float()
    torch.cuda.synchronize()
    ev[0].record(st)
    s.iterate(K)
    img2 = s.resolve()
    ev[1].record(st)
    ev[2].record(st)
    direct = s.adjoint(g, pm)
    ev[3].record(st)
    torch.cuda.synchronize()
    t_fwd, t_adj = ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3])
    s.status()
    same_image = bool(torch.equal(img2, img))
    same_grad = bool(np.array_equal(direct.cpu().numpy(), grad))
    s.destroy()
    bvh.destroy()
    return {"fwd_ms": round(t_fwd, 2), "adjoint_ms": round(t_adj, 2),
            "ratio_fwd_plus_adj_over_fwd": round((t_fwd + t_adj) / t_fwd, 3),
            "autograd": {"forward_ms": round(f_ms, 2), "backward_ms": round(b_ms, 2),
                         "ratio_fwd_plus_bwd_over_fwd": round((f_ms + b_ms) / f_ms, 3),
                         "note": "forward includes creating the handle (device buffers, upload)"},
            "iterations": K, "n_params": len(pm) + 1, "loss": loss,
            "grad_finite": bool(np.all(np.isfinite(grad))), "autograd_equals_direct_call": same_grad,
            "forward_image_identical": same_image,
            "workload": "procedural 250,094 triangles, 1280x720, 2^20 photons/iteration, 16 albedos + Le, "
                        "L2 loss against a render at albedos perturbed by U[-0.1, 0.1]"}


def batch_bench(args, torch, api, scenes):
    """32 procedural scenes of 1k-200k triangles at 128^2-512^2 with 2^16-2^20
    photons each: K iterations of all of them, one persistent launch per stage
    (autotuned chunk/block, hipGraph per iteration), against the same scenes
    rendered one handle after another."""
    work = scenes.batch_workload()
    K = args.batch_iters
    prm = [api.sppm_params(Np, alpha=0.7, r0=r0, seed=100 + i) for i, (_, Np, r0) in enumerate(work)]
    st = torch.cuda.current_stream()
    t0 = time.perf_counter()
    b = api.Batch([w[0] for w in work], prm, autotune=True)
    t_setup = time.perf_counter() - t0
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    e[0].record(st)
    b.iterate(K)
    e[1].record(st)
    torch.cuda.synchronize()
    t_batch = e[0].elapsed_time(e[1])
    b.status()
    info = b.info()
    b.destroy()
    singles = [api.Sppm(w[0], p) for w, p in zip(work, prm)]
    torch.cuda.synchronize()
    e[2].record(st)
    for s in singles:
        s.iterate(K)
    e[3].record(st)
    torch.cuda.synchronize()
    t_seq = e[2].elapsed_time(e[3])
    for s in singles:
        s.destroy()
    photons = sum(Np for _, Np, _ in work) * K
    return {"photons_per_s": round(photons / (t_batch * 1e-3), 1), "ms": round(t_batch, 2),
            "sequential_ms": round(t_seq, 2), "speedup_vs_sequential": round(t_seq / t_batch, 3),
            "iterations": K, "scenes": len(work), "triangles": int(sum(w[0].n_tri for w in work)),
            "pixels": int(sum(w[0].camera.width * w[0].camera.height for w in work)),
            "photons_per_iteration": int(sum(Np for _, Np, _ in work)),
            "chunk": info["chunk"], "block": info["block"], "graph": info["uses_graph"],
            "autotune_ms_per_iter": [[c, bl, round(ms, 3)] for c, bl, ms in info["candidates"]],
            "setup_s": round(t_setup, 2)}


def achievable_bandwidth(torch, api):
    """Measured streaming bandwidth of the device with the library's own stream
    kernel (pm_probe_stream): a 1 GiB copy (read + write bytes) and a 1 GiB
    read (the traversal's bytes are almost all reads); best of 5 each.  torch's
    copy_ of the same buffer is listed for comparison."""
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = torch.zeros(1, dtype=torch.int32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def best_ms(fn):
        fn()
        best = 1e30
        for _ in range(5):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    copy_ms = best_ms(lambda: api.probe_stream(src, dst))
    assert torch.equal(dst, src)
    read_ms = best_ms(lambda: api.probe_stream(src, out=out))
    torch_copy_ms = best_ms(lambda: dst.copy_(src))
    nb = src.numel() * 4
    del src, dst
    return {"kernel": "pm_probe_stream", "bytes": nb, "copy_GBps": round(2 * nb / (copy_ms * 1e-3) / 1e9, 1),
            "read_GBps": round(nb / (read_ms * 1e-3) / 1e9, 1),
            "torch_copy_GBps": round(2 * nb / (torch_copy_ms * 1e-3) / 1e9, 1)}


def dependent_read_rate(torch, api, n_lanes, steps, log2_rows=24):
    """Achievable rate of dependent random 16-byte reads (pm_probe_chase):
    n_lanes chains of `steps` reads each over 2^log2_rows random rows (256 MiB
    by default, about the size of the soup's BVH): the access pattern of the
    incoherent walk without its arithmetic.  Best of 5."""
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    rows = torch.randint(-2**31, 2**31 - 1, (1 << log2_rows, 4), dtype=torch.int32, device="cuda", generator=g)
    out = torch.empty(n_lanes, dtype=torch.int32, device="cuda")
    api.probe_chase(rows, steps, n_lanes, out=out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = 1e30
    for _ in range(5):
        e0.record()
        api.probe_chase(rows, steps, n_lanes, out=out)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del rows, out
    rate = n_lanes * steps / (best * 1e-3)
    return {"rows_bytes": 16 << log2_rows, "lanes": n_lanes, "steps": steps, "ms": round(best, 4),
            "reads_per_s": round(rate, 1), "GBps": round(16 * rate / 1e9, 1)}


def cpu_baseline(tb, scenes):
    import oracle
    nth = _cpu_threads()
    coh, inc = tb["rays"]
    rng = np.random.default_rng(5)
    sample = np.concatenate([coh[rng.choice(len(coh), 1 << 18, replace=False)],
                             inc[rng.choice(len(inc), 1 << 18, replace=False)]])
    t0 = time.perf_counter()
    osc = oracle.OracleScene(tb["scene"], use_bvh=True)
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    osc.trace(sample, nthreads=nth)
    dt = time.perf_counter() - t0
    bf = sample[:: len(sample) // 512][:512]
    t0 = time.perf_counter()
    osc.trace(bf, brute_force=True, nthreads=nth)
    dt_bf = time.perf_counter() - t0
    # the oracle's SPPM: the full box configuration, and one reduced iteration of the procedural scene
    sppm = {}
    box = oracle.OracleScene(scenes.box_scene(64, 64))
    t0 = time.perf_counter()
    oracle.sppm_run(box, 1, 1 << 14, 2, r0=0.05 * np.sqrt(3.0), nthreads=nth)
    dt_box = (time.perf_counter() - t0) / 2
    sppm["box_64x64_2^14_photons"] = {"s_per_iteration": round(dt_box, 4),
                                      "photons_per_s": round((1 << 14) / dt_box, 1)}
    sc = scenes.procedural_scene()
    v = sc.verts.reshape(-1, 3)
    diag = float(np.linalg.norm(v.max(0) - v.min(0)))
    proc = oracle.OracleScene(sc, use_bvh=True)
    t0 = time.perf_counter()
    oracle.sppm_run(proc, 3, 1 << 20, 2, r0=0.05 * diag * 64 / 1280, nthreads=nth)
    dt_proc = (time.perf_counter() - t0) / 2
    sppm["procedural_1280x720_2^20_photons"] = {"s_per_iteration": round(dt_proc, 3),
                                                "photons_per_s": round((1 << 20) / dt_proc, 1),
                                                "note": "2 of the configuration's 64 iterations"}
    return {"value": len(sample) / dt / 1e6, "unit": "Mrays/s", "cores": nth, "kind": "oracle", "host": _host_info(),
            "sample": (f"oracle median-split BVH over the same 2^20-triangle soup, 2^18 coherent + 2^18 "
                       f"incoherent rays sampled from the workload (build {t_build:.2f} s not counted); "
                       f"brute force over all triangles: {len(bf) / dt_bf:.1f} rays/s on 512 of them"),
            "sppm": sppm}


def main():
    args = _parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (rays, and the photon "
              "index range of an iteration, would be sharded per GPU with one integer all-reduce of the "
              "per-pixel counts and fluxes).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1505_06022_amd import api, scenes
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe:   # the library's stream copy of 1 GiB, three times (calibrates HBM byte counters)
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            api.probe_stream(src, dst)
        torch.cuda.synchronize()
        del src, dst
    if args.only_sppm:
        sp = sppm_bench(args, torch, api, scenes)
        print(json.dumps({"sppm_only": True, "photons_per_s": round(sp["photons_per_s"], 1),
                          "iteration_ms": round(sp["iteration_ms"], 3), "stored_photons": sp["n_stored"],
                          "full_render_64_iterations": sp["full_render"], "roofline": sp["roofline"],
                          "workload": sp["workload"]}), flush=True)
        return
    tb = traversal_bench(args, torch, api, scenes)
    out = {
        "metric": "Mrays/s traversal + SPPM photons/s; fwd+adjoint vs fwd time at matched RMSE",
        # value: the first part (closest-hit traversal, MTBVH); the other two are
        # sppm.photons_per_s and adjoint.ratio_fwd_plus_adj_over_fwd below
        "value_part": "Mrays/s traversal (closest hit, MTBVH)",
        "value": round(tb["n_rays"] / (tb["step_ms"] * 1e-3) / 1e6, 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(tb["step_ms"], 4),
        "prewarm_steps": tb["prewarm_steps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "traversal: 2^20 random triangles (lognormal(-5,0.5) edges), SAH 32 bins leaf<=4 "
                               f"node cost {tb['trav_cost']:g}, spatial splits alpha={tb['split_alpha']:g}, "
                               "1920x1080 coherent + 2^21 incoherent rays",
                   "n_rays": tb["n_rays"], "n_tri": 1 << 20, "parallelism": "none",
                   "trace_options": {"coherent": [args.coherent, dict(KERNEL_VARIANTS)[args.coherent]],
                                     "incoherent": [args.incoherent, dict(KERNEL_VARIANTS)[args.incoherent]]}},
        "coherent_mrays_s": round(tb["coherent_mrays"], 2),
        "incoherent_mrays_s": round(tb["incoherent_mrays"], 2),
        "kernel_mrays_s": round(tb["n_rays"] / (tb["kern_ms"].mean() * 1e-3) / 1e6, 2),
        "one_after_another_mrays_s": round(tb["n_rays"] / (tb["batch_ms"].sum() * 1e-3) / 1e6, 2),
        "bvh": dict({k: tb["info"][k] for k in ("n_tri", "n_refs", "n_nodes", "n_leaves", "depth", "sah_cost",
                                                 "device_bytes", "build_ms")}, split_alpha=tb["split_alpha"],
                    trav_cost=tb["trav_cost"]),
        "kernel_variants": tb["variants"],
        "gpu_lbvh": tb["lbvh"],
        "tbvh_ablation": ({"single_link_set": tb["tbvh"],
                           "mtbvh_over_mean_tbvh": round(tb["n_rays"] / (tb["batch_ms"].sum() * 1e-3) / 1e6 /
                                                         float(np.mean([v["mrays_s"] for v in tb["tbvh"].values()])), 3)}
                          if tb["tbvh"] else None),
        "traversal_stats": [{"rays": int(n), "boxes_per_ray": round(vn / n, 2), "tris_per_ray": round(vt / n, 2)}
                            for vn, vt, n in tb["per_batch"]],
        "roofline": {"bound": "hbm", "achieved": round(tb["achieved"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(tb["achieved"] / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                     "kernel": "pm_trace_rays_multi call: k_hist_count + column and bucket scans + k_hist_scatter, then one launch of "
                               "k_trace_perm_then_tiles (the incoherent batch's postponed walk, then the camera "
                               "batch's packets over 8x8 pixel tiles)",
                     "bytes_per_launch": tb["per_launch_bytes"],
                     "avg_launch_ms": round(float(tb["kern_ms"].mean()), 4),
                     "alone_ms_by_batch": [round(float(x), 4) for x in tb["batch_ms"]]},
    }
    ach = achievable_bandwidth(torch, api)
    best = max(ach["copy_GBps"], ach["read_GBps"])
    out["roofline"]["achievable"] = dict(ach, frac=round(tb["achieved"] / best, 4))
    # the incoherent walk (node visits per second, bucketing included) against chains of dependent random
    # reads of the same length per lane: over a BVH-sized buffer (reads served by the Infinity Cache and
    # HBM) and over 4 MiB (one XCD's L2 holds it: the rate of a walk whose every node read hits L2)
    vn_inc, _, n_inc = tb["per_batch"][1]
    steps = max(1, int(round(vn_inc / n_inc)))
    node_rate = vn_inc / (float(tb["batch_ms"][1]) * 1e-3)
    far = dependent_read_rate(torch, api, n_inc, steps, log2_rows=24)
    near = dependent_read_rate(torch, api, n_inc, steps, log2_rows=18)
    out["roofline"]["achievable"]["dependent_reads"] = {
        "incoherent_node_visits_per_s": round(node_rate, 1), "random_256MiB": far, "random_4MiB": near,
        "frac_of_4MiB": round(node_rate / near["reads_per_s"], 4),
        "ratio_to_256MiB": round(node_rate / far["reads_per_s"], 3)}
    if not args.no_sppm:
        sp = sppm_bench(args, torch, api, scenes)
        out["sppm"] = {"photons_per_s": round(sp["photons_per_s"], 1), "iteration_ms": round(sp["iteration_ms"], 3),
                       "timed_iterations": args.sppm_iters, "prewarm_iterations": sp["prewarm_iterations"],
                       "full_render_64_iterations": sp["full_render"], "roofline": sp["roofline"],
                       "stored_photons": sp["n_stored"], "workload": sp["workload"],
                       "iteration_ms_by_photon_kernel": sp["variants"],
                       "one_bounce_per_pass_schedule": sp["pass_schedule"],
                       "gather_exact_vs_stochastic_hashing": sp["stochastic_hashing"],
                       "tbvh_ablation": ({"iteration_ms_single_link_set": sp["tbvh"],
                                          "mean_ratio_tbvh_over_mtbvh": round(
                                              float(np.mean(list(sp["tbvh"].values()))) / sp["iteration_ms"], 3)}
                                         if sp["tbvh"] else None)}
    if not args.no_adjoint:
        out["adjoint"] = adjoint_bench(args, torch, api, scenes)
    if not args.no_batch:
        os.environ.setdefault("PM_AUTOTUNE_CACHE", os.path.join("/tmp", "pm_autotune_bench.txt"))
        out["batch"] = batch_bench(args, torch, api, scenes)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(tb, scenes)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
