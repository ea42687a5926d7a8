#!/usr/bin/env python3
"""Benchmark: pill-constraint projections per second of the VIPER rod substep on one MI355X.

Workload: 4096 independent rods x 64 pills (random helices, FP32), 20 substeps x 8
iterations per frame, collision-free; one "step" = one frame of the whole solver
(prediction, 8 x four colour passes of stretch-shear / volume / scale-gradient /
bend-twist projections, velocity update) for all rods.  Inputs are resident in HBM
before timing starts; the timed region holds exactly K frames between
synchronisations.

Prints one JSON line with the throughput, a roofline object for the dominant kernel
(timed per launch with HIP events on the launch stream) and the oracle timed on the
host cores on a bounded sample of the same workload.  Further entries of the same line:
the rate split by constraint type (`config.projections_per_s_by_type`), the 32-pill FP64
rod (`single_rod`), the contact, skinning, skinning-weight (initial and faired),
octopus-shaped and bundling scenes, the two solvers and the optional energy terms
(`solvers`), the bone warm start (`bones`), the one-substep-per-launch kernel
(`substep_kernel`), the helix scene at 16x the rods (`helix_16x`), the measured copy
ceiling (`copy_ceiling`), the adjoint and the serving loop (`serving`, whose p50/p99 frame
latencies are repeated at the top level).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FLOPs per projection / per pill-substep, counted from the closed-form updates in
# csrc/rod_kernels.hip (add, sub, mul, div, sqrt, rsqrt = 1 each; a fused
# multiply-add counts as its multiply and its add).
FLOP = {"ss": 122, "vol": 53, "sg": 16, "bt": 337, "predict": 59, "velocity": 42}
# Bytes one frame launch moves per pill (FP32): state 15 words read + written,
# 13 rest words and one flag word read.
BYTES_PER_PILL_LAUNCH = 4 * (15 + 15 + 13 + 1)
PEAK_FP32_VALU = 78.6e12     # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz, packed FP32 disabled
SURVEY_FLOP_PER_PILL_SUBSTEP = 2750.0   # the survey's estimate of the same work (2.5-3 kFLOP)
PEAK_HBM = 8.0e12


def kernel_source_hash():
    """Hash of what the frame kernel is compiled from: its own definition in rod_kernels.hip,
    the device headers it includes and the build flags (edits to other kernels of
    rod_kernels.hip leave it unchanged)."""
    csrc = os.path.join(ROOT, "paper_1906_05260_amd", "csrc")
    h = hashlib.sha256()
    with open(os.path.join(csrc, "rod_kernels.hip")) as fh:
        src = fh.read()
    i = src.index(" rod_frame_kernel(")
    h.update(src[src.rfind("template <", 0, i):src.index("\n}\n", i) + 3].encode())
    for f in (os.path.join(csrc, "rod_device.h"), os.path.join(csrc, "viper_dev.h"),
              os.path.join(ROOT, "paper_1906_05260_amd", "build.py")):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "%s_%s_counters.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def _dispatch_values(db, counter, name_like):
    """Per-dispatch values of one counter (summed over its hardware instances) for the kernels
    whose name matches, in dispatch order, from a rocprofv3 results database."""
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("SELECT dispatch_id, kernel_name, value FROM counters_collection WHERE counter_name = ? AND "
                       "kernel_name LIKE ? ORDER BY dispatch_id", (counter, name_like)).fetchall()
    con.close()
    return rows


def write_counter_summaries(fetch_db, write_db, copy_fetch_db, copy_write_db, frames, copy_mib):
    """HBM bytes per launch of the FP32 frame kernel on the helix 4096 x 64 workload, from two
    rocprofv3 --pmc runs of this bench (FETCH_SIZE, then WRITE_SIZE; the first `frames` float
    frame-kernel dispatches are the headline's whole-frame launches, the rest the per-substep
    leg's) and two of its --copy-mib run, which scale each counter to known bytes.  Writes
    profiles/rod_frame_kernel{,_substep}_helix4096x64_counters.json with the source hash."""
    like = "%rod_frame_kernel<float%"
    known = copy_mib * (1 << 20)
    scale = {}
    for key, db, counter in (("fetch", copy_fetch_db, "FETCH_SIZE"), ("write", copy_write_db, "WRITE_SIZE")):
        v = [r[2] for r in _dispatch_values(db, counter, "%neg%")]
        if not v:
            raise SystemExit("no copy-reference dispatches in %s" % db)
        scale[key] = known / (float(np.median(v)) * 1024.0)
    fetch = _dispatch_values(fetch_db, "FETCH_SIZE", like)
    write = _dispatch_values(write_db, "WRITE_SIZE", like)
    if len(fetch) <= frames or len(write) <= frames:
        raise SystemExit("expected more than %d frame-kernel dispatches" % frames)
    for suffix, sel in (("", slice(0, frames)), ("_substep", slice(frames + 1, None))):
        f = float(np.mean([r[2] for r in fetch[sel]]))
        w = float(np.mean([r[2] for r in write[sel]]))
        rd, wr = f * 1024.0 * scale["fetch"], w * 1024.0 * scale["write"]
        rec = {"kernel": fetch[0][1].split("(")[0].replace("void viper::", ""), "workload": "helix4096x64",
               "launch": "one frame (20 substeps)" if not suffix else "one substep",
               "source_hash": kernel_source_hash(), "dispatches": len(fetch[sel]),
               "fetch_kib_per_dispatch": f, "write_kib_per_dispatch": w,
               "fetch_scale": scale["fetch"], "write_scale": scale["write"],
               "hbm_bytes_per_launch": rd + wr, "hbm_read_bytes_per_launch": rd, "hbm_write_bytes_per_launch": wr,
               "copy_reference": "torch neg over %d MiB (bench.py --copy-mib %d)" % (copy_mib, copy_mib),
               "source_files": ["paper_1906_05260_amd/csrc/rod_kernels.hip (rod_frame_kernel)",
                                "paper_1906_05260_amd/csrc/rod_device.h", "paper_1906_05260_amd/csrc/viper_dev.h",
                                "paper_1906_05260_amd/build.py"]}
        path = os.path.join(ROOT, "profiles", "rod_frame_kernel%s_helix4096x64_counters.json" % suffix)
        with open(path, "w") as fh:
            json.dump(rec, fh, indent=1)
            fh.write("\n")
        print(path, json.dumps(rec), flush=True)


def sync_diverged(viper, sc, desc):
    """viper_sync; on the NaN status, the number of rods with a non-finite state instead of an
    error.  Some soft helices of the random-compliance workload go unstable (scales through
    zero) within the first frames, in the FP64 oracle too, and such a rod can overflow in FP32
    after tens of frames; rods are independent, so the rest of the scene is unaffected."""
    try:
        sc.sync()
        return 0
    except viper.ViperError as e:
        if e.status != viper.ERR_NAN:
            raise
    st = sc.state()
    bad = ~(np.isfinite(st["x"]).all(1) & np.isfinite(st["s"]) & np.isfinite(st["q"]).all(1))
    return len(set((np.searchsorted(desc.rod_offsets, np.nonzero(bad)[0], side="right") - 1).tolist()))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(desc, dt, sub, iters, rods, threads):
    """The oracle (FP64, rods split across threads; rods are independent without
    contacts, so the result equals the serial run) on a bounded sample of the workload."""
    import oracle
    sample = desc.subset(range(rods))
    o = oracle.OracleScene(sample, "f64")
    t0 = time.perf_counter()
    n = o.step(dt, sub, iters, threads=threads)
    el = time.perf_counter() - t0
    return {"value": n / el, "unit": "projections/s", "cores": threads, "kind": "oracle",
            "host_cores": os.cpu_count(),
            "sample": "%d of %d rods, 1 frame (%d substeps x %d iterations), FP64, %d threads on %s (%d cores "
                      "visible)" % (rods, desc.num_rods, sub, iters, threads, cpu_model(), os.cpu_count() or 0),
            "seconds": el, "pill_substeps_per_s": sample.num_pills * sub / el}


def copy_reference(torch, dev, mib, steps):
    """A plain elementwise copy kernel (read n bytes, write n bytes) of known size."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.3:       # bring the clocks up before timing
        torch.neg(a, out=b)
        torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        torch.neg(a, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    rec = {"kernel": "neg (elementwise copy)", "bytes_read": 4 * n, "bytes_written": 4 * n,
           "ms_per_launch": ms, "GB_per_s": 8 * n / (ms * 1e-3) / 1e9}
    del a, b
    return rec


def adjoint_timing(torch, viper, scenes, dev, reps=5):
    """Forward with per-substep checkpoints and backward of one frame on 1024 straight rods x
    32 pills (FP32, 20 substeps x 8 iterations), L = sum |x_free_end - target|^2.  Each
    repetition runs every measured call once untimed on the same scenes and buffers, then times
    the second: the plain frame, the checkpointed frame and the backward (HIP events on the
    launch stream; medians over the repetitions)."""
    desc, targets = scenes.straight_rods(1024, 32, seed=4)
    dt, sub, iters = 1.0 / 60.0, 20, 8
    st = torch.cuda.current_stream()
    times = {"plain": [], "forward": [], "backward": []}
    last = torch.as_tensor(desc.rod_offsets[1:] - 1, device=dev, dtype=torch.long)
    tg = torch.as_tensor(targets, device=dev, dtype=torch.float32)
    for r in range(reps):
        sc = viper.Scene(desc, "f32", device=dev)
        nc, nw = sc.adjoint_sizes(1, sub, iters)
        ckpt = torch.empty(nc, dtype=torch.uint8, device=dev)
        work = torch.empty(nw, dtype=torch.uint8, device=dev)
        ref = viper.Scene(desc, "f32", device=dev)
        for timed in (False, True):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
            ev[0].record(st)
            ref.step(dt, sub, iters, mode=viper.MODE_FRAME)
            ev[1].record(st)
            ev[2].record(st)
            sc.step_checkpointed(dt, 1, sub, iters, ckpt=ckpt)
            ev[3].record(st)
            x = sc.get("x")
            g = torch.zeros_like(x)
            g[last] = 2.0 * (x[last] - tg)
            ev[4].record(st)
            sc.backward(dt, 1, sub, iters, ckpt, g, work=work)
            ev[5].record(st)
            torch.cuda.synchronize()
            sc.sync()
            ref.sync()
            if timed:
                times["plain"].append(ev[0].elapsed_time(ev[1]))
                times["forward"].append(ev[2].elapsed_time(ev[3]))
                times["backward"].append(ev[4].elapsed_time(ev[5]))
    med = {k: float(sorted(v)[len(v) // 2]) for k, v in times.items()}
    return {"workload": "straight1024x32", "frames": 1, "substeps": sub, "iterations": iters, "dtype": "f32",
            "plain_frame_ms": med["plain"], "forward_checkpointed_ms": med["forward"],
            "backward_ms": med["backward"], "backward_over_forward": med["backward"] / med["plain"],
            "backward_over_checkpointed_forward": med["backward"] / med["forward"],
            "checkpoint_bytes": nc, "backward_scratch_bytes": nw,
            "params": desc.num_pills + desc.num_rods}


def single_rod_timing(torch, viper, scenes, dev, frames=120):
    """One 32-pill rod in FP64, 10 substeps x 4 iterations, 120 frames: launch/latency-bound;
    GPU microseconds per frame (one frame kernel each) next to the oracle's."""
    import oracle
    desc = scenes.straight_rod(32)
    dt, sub, iters = 1.0 / 60.0, 10, 4
    sc = viper.Scene(desc, "f64", device=dev)
    sc.step(dt, sub, iters)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(frames):
        sc.step(dt, sub, iters)
    e1.record(st)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e6 / frames
    o = oracle.OracleScene(desc, "f64")
    t1 = time.perf_counter()
    for _ in range(frames):
        o.step(dt, sub, iters)
    cpu = (time.perf_counter() - t1) * 1e6 / frames
    return {"workload": "single_rod32_f64", "frames": frames, "substeps": sub, "iterations": iters,
            "gpu_us_per_frame": e0.elapsed_time(e1) * 1e3 / frames, "gpu_wall_us_per_frame": wall,
            "oracle_us_per_frame_1core": cpu}


def contact_skin_timing(torch, viper, scenes, dev, frames=10):
    """The muscle scene (64 muscles, ~45k pills, FP32, uniform-grid pill-pill contacts,
    20 substeps x 8 iterations) and LBS skinning of its 200k-vertex mesh: ms per frame
    and per skinning pass, timed with HIP events on the launch stream."""
    desc, mesh = scenes.muscle_scene(64, seed=2)
    sc = viper.Scene(desc, "f32", device=dev, collisions=True)
    sid = sc.create_skin(mesh.rest_v, mesh.caps, mesh.w)
    dt, sub, iters = 1.0 / 60.0, 20, 8
    for _ in range(2):
        sc.step(dt, sub, iters)
    sc.sync()
    st = torch.cuda.current_stream()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    out = torch.empty((mesh.rest_v.shape[0], 3), dtype=torch.float32, device=dev)
    e3, e4 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(frames):
        sc.step(dt, sub, iters)                       # GRAPH: the captured frame replayed
    e1.record(st)
    for _ in range(frames):
        sc.skin(sid, out=out)
    e2.record(st)
    for _ in range(frames):
        sc.step(dt, sub, iters, mode=viper.MODE_ITERATION)   # the same launches, eager
    e3.record(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(frames):
        sc.step(dt, sub, iters)
    torch.cuda.synchronize()
    wall_graph = (time.perf_counter() - t0) * 1e3 / frames
    sc.sync()
    frame_ms = e0.elapsed_time(e1) / frames
    skin_ms = e1.elapsed_time(e2) / frames
    eager_ms = e2.elapsed_time(e3) / frames
    V = int(mesh.rest_v.shape[0])
    skin_bytes = 56 * V + 48 * sc.capsules     # rest vertex 12 + 4 ids 16 + 4 weights 16 + out 12; transforms
    # initial skinning weights of the same mesh (Sec. 7.4; brute force over every capsule), on a
    # fresh scene at the rest pose
    rest_sc = viper.Scene(desc, "f32", device=dev, collisions=True)
    e7, e8 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rest_sc.skin_weights(mesh.rest_v[:1024])
    e7.record(st)
    rest_sc.skin_weights(mesh.rest_v)
    e8.record(st)
    torch.cuda.synchronize()
    weights_ms = e7.elapsed_time(e8)
    del rest_sc
    # the same skinning with a mesh far beyond the caches: the 200k-vertex mesh tiled to
    # ~16.6M vertices (0.93 GB of vertex data); every tile references the same capsules.  The
    # mesh numbers its vertices by first capsule; the same mesh numbered along each muscle's
    # axis (random around it) is timed beside it
    reps = (16 << 20) // V
    VL = reps * V

    def large_pass(m):
        big_caps = np.tile(m.caps, (reps, 1))
        big_w = np.tile(m.w, (reps, 1))
        big_v = np.tile(m.rest_v, (reps, 1))
        sid_l = sc.create_skin(big_v, big_caps, big_w)
        del big_caps, big_w, big_v
        out_l = torch.empty((VL, 3), dtype=torch.float32, device=dev)
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 0.3:       # the host-side set-up left the GPU idle: clocks up first
            sc.skin(sid_l, out=out_l)
            torch.cuda.synchronize()
        e5, e6 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e5.record(st)
        for _ in range(frames):
            sc.skin(sid_l, out=out_l)
        e6.record(st)
        torch.cuda.synchronize()
        sc._skins[sid_l] = None                     # free the device copies
        return e5.elapsed_time(e6) / frames

    skin_l_ms = large_pass(mesh)
    _, mesh_axis = scenes.muscle_scene(64, seed=2, capsule_order=False)
    skin_axis_ms = large_pass(mesh_axis)
    skin_l_bytes = 56 * VL + 48 * sc.capsules
    # skinning weights faired over a closed 200k-vertex tube mesh on the muscles' envelopes
    # (4 Jacobi iterations), on a fresh scene at the rest pose
    tube = scenes.tube_mesh(desc, V, seed=2, jitter=0.05)
    rest_sc = viper.Scene(desc, "f32", device=dev, collisions=True)
    rest_sc.skin_weights_faired(tube.rest_v[:1024], tube.tris[:0], 1)
    t0 = time.perf_counter()
    rest_sc.skin_weights_faired(tube.rest_v, tube.tris, 4, 0.5)
    faired_s = time.perf_counter() - t0
    del rest_sc
    return {"workload": "muscle64_%dpills" % desc.num_pills, "pills": desc.num_pills, "capsules": sc.capsules,
            "contact_pairs_last_substep": int(len(sc.contacts())), "frame_ms": frame_ms,
            "frame_ms_eager_launches": eager_ms, "frame_ms_wall_graph": wall_graph,
            "pill_substeps_per_s": desc.num_pills * sub / (frame_ms * 1e-3),
            # per substep: the velocity update (which also predicts the next substep, starts its
            # detection and runs its first rod iteration), 6 detection launches (cell keys, cell
            # scan, bucket scatter, count pass, candidate scan, emit pass), a contact pass per
            # iteration and a rod iteration per iteration but the first; the first substep's
            # prediction and first rod iteration
            "launches_per_frame": 2 + sub * (1 + 4 + iters + (iters - 1)),
            "skin_vertices": V, "skin_ms": skin_ms, "skin_weights_ms": weights_ms,
            "skin_algorithmic_GB_per_s": skin_bytes / (skin_ms * 1e-3) / 1e9,
            "skin_large": {"vertices": VL, "ms": skin_l_ms, "algorithmic_bytes": skin_l_bytes,
                           "GB_per_s": skin_l_bytes / (skin_l_ms * 1e-3) / 1e9,
                           "hbm_frac": skin_l_bytes / (skin_l_ms * 1e-3) / PEAK_HBM,
                           "vertex_order": "by first capsule",
                           "axis_order_ms": skin_axis_ms,
                           "axis_order_GB_per_s": skin_l_bytes / (skin_axis_ms * 1e-3) / 1e9},
            "skin_weights_faired": {"vertices": int(tube.rest_v.shape[0]), "triangles": int(tube.tris.shape[0]),
                                    "iterations": 4, "wall_s_with_host_graph": faired_s}}


def paper_shaped_timing(torch, viper, scenes, dev, frames=10):
    """The paper's octopus-sized scene (100 models x 37 pills, inter-model collisions, each
    skinned to 6.5k vertices): ms per frame at 20 x 8 and per skinning pass, beside the
    paper's ~7 ms per frame on one GTX 1080 (its substeps and iterations are unstated)."""
    desc, mesh = scenes.octopus_scene()
    sc = viper.Scene(desc, "f32", device=dev, collisions=True)
    sid = sc.create_skin(mesh.rest_v, mesh.caps, mesh.w)
    out = torch.empty((mesh.rest_v.shape[0], 3), dtype=torch.float32, device=dev)
    res = {"workload": "octopus100x37", "pills": desc.num_pills, "skin_vertices": int(mesh.rest_v.shape[0])}
    st = torch.cuda.current_stream()
    for sub, it in ((20, 8), (4, 4)):
        for _ in range(2):
            sc.step(1.0 / 60.0, sub, it)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(st)
        for _ in range(frames):
            sc.step(1.0 / 60.0, sub, it)
        e1.record(st)
        for _ in range(frames):
            sc.step(1.0 / 60.0, sub, it)
            sc.skin(sid, out=out)
        e2.record(st)
        torch.cuda.synchronize()
        res["frame_ms_%dx%d" % (sub, it)] = e0.elapsed_time(e1) / frames
        res["frame_plus_skin_ms_%dx%d" % (sub, it)] = e1.elapsed_time(e2) / frames
    sc.sync()
    res["paper_ms_gtx1080"] = 7.0
    return res


def bundling_timing(torch, viper, scenes, dev, frames=10):
    """The 64-muscle scene (FP32, contacts, 20 substeps x 8 iterations) with one bundling
    cross-section per pill index of each muscle (Sec. 7.3 shape matching after the
    iterations of every substep): ms per frame beside the same scene without sections.
    The difference is mostly not the two bundling kernels (~35 us per substep): the hard
    projection leaves this synthetic muscle faster-moving and more crowded, and the
    neighbour search walks more."""
    res = {}
    for bundling in (False, True):
        desc, _ = scenes.muscle_scene(64, seed=2, mesh_vertices=0, bundling=bundling)
        sc = viper.Scene(desc, "f32", device=dev, collisions=True)
        for _ in range(2):
            sc.step(1.0 / 60.0, 20, 8)
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(frames):
            sc.step(1.0 / 60.0, 20, 8)
        e1.record(st)
        torch.cuda.synchronize()
        sc.sync()
        res["frame_ms_bundled" if bundling else "frame_ms_plain"] = e0.elapsed_time(e1) / frames
        if bundling:
            res.update(workload="muscle64_%dpills_bundled" % desc.num_pills,
                       sections=int(len(desc.section_offsets) - 1), section_entries=int(desc.section_offsets[-1]))
    res["bundling_ms_per_substep"] = (res["frame_ms_bundled"] - res["frame_ms_plain"]) / 20
    return res


def solver_timing(torch, viper, scenes, dev, frames=5):
    """The helix workload (4096 x 64, FP32, 20 substeps x 8 iterations) in ITERATION mode
    (one launch per constraint iteration), coloured Gauss-Seidel beside Jacobi with averaging
    (Sec. 7): ms per frame, HIP events on the launch stream."""
    import dataclasses
    base = scenes.helix_rods(4096, 64, seed=1)
    res = {"workload": "helix4096x64_iteration_mode"}
    for solver in ("gauss_seidel", "jacobi"):
        sc = viper.Scene(dataclasses.replace(base, solver=solver), "f32", device=dev)
        sc.step(1.0 / 60.0, 20, 8, mode=viper.MODE_ITERATION)
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(frames):
            sc.step(1.0 / 60.0, 20, 8, mode=viper.MODE_ITERATION)
        e1.record(st)
        torch.cuda.synchronize()
        sc.sync()
        res["frame_ms_" + solver] = e0.elapsed_time(e1) / frames
    # the fused frame kernel (one launch per frame) with the optional cross-section stretch
    # (eq. stretch_xy) on every rod, beside the same kernel without it
    for name, c in (("frame_ms_fused", None), ("frame_ms_fused_cross_stretch", np.full(base.num_rods, 1e-7))):
        sc = viper.Scene(dataclasses.replace(base, cross_compliance=c), "f32", device=dev)
        sc.step(1.0 / 60.0, 20, 8, mode=viper.MODE_FRAME)
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(frames):
            sc.step(1.0 / 60.0, 20, 8, mode=viper.MODE_FRAME)
        e1.record(st)
        torch.cuda.synchronize()
        sc.sync()
        res[name] = e0.elapsed_time(e1) / frames
    return res


def large_timing(torch, viper, scenes, dev, rods=65536, frames=5):
    """The helix workload at 16x the rods (65,536 x 64 = 4.2M pills, FP32, 20 x 8): its workspace
    (~1.4 GB) no longer fits the 256 MB MALL; a frame launch still reads and writes the state
    once, so the kernel stays VALU-bound.  ms per frame launch (HIP events on the launch
    stream) and the same VALU roofline as the headline."""
    desc = scenes.helix_rods(rods, 64, seed=1)
    sc = viper.Scene(desc, "f32", device=dev)
    sc.step(1.0 / 60.0, 20, 8, mode=viper.MODE_FRAME)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(frames):
        sc.step(1.0 / 60.0, 20, 8, mode=viper.MODE_FRAME)
    e1.record(st)
    torch.cuda.synchronize()
    sc.sync()
    ms = e0.elapsed_time(e1) / frames
    P = desc.num_pills
    edges, bts = P - desc.num_rods, P - 2 * desc.num_rods
    flop = 20 * (8 * (edges * (FLOP["ss"] + FLOP["vol"] + FLOP["sg"]) + bts * FLOP["bt"]) +
                 P * (FLOP["predict"] + FLOP["velocity"]))
    return {"workload": "helix%dx64" % rods, "pills": P, "ms_per_frame": ms,
            "projections_per_s": sc.projections_per_iteration * 8 * 20 / (ms * 1e-3),
            "tflops": flop / (ms * 1e-3) / 1e12, "frac": flop / (ms * 1e-3) / PEAK_FP32_VALU,
            "algorithmic_GB_per_s": BYTES_PER_PILL_LAUNCH * P / (ms * 1e-3) / 1e9}


def substep_kernel_timing(torch, viper, scenes, dev, frames=3):
    """The helix workload (4096 x 64, FP32, 8 iterations) with one launch per substep
    (VIPER_MODE_SUBSTEP: the state streamed through HBM every substep), each launch timed with
    HIP events on the launch stream: us per launch, algorithmic GB/s against 8 TB/s, and the
    HBM bytes per launch from the committed counter summary (when taken on this source)."""
    desc = scenes.helix_rods(4096, 64, seed=1)
    sc = viper.Scene(desc, "f32", device=dev)
    h = 1.0 / 60.0 / 20
    sc.step(h, 1, 8, mode=viper.MODE_SUBSTEP)
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20 * frames)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(st)
        sc.step(h, 1, 8, mode=viper.MODE_SUBSTEP)
        b.record(st)
    torch.cuda.synchronize()
    sc.sync()
    us = sum(a.elapsed_time(b) for a, b in ev) / len(ev) * 1e3
    P = desc.num_pills
    nbytes = BYTES_PER_PILL_LAUNCH * P
    traffic = measured_traffic("rod_frame_kernel_substep", "helix4096x64")
    return {"workload": "helix4096x64", "kernel": "rod_frame_kernel (one substep per launch)", "us_per_launch": us,
            "algorithmic_bytes_per_launch": nbytes, "algorithmic_GB_per_s": nbytes / (us * 1e-6) / 1e9,
            "hbm_frac": nbytes / (us * 1e-6) / PEAK_HBM, "traffic": traffic,
            "counter_GB_per_s": traffic / (us * 1e-6) / 1e9 if traffic else None}


def bones_timing(torch, viper, scenes, dev, calls=50):
    """The bone warm start (Sec. 8.2) on the helix workload (4096 x 64, FP32): two bones, every
    pill blended between them by its position along its rod; us per set_bones call (HIP events
    on the launch stream) and algorithmic GB/s (per pill: two weights 16 B, two ids 8 B, the
    position read and written 24 B, its rod index 4 B)."""
    import dataclasses
    d = scenes.helix_rods(4096, 64, seed=1)
    u = np.tile(np.linspace(0.0, 1.0, 64), 4096)
    rest = np.tile(np.hstack([np.eye(3), np.zeros((3, 1))])[None], (2, 1, 1))
    d = dataclasses.replace(d, bone_rest=rest, pill_bones=np.tile(np.array([[0, 1]], np.int32), (d.num_pills, 1)),
                            pill_bone_weights=np.stack([1.0 - u, u], 1))
    sc = viper.Scene(d, "f32", device=dev)
    c, sn = np.cos(1e-4), np.sin(1e-4)
    frames = []
    for f in range(calls + 1):
        T = rest.copy()
        T[0, :2, :2] = [[c, -sn], [sn, c]]        # small turns either way keep the scene in place
        T[0, 0, 3] = 1e-5 * (f % 2)
        T[1, 1, 3] = -1e-5 * (f % 2)
        frames.append(T)
    sc.set_bones(frames[0])
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for f in range(1, calls + 1):
        sc.set_bones(frames[f])
    e1.record(st)
    torch.cuda.synchronize()
    sc.sync()
    us = e0.elapsed_time(e1) * 1e3 / calls
    return {"workload": "helix4096x64_two_bones", "pills": d.num_pills, "us_per_call": us,
            "algorithmic_GB_per_s": 52.0 * d.num_pills / (us * 1e-6) / 1e9}


def serving_run(torch, scenes, serve, seconds, plain_limit):
    """Poisson arrivals (200/s) of helix and muscle scenes of 1k-200k pills (log-uniform; muscle
    scenes skinned, 4 mesh vertices per pill), 60 frames each; continuous batching vs the plain
    per-scene path on the same requests (the plain path starts no request after `plain_limit`
    s of wall time).  A scene that diverges is dropped by both paths at the same frame."""
    t0 = time.perf_counter()
    reqs = scenes.serving_requests(rate=200, duration=seconds, seed=3)
    gen_s = time.perf_counter() - t0
    log("serving: %d requests built in %.1f s" % (len(reqs), gen_s))
    b = serve.serve_batched(reqs, pool_bytes=64 << 30, progress=log)
    torch.cuda.synchronize()
    p = serve.serve_plain(reqs, progress=None, time_limit=plain_limit)
    keep = ("frames", "latency_ms_p50", "latency_ms_p99", "ttff_ms_p50", "ttff_ms_p99", "pill_frames_per_s", "wall_s")
    fail = lambda r: {"requests": len(r["failed"]), "kinds": sorted({f["kind"] for f in r["failed"]}),
                      "pills": int(sum(f["pills"] for f in r["failed"]))}
    return {"workload": "poisson200x%.2fs_1k-200k_60frames" % seconds, "requests": len(reqs),
            "pills": int(sum(r.desc.num_pills for r in reqs)),
            "contact_requests": int(sum(r.kind == "muscle" for r in reqs)),
            "skinned_vertices": int(sum(r.mesh.rest_v.shape[0] for r in reqs if r.mesh is not None)),
            "batched": dict({k: b[k] for k in keep + ("steps", "peak_resident_bytes", "per_class", "host_s")},
                            failed=fail(b)),
            "plain": dict({k: p[k] for k in keep + ("requests_served", "requests_not_served")}, failed=fail(p),
                          time_limit_s=plain_limit)}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rods", type=int, default=4096)
    ap.add_argument("--pills", type=int, default=64)
    ap.add_argument("--substeps", type=int, default=20)
    ap.add_argument("--iters", type=int, default=8)
    ap.add_argument("--mode", default="frame", choices=["frame", "substep"])
    ap.add_argument("--cpu-rods", type=int, default=4096)
    ap.add_argument("--cpu-threads", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-contacts", action="store_true")
    ap.add_argument("--no-solvers", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=1.0,
                    help="arrival window of the serving workload (Poisson, 200 requests/s)")
    ap.add_argument("--plain-limit", type=float, default=30.0,
                    help="wall seconds after which the plain serving path starts no further request")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the serving comparison (prints its JSON object)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="instead of the solver, time a plain device copy of this many MiB (the "
                         "reference kernel for scaling HBM byte counters)")
    ap.add_argument("--counter-summaries", nargs=4, metavar=("FETCH_DB", "WRITE_DB", "COPY_FETCH_DB", "COPY_WRITE_DB"),
                    help="write the frame kernel's HBM counter summaries under profiles/ from four rocprofv3 "
                         "--pmc result databases (no GPU needed); --counter-frames and --copy-mib as in those runs")
    ap.add_argument("--counter-frames", type=int, default=4,
                    help="whole-frame launches (warmup + steps) of the counted bench run")
    args = ap.parse_args()
    if args.counter_summaries:
        write_counter_summaries(*args.counter_summaries, frames=args.counter_frames, copy_mib=args.copy_mib or 1024)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X "
              "(rods and scenes are independent; see the sharding note in the design document)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1906_05260_amd import scenes, viper

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_mib:
        print(json.dumps(copy_reference(torch, dev, args.copy_mib, args.steps)), flush=True)
        return
    if args.serve_only:
        from paper_1906_05260_amd import serve
        print(json.dumps(serving_run(torch, scenes, serve, args.serve_seconds, args.plain_limit)), flush=True)
        return
    dt, sub, iters = 1.0 / 60.0, args.substeps, args.iters
    desc = scenes.helix_rods(args.rods, args.pills, seed=1)
    sc = viper.Scene(desc, "f32", device=dev)
    mode = viper.MODE_FRAME if args.mode == "frame" else viper.MODE_SUBSTEP
    for _ in range(args.warmup):
        sc.step(dt, sub, iters, mode=mode)
    sync_diverged(viper, sc, desc)
    stream = torch.cuda.current_stream()
    K = args.steps
    launches = K if mode == viper.MODE_FRAME else K * sub
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(launches)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        if mode == viper.MODE_FRAME:
            ev[k][0].record(stream)
            sc.step(dt, sub, iters, mode=mode)
            ev[k][1].record(stream)
        else:
            for j in range(sub):
                e = ev[k * sub + j]
                e[0].record(stream)
                sc.step(dt / sub, 1, iters, mode=mode)
                e[1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    diverged = sync_diverged(viper, sc, desc)
    kern_ms = sum(a.elapsed_time(b) for a, b in ev) / launches

    P = desc.num_pills
    edges = P - desc.num_rods
    bts = P - 2 * desc.num_rods
    proj_per_frame = sc.projections_per_iteration * iters * sub
    value = proj_per_frame * K / elapsed
    # the same rate split by constraint type (a type counts on the rods whose compliance for it
    # is finite: edges for stretch-shear, volume and scale gradient, interior vertices for
    # bend-twist)
    comp = np.asarray(desc.compliance, float).reshape(-1, 4)
    n_rod = np.diff(np.asarray(desc.rod_offsets))
    per_iter = {t: int(np.sum(np.where(np.isfinite(comp[:, i]), n_rod - (2 if t == "bt" else 1), 0)))
                for i, t in enumerate(("ss", "vol", "sg", "bt"))}
    assert sum(per_iter.values()) == sc.projections_per_iteration
    by_type = {t: v * iters * sub * K / elapsed for t, v in per_iter.items()}
    flop_sub = iters * (edges * (FLOP["ss"] + FLOP["vol"] + FLOP["sg"]) + bts * FLOP["bt"]) + \
        P * (FLOP["predict"] + FLOP["velocity"])
    flop_launch = flop_sub * (sub if mode == viper.MODE_FRAME else 1)
    bytes_launch = BYTES_PER_PILL_LAUNCH * P
    achieved = flop_launch / (kern_ms * 1e-3)
    workload = "helix%dx%d" % (args.rods, args.pills)
    kname = "rod_frame_kernel"
    # the survey's estimate of the work, 2.5-3 kFLOP per pill-substep (midpoint), beside the
    # count from the closed forms above
    flop_survey = SURVEY_FLOP_PER_PILL_SUBSTEP * P * (sub if mode == viper.MODE_FRAME else 1)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VALU, "traffic": measured_traffic(kname + ("" if mode == viper.MODE_FRAME
                                                                                 else "_substep"), workload),
            "kernel": kname, "kernel_ms": kern_ms, "flop_per_launch": flop_launch,
            "frac_at_survey_flop_count": flop_survey / (kern_ms * 1e-3) / PEAK_FP32_VALU,
            "frac_of_packed_fp32_peak": achieved / 157.3e12,
            "algorithmic_bytes_per_launch": bytes_launch,
            "algorithmic_hbm_frac": bytes_launch / (kern_ms * 1e-3) / PEAK_HBM}
    out = {
        "metric": "pill-constraint projections/sec at fixed iters; served p50/p99 frame latency",
        "value": value,
        "unit": "projections/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded random helices)",
        "config": {"workload": workload, "rods": args.rods, "pills_per_rod": args.pills, "substeps": sub,
                   "iterations": iters, "frames_timed": K, "collisions": False, "launch": args.mode,
                   "pill_substeps_per_s": P * sub * K / elapsed, "projections_per_s_by_type": by_type,
                   "rods_nonfinite_at_end": diverged},
        "roofline": roof,
    }
    log("headline: %.3f ms/frame, rod kernel %.3f ms" % (elapsed * 1e3 / K, kern_ms))
    out["single_rod"] = single_rod_timing(torch, viper, scenes, dev)
    if not args.no_contacts:
        out["contacts_skinning"] = contact_skin_timing(torch, viper, scenes, dev)
        out["paper_shaped"] = paper_shaped_timing(torch, viper, scenes, dev)
        log("contacts and skinning done")
        out["bundling"] = bundling_timing(torch, viper, scenes, dev)
        log("bundling done")
    if not args.no_solvers:
        out["solvers"] = solver_timing(torch, viper, scenes, dev)
        log("solvers done")
    out["bones"] = bones_timing(torch, viper, scenes, dev)
    log("bones done")
    out["substep_kernel"] = substep_kernel_timing(torch, viper, scenes, dev)
    log("substep kernel done")
    if not args.no_solvers:
        out["helix_16x"] = large_timing(torch, viper, scenes, dev)
        log("16x helix done")
    if not args.no_adjoint:
        out["adjoint"] = adjoint_timing(torch, viper, scenes, dev)
        log("adjoint done")
    # the measured copy ceiling beside the 8 TB/s specification (1 GiB read + 1 GiB written)
    out["copy_ceiling"] = copy_reference(torch, dev, 1024, 20)
    log("copy ceiling done")
    if not args.no_serve:
        from paper_1906_05260_amd import serve
        out["serving"] = serving_run(torch, scenes, serve, args.serve_seconds, args.plain_limit)
        log("serving done")
        out["latency_ms_p50"] = out["serving"]["batched"]["latency_ms_p50"]
        out["latency_ms_p99"] = out["serving"]["batched"]["latency_ms_p99"]
    if not args.no_cpu:
        threads = max(1, min(args.cpu_threads, os.cpu_count() or 1))
        out["cpu_baseline"] = cpu_baseline(desc, dt, sub, iters, min(args.cpu_rods, desc.num_rods), threads)
        out["cpu_baseline"]["serial"] = cpu_baseline(desc, dt, sub, iters, min(256, desc.num_rods), 1)
        log("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
