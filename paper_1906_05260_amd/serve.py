"""Serving loop: continuous batching of rod scenes on one GPU.

Requests (a scene and a number of frames) arrive over time.  The batched server keeps
every admitted scene resident in one device pool and advances them frame by frame in two
independent classes (one launch for all collision-free scenes, one shared launch sequence
for all scenes with contacts), each class on its own stream.  Requests that arrive while
a step runs are admitted as soon as a slot and a free range of the pool's HBM fit their
footprint; their uploads run on a copy stream and they join their class's next step.  Finished scenes are retired, which frees their
range.  The plain path serves the same requests first-come first-served, one scene at a
time with its own launches, as a baseline.

Muscle requests carry a skinning mesh; both paths skin it after every frame (Sec. 7.4),
on the stream that stepped the scene.  Every finished class step is followed by a check of
its scenes' device-side conditions (non-finite state, diverged contact detection, contact
overflow): a failing scene is retired at once and reported, and its frame is not counted.

Reported per run: frame latency p50/p99 (latency of frame k = completion of frame k minus
the moment it became ready: the arrival for frame 0, the previous frame's completion
after), time to first frame p50/p99, pill-frames/s, peak resident bytes, failed requests.
"""
from __future__ import annotations

import time
from collections import deque

import numpy as np

from . import viper


def _summary(lat, ttff, pill_frames, t_first, t_last, extra=None):
    lat = np.asarray(lat) * 1e3
    ttff = np.asarray(ttff) * 1e3
    span = max(t_last - t_first, 1e-9)
    out = {
        "frames": int(lat.size),
        "latency_ms_p50": float(np.percentile(lat, 50)) if lat.size else None,
        "latency_ms_p99": float(np.percentile(lat, 99)) if lat.size else None,
        "ttff_ms_p50": float(np.percentile(ttff, 50)) if ttff.size else None,
        "ttff_ms_p99": float(np.percentile(ttff, 99)) if ttff.size else None,
        "pill_frames_per_s": pill_frames / span,
        "wall_s": span,
    }
    if extra:
        out.update(extra)
    return out


def serve_batched(requests, pool_bytes, dt=1.0 / 60.0, substeps=20, iterations=8, max_scenes=512,
                  precision="f32", device="cuda:0", on_finish=None, progress=None):
    """Continuous batching over a device pool.

    The collision-free scenes and the scenes with contacts are two classes, each stepped
    one frame at a time on its own stream (viper_pool_step_ex), each with at most one step
    in flight: a collision-free frame (one launch for all of them) does not wait for the
    contact scenes' longer launch sequence.  Arrivals are admitted while steps run (uploads
    on a copy stream) and join their class's next step; a finished scene is retired as soon
    as its class's step completes.  `on_finish(request, scene)` (optional) is called with
    each finished scene before it is retired; `progress(msg)` (optional) receives a line
    every 100 class steps and while a step has run for more than 5 s.  A request whose
    footprint exceeds the whole empty pool raises RuntimeError."""
    import torch
    pool = viper.Pool(pool_bytes, max_scenes=max_scenes, precision=precision, device=device)
    copy_stream = torch.cuda.Stream(device=device)
    # the collision-free class steps on the caller's current stream, the contact class on one
    # more: few streams, so that each keeps a hardware queue of its own
    lanes = {1: {"stream": torch.cuda.current_stream(device), "event": None, "members": []},
             2: {"stream": torch.cuda.Stream(device=device), "event": None, "members": []}}
    lat_cls = {1: [], 2: []}
    pending = deque(sorted(requests, key=lambda r: r.arrival))
    waiting = deque()
    resident = {}                     # slot -> [request, frames done, t_ready, class, skin]
    failed = []
    lat, ttff = [], []
    pill_frames = 0
    peak_bytes = 0
    steps = 0
    host = {"admit_s": 0.0, "step_enqueue_s": 0.0, "gpu_wait_s": 0.0, "retire_s": 0.0}
    t0 = time.perf_counter()
    last_report = [t0]

    def admit_ready():
        nonlocal peak_bytes
        ta = time.perf_counter()
        now = ta - t0
        while pending and pending[0].arrival <= now:
            waiting.append(pending.popleft())
        while waiting:
            r = waiting[0]
            slot = pool.admit(r.desc, stream=copy_stream)
            if slot is None:
                if not resident and all(lanes[c]["event"] is None for c in (1, 2)):
                    raise RuntimeError("request of %d pills does not fit the empty pool (%d bytes)" %
                                       (r.desc.num_pills, pool_bytes))
                break
            waiting.popleft()
            skin = None
            if getattr(r, "mesh", None) is not None:
                sc = pool.scene(slot)
                sid = sc.create_skin(r.mesh.rest_v, r.mesh.caps, r.mesh.w, stream=copy_stream)
                skin = (sc, sid, torch.empty((r.mesh.rest_v.shape[0], 3), dtype=torch.float32, device=device))
            resident[slot] = [r, 0, r.arrival, 2 if r.desc.collisions else 1, skin]
        info = pool.info()
        peak_bytes = max(peak_bytes, pool_bytes - info["free_bytes"])
        host["admit_s"] += time.perf_counter() - ta

    def launch(cls):
        nonlocal steps
        lane = lanes[cls]
        members = [k for k, v in resident.items() if v[3] == cls]
        if not members:
            return
        ts = time.perf_counter()
        pool.step(dt, substeps, iterations, stream=lane["stream"], classes=cls)
        for k in members:                               # skinning of each stepped mesh (Sec. 7.4)
            sk = resident[k][4]
            if sk is not None:
                sk[0].skin(sk[1], out=sk[2], stream=lane["stream"])
        ev = torch.cuda.Event()
        ev.record(lane["stream"])
        host["step_enqueue_s"] += time.perf_counter() - ts
        lane["event"], lane["members"] = ev, members
        lane["t0"] = time.perf_counter()
        steps += 1
        now = time.perf_counter()
        # every 100 class steps, and at least every 5 s while steps are slow
        if progress is not None and (steps % 100 == 0 or now - last_report[0] > 5.0):
            last_report[0] = now
            progress("batched: %d class steps (class %d, %d scenes in it), %d resident, %d waiting, %d pending, "
                     "t=%.2fs" % (steps, cls, len(members), len(resident), len(waiting), len(pending), now - t0))

    def complete(cls):
        nonlocal pill_frames
        lane = lanes[cls]
        t_done = time.perf_counter() - t0
        for slot in lane["members"]:
            st = resident[slot]
            r = st[0]
            code = pool.status(slot)      # this step has completed: its status copy has landed
            if code != viper.OK:
                failed.append({"arrival": r.arrival, "kind": r.kind, "pills": r.desc.num_pills,
                               "frames_done": st[1], "status": code})
                if progress is not None:
                    progress("batched: %s request of %d pills failed at frame %d (status %d)" %
                             (r.kind, r.desc.num_pills, st[1], code))
                pool.retire(slot, stream=lane["stream"])
                del resident[slot]
                continue
            lat.append(t_done - st[2])
            lat_cls[cls].append(t_done - st[2])
            if st[1] == 0:
                ttff.append(t_done - r.arrival)
            st[1] += 1
            st[2] = t_done
            pill_frames += r.desc.num_pills
            if st[1] == r.frames:
                if on_finish is not None:
                    on_finish(r, pool.scene(slot))
                tr = time.perf_counter()
                pool.retire(slot, stream=lane["stream"])
                host["retire_s"] += time.perf_counter() - tr
                del resident[slot]
        lane["event"], lane["members"] = None, []

    while pending or waiting or resident:
        admit_ready()
        for cls in (1, 2):
            if lanes[cls]["event"] is None:
                launch(cls)
        busy = [c for c in (1, 2) if lanes[c]["event"] is not None]
        if not busy:
            if pending:
                time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - t0)))
            continue
        done = [c for c in busy if lanes[c]["event"].query()]
        if not done:
            tw = time.perf_counter()
            time.sleep(20e-6)
            host["gpu_wait_s"] += time.perf_counter() - tw
            if progress is not None and tw - last_report[0] > 5.0:
                last_report[0] = tw
                progress("batched: waiting on %s, in flight for %.1f s; %d resident, %d waiting, %d pending, "
                         "t=%.2fs" % (", ".join("class %d (%d scenes)" % (c, len(lanes[c]["members"])) for c in busy),
                                      max(tw - lanes[c]["t0"] for c in busy), len(resident), len(waiting),
                                      len(pending), tw - t0))
            continue
        for c in done:
            complete(c)
    t_last = time.perf_counter() - t0
    t_first = min(r.arrival for r in requests) if requests else 0.0
    per_class = {}
    for cls, name in ((1, "collision_free"), (2, "contacts")):
        v = np.asarray(lat_cls[cls]) * 1e3
        per_class[name] = {"frames": int(v.size),
                           "latency_ms_p50": float(np.percentile(v, 50)) if v.size else None,
                           "latency_ms_p99": float(np.percentile(v, 99)) if v.size else None}
    return _summary(lat, ttff, pill_frames, t_first, t_last,
                    {"path": "batched", "steps": steps, "peak_resident_bytes": int(peak_bytes),
                     "per_class": per_class, "host_s": {k: round(v, 4) for k, v in host.items()},
                     "failed": failed})


def serve_plain(requests, dt=1.0 / 60.0, substeps=20, iterations=8, precision="f32", device="cuda:0",
                on_finish=None, progress=None, time_limit=None):
    """First-come first-served, one scene at a time: one viper_step per frame, then the skinning
    of its mesh, then viper_sync (which waits for the frame and reads its status; a failing
    scene is dropped and reported).  With `time_limit` (s of wall time) no further request is
    started after that point; those left are reported as not served."""
    import torch
    lat, ttff = [], []
    failed = []
    pill_frames = 0
    reqs = sorted(requests, key=lambda r: r.arrival)
    served = 0
    t0 = time.perf_counter()
    for r in reqs:
        now = time.perf_counter() - t0
        if time_limit is not None and now > time_limit:
            break
        if now < r.arrival:
            time.sleep(r.arrival - now)
        sc = viper.Scene(r.desc, precision, device=device)
        skin = None
        if getattr(r, "mesh", None) is not None:
            sid = sc.create_skin(r.mesh.rest_v, r.mesh.caps, r.mesh.w)
            skin = (sid, torch.empty((r.mesh.rest_v.shape[0], 3), dtype=torch.float32, device=device))
        t_ready = r.arrival
        for k in range(r.frames):
            sc.step(dt, substeps, iterations)
            if skin is not None:
                sc.skin(skin[0], out=skin[1])
            try:
                sc.sync()
            except viper.ViperError as e:
                failed.append({"arrival": r.arrival, "kind": r.kind, "pills": r.desc.num_pills, "frames_done": k,
                               "status": e.status})
                break
            t_done = time.perf_counter() - t0
            lat.append(t_done - t_ready)
            if k == 0:
                ttff.append(t_done - r.arrival)
            t_ready = t_done
            pill_frames += r.desc.num_pills
        served += 1
        if on_finish is not None:
            on_finish(r, sc)
        del sc
        if progress is not None:
            progress("plain: request done (%d pills), t=%.2fs" % (r.desc.num_pills, time.perf_counter() - t0))
    t_last = time.perf_counter() - t0
    t_first = min(r.arrival for r in requests) if requests else 0.0
    return _summary(lat, ttff, pill_frames, t_first, t_last,
                    {"path": "plain", "failed": failed, "requests_served": served,
                     "requests_not_served": len(reqs) - served})
