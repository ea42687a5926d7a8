"""ctypes binding of libviper.so (include/viper.h): argument marshalling only.

Every step of the solver runs in the HIP kernels of ``csrc/``; PyTorch only
provides the device workspace and the stream.  Importing this module on a
machine where the library is missing raises immediately -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libviper.so")

OK, ERR_INVALID, ERR_NO_CAPACITY, ERR_CAPACITY, ERR_NAN, ERR_DEVICE = range(6)
F32, F64 = 0, 1
MODE_AUTO, MODE_FRAME, MODE_SUBSTEP, MODE_ITERATION, MODE_GRAPH = range(5)
X, V, S, SDOT, Q, OMEGA, RADIUS, XDET, SDET, XLOCAL = range(10)
FIELD_WIDTH = {X: 3, V: 3, S: 1, SDOT: 1, Q: 4, OMEGA: 3, RADIUS: 1, XDET: 3, SDET: 1, XLOCAL: 3}
FIELD_NAMES = {"x": X, "v": V, "s": S, "sd": SDOT, "q": Q, "om": OMEGA, "radius": RADIUS, "xdet": XDET,
               "sdet": SDET, "xlocal": XLOCAL}
# fields that restore a scene exactly (bit for bit)
CHECKPOINT_FIELDS = ("xlocal", "v", "s", "sd", "q", "om")

# Every symbol declared in include/viper.h.
ABI_SYMBOLS = [
    "viper_scene_footprint", "viper_create_scene", "viper_step", "viper_step_ex", "viper_get_state",
    "viper_set_state", "viper_get_contacts", "viper_create_skin", "viper_skin", "viper_sync",
    "viper_destroy_scene", "viper_scene_info", "viper_last_error",
    "viper_pool_create", "viper_pool_admit", "viper_pool_step", "viper_pool_retire", "viper_pool_scene",
    "viper_pool_info", "viper_pool_destroy",
    "viper_adjoint_sizes", "viper_step_checkpointed", "viper_step_backward", "viper_pool_step_ex",
    "viper_skin_weights", "viper_set_bones", "viper_set_floor", "viper_contact_stats", "viper_pool_status", "viper_step_backward_static",
    "viper_skin_fair_work_bytes", "viper_skin_weights_faired",
]


class ViperError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("viper status %d: %s" % (status, msg))
        self.status = status


class SceneDescC(ctypes.Structure):
    _fields_ = [
        ("num_rods", ctypes.c_int32),
        ("rod_offsets", ctypes.c_void_p),
        ("rest_pos", ctypes.c_void_p),
        ("rest_radius", ctypes.c_void_p),
        ("pinned", ctypes.c_void_p),
        ("activation", ctypes.c_void_p),
        ("compliance", ctypes.c_void_p),
        ("group", ctypes.c_void_p),
        ("density", ctypes.c_double),
        ("gravity", ctypes.c_double * 3),
        ("precision", ctypes.c_int32),
        ("collisions", ctypes.c_int32),
        ("contact_capacity_per_capsule", ctypes.c_int32),
        ("num_sections", ctypes.c_int32),
        ("section_offsets", ctypes.c_void_p),
        ("section_pills", ctypes.c_void_p),
        ("floor_on", ctypes.c_int32),
        ("floor_normal", ctypes.c_double * 3),
        ("floor_offset", ctypes.c_double),
        ("solver", ctypes.c_int32),
        ("cross_compliance", ctypes.c_void_p),
        ("num_bones", ctypes.c_int32),
        ("bone_rest", ctypes.c_void_p),
        ("pill_bones", ctypes.c_void_p),
        ("pill_bone_weights", ctypes.c_void_p),
        ("bending_compliance", ctypes.c_void_p),
        ("volume_bending", ctypes.c_int32),
    ]


class ContactInfoC(ctypes.Structure):
    """Mirror of viper_contact_info."""
    _fields_ = [
        ("walk_entries", ctypes.c_int64),
        ("oversized", ctypes.c_int32),
        ("excluded", ctypes.c_int32),
        ("skipped", ctypes.c_int32),
        ("cell_bin", ctypes.c_int32),
        ("cell_width", ctypes.c_double),
        ("cell_radius_limit", ctypes.c_double),
        ("coarse_bin", ctypes.c_int32),
        ("coarse_capsules", ctypes.c_int32),
        ("coarse_width", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libviper.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, I32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        for name in ABI_SYMBOLS:
            getattr(L, name).restype = ctypes.c_int
        L.viper_last_error.restype = ctypes.c_char_p
        L.viper_scene_footprint.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
        L.viper_create_scene.argtypes = [P, P, ctypes.c_size_t, P, ctypes.POINTER(P)]
        L.viper_step.argtypes = [P, D, I32, I32, P]
        L.viper_step_ex.argtypes = [P, D, I32, I32, I32, P]
        L.viper_get_state.argtypes = [P, I32, P, P]
        L.viper_set_state.argtypes = [P, I32, P, P]
        L.viper_get_contacts.argtypes = [P, P, I32, ctypes.POINTER(I32), P]
        L.viper_create_skin.argtypes = [P, I32, P, P, P, P, ctypes.POINTER(I32)]
        L.viper_skin.argtypes = [P, I32, P, P]
        L.viper_sync.argtypes = [P, P]
        L.viper_destroy_scene.argtypes = [P]
        L.viper_scene_info.argtypes = [P] + [ctypes.POINTER(ctypes.c_int64)] * 4
        L.viper_pool_create.argtypes = [P, ctypes.c_size_t, I32, I32, P, ctypes.POINTER(P)]
        L.viper_pool_admit.argtypes = [P, P, P, ctypes.POINTER(I32)]
        L.viper_pool_step.argtypes = [P, D, I32, I32, P]
        L.viper_pool_step_ex.argtypes = [P, D, I32, I32, I32, P]
        L.viper_pool_retire.argtypes = [P, I32, P]
        L.viper_pool_scene.argtypes = [P, I32, ctypes.POINTER(P)]
        L.viper_pool_info.argtypes = [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                      ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_int64)]
        L.viper_pool_destroy.argtypes = [P]
        SZ = ctypes.c_size_t
        L.viper_adjoint_sizes.argtypes = [P, I32, I32, I32, ctypes.POINTER(SZ), ctypes.POINTER(SZ)]
        L.viper_step_checkpointed.argtypes = [P, D, I32, I32, I32, P, SZ, P]
        L.viper_step_backward.argtypes = [P, D, I32, I32, I32, P, P, P, SZ, P, P, P]
        L.viper_contact_stats.argtypes = [P, ctypes.POINTER(ContactInfoC), P]
        L.viper_step_backward_static.argtypes = [P, D, I32, I32, I32, P, P, P, P, P]
        L.viper_skin_fair_work_bytes.argtypes = [I32, I32, P, ctypes.POINTER(ctypes.c_size_t)]
        L.viper_skin_weights_faired.argtypes = [P, I32, P, I32, P, I32, D, P, ctypes.c_size_t, P, P, P]
        L.viper_pool_status.argtypes = [P, I32, ctypes.POINTER(I32)]
        _lib = L
    return _lib


def check(status):
    if status != OK:
        raise ViperError(status, lib().viper_last_error().decode())


class _DescHolder:
    """Keeps the numpy arrays behind a SceneDescC alive."""

    def __init__(self, desc, precision, collisions=None, capacity=16):
        self.arrays = dict(
            off=np.ascontiguousarray(desc.rod_offsets, np.int32),
            pos=np.ascontiguousarray(desc.rest_pos, np.float64).reshape(-1),
            rad=np.ascontiguousarray(desc.rest_radius, np.float64),
            pin=np.ascontiguousarray(desc.pinned, np.uint8),
            act=np.ascontiguousarray(desc.activation, np.float64),
            comp=np.ascontiguousarray(desc.compliance, np.float64).reshape(-1),
            grp=np.ascontiguousarray(desc.group, np.int32),
        )
        a = self.arrays
        c = SceneDescC()
        c.num_rods = int(desc.num_rods)
        c.rod_offsets = a["off"].ctypes.data
        c.rest_pos = a["pos"].ctypes.data
        c.rest_radius = a["rad"].ctypes.data
        c.pinned = a["pin"].ctypes.data
        c.activation = a["act"].ctypes.data
        c.compliance = a["comp"].ctypes.data
        c.group = a["grp"].ctypes.data
        c.density = float(desc.density)
        for i in range(3):
            c.gravity[i] = float(desc.gravity[i])
        c.precision = F64 if precision in ("f64", F64) else F32
        c.collisions = int(bool(desc.collisions if collisions is None else collisions))
        c.contact_capacity_per_capsule = int(capacity)
        if getattr(desc, "section_offsets", None) is not None:
            a["soff"] = np.ascontiguousarray(desc.section_offsets, np.int32)
            a["spill"] = np.ascontiguousarray(desc.section_pills, np.int32)
            c.num_sections = int(a["soff"].shape[0] - 1)
            c.section_offsets = a["soff"].ctypes.data
            c.section_pills = a["spill"].ctypes.data
        if getattr(desc, "floor", None) is not None:
            c.floor_on = 1
            for i in range(3):
                c.floor_normal[i] = float(desc.floor[i])
            c.floor_offset = float(desc.floor[3])
        c.solver = 1 if getattr(desc, "solver", "gauss_seidel") == "jacobi" else 0
        if getattr(desc, "cross_compliance", None) is not None:
            a["sr"] = np.ascontiguousarray(desc.cross_compliance, np.float64).reshape(-1)
            if a["sr"].shape[0] != c.num_rods:
                raise ValueError("cross_compliance needs one value per rod")
            c.cross_compliance = a["sr"].ctypes.data
        if getattr(desc, "bone_rest", None) is not None:
            a["brest"] = np.ascontiguousarray(desc.bone_rest, np.float64).reshape(-1)
            a["pbone"] = np.ascontiguousarray(desc.pill_bones, np.int32).reshape(-1)
            a["pbw"] = np.ascontiguousarray(desc.pill_bone_weights, np.float64).reshape(-1)
            if a["brest"].shape[0] % 12 or a["pbone"].shape[0] != 2 * desc.num_pills or \
                    a["pbw"].shape[0] != 2 * desc.num_pills:
                raise ValueError("bone_rest needs [nb, 3, 4]; pill_bones and pill_bone_weights [P, 2]")
            c.num_bones = a["brest"].shape[0] // 12
            c.bone_rest = a["brest"].ctypes.data
            c.pill_bones = a["pbone"].ctypes.data
            c.pill_bone_weights = a["pbw"].ctypes.data
        if getattr(desc, "bending_compliance", None) is not None:
            a["sb"] = np.ascontiguousarray(desc.bending_compliance, np.float64).reshape(-1)
            if a["sb"].shape[0] != c.num_rods:
                raise ValueError("bending_compliance needs one value per rod")
            c.bending_compliance = a["sb"].ctypes.data
        c.volume_bending = 1 if getattr(desc, "volume_bending", False) else 0
        self.c = c


def footprint(desc, precision="f32", collisions=None, capacity=16) -> int:
    h = _DescHolder(desc, precision, collisions, capacity)
    n = ctypes.c_size_t(0)
    check(lib().viper_scene_footprint(ctypes.byref(h.c), ctypes.byref(n)))
    return int(n.value)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Scene:
    """A VIPER scene resident in one device workspace (a torch uint8 tensor)."""

    def __init__(self, desc, precision="f32", device="cuda:0", collisions=None, capacity=16, stream=None,
                 workspace=None):
        import torch
        self.desc = desc
        self.precision = F64 if precision in ("f64", F64) else F32
        self.dtype = torch.float64 if self.precision == F64 else torch.float32
        self.device = torch.device(device)
        h = _DescHolder(desc, precision, collisions, capacity)
        nbytes = ctypes.c_size_t(0)
        check(lib().viper_scene_footprint(ctypes.byref(h.c), ctypes.byref(nbytes)))
        self.nbytes = int(nbytes.value)
        if workspace is None:
            workspace = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=self.device)
        self.workspace = workspace
        handle = ctypes.c_void_p()
        check(lib().viper_create_scene(ctypes.byref(h.c), ctypes.c_void_p(workspace.data_ptr()),
                                       ctypes.c_size_t(workspace.numel()), _stream_ptr(stream),
                                       ctypes.byref(handle)))
        self.handle = handle
        self.P = int(desc.num_pills)
        self.num_rods = int(desc.num_rods)
        self._skins = []
        pills, rods, caps, ppi = (ctypes.c_int64() for _ in range(4))
        check(lib().viper_scene_info(self.handle, ctypes.byref(pills), ctypes.byref(rods), ctypes.byref(caps),
                                     ctypes.byref(ppi)))
        self.capsules = int(caps.value)
        self.projections_per_iteration = int(ppi.value)

    @classmethod
    def attach(cls, handle, desc, precision, device):
        """Wrap a scene handle owned elsewhere (a pool slot); it is not destroyed here."""
        import torch
        self = cls.__new__(cls)
        self.desc = desc
        self.precision = F64 if precision in ("f64", F64) else F32
        self.dtype = torch.float64 if self.precision == F64 else torch.float32
        self.device = torch.device(device)
        self.handle = handle
        self._owned = False
        self.P = int(desc.num_pills)
        self.num_rods = int(desc.num_rods)
        self._skins = []
        pills, rods, caps, ppi = (ctypes.c_int64() for _ in range(4))
        check(lib().viper_scene_info(self.handle, ctypes.byref(pills), ctypes.byref(rods), ctypes.byref(caps),
                                     ctypes.byref(ppi)))
        self.capsules = int(caps.value)
        self.projections_per_iteration = int(ppi.value)
        return self

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and getattr(self, "_owned", True):
            try:
                lib().viper_destroy_scene(h)
            except Exception:
                pass
            self.handle = None

    def step(self, dt, substeps, iterations, mode=MODE_AUTO, stream=None):
        check(lib().viper_step_ex(self.handle, float(dt), int(substeps), int(iterations), int(mode),
                                  _stream_ptr(stream)))

    def get(self, which, stream=None):
        import torch
        which = FIELD_NAMES.get(which, which)
        dtype = torch.float64 if which == XDET else self.dtype
        out = torch.empty((self.P, FIELD_WIDTH[which]), dtype=dtype, device=self.device)
        check(lib().viper_get_state(self.handle, int(which), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out if FIELD_WIDTH[which] > 1 else out.view(-1)

    def set(self, which, values, stream=None):
        import torch
        which = FIELD_NAMES.get(which, which)
        t = torch.as_tensor(values).to(device=self.device, dtype=self.dtype).contiguous()
        assert t.numel() == self.P * FIELD_WIDTH[which]
        check(lib().viper_set_state(self.handle, int(which), ctypes.c_void_p(t.data_ptr()), _stream_ptr(stream)))
        self._keep_alive = t

    def state(self, local=False):
        """All state fields as float64 numpy arrays (synchronises).  With local=True the
        positions are the stored rod-anchor-relative values (key "x")."""
        import torch
        out = {k: self.get(k) for k in ("x", "v", "s", "sd", "q", "om")}
        if local:
            out["x"] = self.get("xlocal")
        torch.cuda.synchronize(self.device)
        return {k: v.double().cpu().numpy() for k, v in out.items()}

    def contacts(self, stream=None):
        n = ctypes.c_int32(0)
        st = lib().viper_get_contacts(self.handle, None, 0, ctypes.byref(n), _stream_ptr(stream))
        if st not in (OK, ERR_NO_CAPACITY):
            check(st)
        out = np.zeros((max(int(n.value), 1), 2), np.int32)
        check(lib().viper_get_contacts(self.handle, ctypes.c_void_p(out.ctypes.data), int(out.shape[0]),
                                       ctypes.byref(n), _stream_ptr(stream)))
        return out[: int(n.value)].copy()

    def contact_stats(self, stream=None):
        """Record of the last contact detection (include/viper.h, viper_contact_info) as a dict
        (synchronises)."""
        c = ContactInfoC()
        check(lib().viper_contact_stats(self.handle, ctypes.byref(c), _stream_ptr(stream)))
        return {name: getattr(c, name) for name, _ in ContactInfoC._fields_}

    def create_skin(self, rest_v, caps, w, stream=None):
        import torch
        rv = torch.as_tensor(rest_v, dtype=torch.float32).to(self.device).contiguous()
        cp = torch.as_tensor(caps, dtype=torch.int32).to(self.device).contiguous()
        ww = torch.as_tensor(w, dtype=torch.float32).to(self.device).contiguous()
        sid = ctypes.c_int32(-1)
        check(lib().viper_create_skin(self.handle, int(rv.shape[0]), ctypes.c_void_p(rv.data_ptr()),
                                      ctypes.c_void_p(cp.data_ptr()), ctypes.c_void_p(ww.data_ptr()),
                                      _stream_ptr(stream), ctypes.byref(sid)))
        self._skins.append((rv, cp, ww))
        return int(sid.value)

    def skin(self, skin_id, out=None, stream=None):
        import torch
        V = int(self._skins[skin_id][0].shape[0])
        if out is None:
            out = torch.empty((V, 3), dtype=torch.float32, device=self.device)
        check(lib().viper_skin(self.handle, int(skin_id), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def skin_weights(self, rest_v, stream=None):
        """Initial skinning weights (include/viper.h, viper_skin_weights) of rest vertices at the
        scene's current pose: (capsule ids [V,4] int32, weights [V,4] float32) device tensors."""
        import torch
        rv = torch.as_tensor(rest_v, dtype=torch.float32).to(self.device).contiguous()
        V = int(rv.shape[0])
        caps = torch.empty((V, 4), dtype=torch.int32, device=self.device)
        w = torch.empty((V, 4), dtype=torch.float32, device=self.device)
        check(lib().viper_skin_weights(self.handle, V, ctypes.c_void_p(rv.data_ptr()), ctypes.c_void_p(caps.data_ptr()),
                                       ctypes.c_void_p(w.data_ptr()), _stream_ptr(stream)))
        self._keep_alive = rv
        return caps, w

    def skin_weights_faired(self, rest_v, tris, iterations, lam=0.5, stream=None):
        """Skinning weights faired over the mesh (include/viper.h, viper_skin_weights_faired):
        (capsule ids [V,4] int32, weights [V,4] float32) device tensors (synchronises)."""
        import torch
        rv = torch.as_tensor(rest_v, dtype=torch.float32).to(self.device).contiguous()
        V = int(rv.shape[0])
        t = np.ascontiguousarray(tris, np.int32).reshape(-1, 3)
        nb = ctypes.c_size_t(0)
        check(lib().viper_skin_fair_work_bytes(V, int(t.shape[0]), ctypes.c_void_p(t.ctypes.data), ctypes.byref(nb)))
        work = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=self.device)
        caps = torch.empty((V, 4), dtype=torch.int32, device=self.device)
        w = torch.empty((V, 4), dtype=torch.float32, device=self.device)
        check(lib().viper_skin_weights_faired(self.handle, V, ctypes.c_void_p(rv.data_ptr()), int(t.shape[0]),
                                              ctypes.c_void_p(t.ctypes.data), int(iterations), float(lam),
                                              ctypes.c_void_p(work.data_ptr()), ctypes.c_size_t(work.numel()),
                                              ctypes.c_void_p(caps.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                              _stream_ptr(stream)))
        return caps, w

    def set_floor(self, plane, stream=None):
        """Move the floor (include/viper.h, viper_set_floor) to plane = (nx, ny, nz, d)."""
        n = np.ascontiguousarray(plane[:3], np.float64)
        check(lib().viper_set_floor(self.handle, ctypes.c_void_p(n.ctypes.data), ctypes.c_double(float(plane[3])),
                                    _stream_ptr(stream)))

    def set_bones(self, transforms, stream=None):
        """The bones' transforms of a new frame, [nb, 3, 4] (include/viper.h, viper_set_bones):
        every pill with bone weight moves by the blend of its bones' motions (Sec. 8.2)."""
        t = np.ascontiguousarray(transforms, np.float64).reshape(-1)
        check(lib().viper_set_bones(self.handle, ctypes.c_void_p(t.ctypes.data), _stream_ptr(stream)))

    def sync(self, stream=None):
        check(lib().viper_sync(self.handle, _stream_ptr(stream)))

    # ---- adjoint (include/viper.h, viper_adjoint_sizes / viper_step_checkpointed / viper_step_backward)

    def adjoint_sizes(self, frames, substeps, iterations):
        c, w = ctypes.c_size_t(0), ctypes.c_size_t(0)
        check(lib().viper_adjoint_sizes(self.handle, int(frames), int(substeps), int(iterations), ctypes.byref(c),
                                        ctypes.byref(w)))
        return int(c.value), int(w.value)

    def step_checkpointed(self, dt, frames, substeps, iterations, ckpt=None, stream=None):
        """Advance ``frames`` frames (FRAME mode) writing the per-substep checkpoint; returns it."""
        import torch
        nc, _ = self.adjoint_sizes(frames, substeps, iterations)
        if ckpt is None:
            ckpt = torch.empty(max(nc, 1), dtype=torch.uint8, device=self.device)
        check(lib().viper_step_checkpointed(self.handle, float(dt), int(frames), int(substeps), int(iterations),
                                            ctypes.c_void_p(ckpt.data_ptr()), ctypes.c_size_t(ckpt.numel()),
                                            _stream_ptr(stream)))
        return ckpt

    def backward(self, dt, frames, substeps, iterations, ckpt, dl_dx, work=None, stream=None):
        """(dL/d rest radius [P], dL/d activation [R]) as float64 device tensors."""
        import torch
        _, nw = self.adjoint_sizes(frames, substeps, iterations)
        if work is None:
            work = torch.empty(max(nw, 1), dtype=torch.uint8, device=self.device)
        g = torch.as_tensor(dl_dx).to(device=self.device, dtype=self.dtype).contiguous()
        assert g.numel() == 3 * self.P
        drbar = torch.empty(self.P, dtype=torch.float64, device=self.device)
        dact = torch.empty(self.num_rods, dtype=torch.float64, device=self.device)
        check(lib().viper_step_backward(self.handle, float(dt), int(frames), int(substeps), int(iterations),
                                        ctypes.c_void_p(ckpt.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                        ctypes.c_void_p(work.data_ptr()), ctypes.c_size_t(work.numel()),
                                        ctypes.c_void_p(drbar.data_ptr()), ctypes.c_void_p(dact.data_ptr()),
                                        _stream_ptr(stream)))
        self._keep_alive = (g, work)
        return drbar, dact


def backward_static(scene, dt, frames, substeps, iterations, ckpt, dl_dx, stream=None):
    """viper_step_backward_static (no work buffer; the library's static scratch): (dL/d rest
    radius [P], dL/d activation [R]) as float64 device tensors."""
    import torch
    g = torch.as_tensor(dl_dx).to(device=scene.device, dtype=scene.dtype).contiguous()
    assert g.numel() == 3 * scene.P
    drbar = torch.empty(scene.P, dtype=torch.float64, device=scene.device)
    dact = torch.empty(scene.num_rods, dtype=torch.float64, device=scene.device)
    check(lib().viper_step_backward_static(scene.handle, float(dt), int(frames), int(substeps), int(iterations),
                                           ctypes.c_void_p(ckpt.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                           ctypes.c_void_p(drbar.data_ptr()), ctypes.c_void_p(dact.data_ptr()),
                                           _stream_ptr(stream)))
    scene._keep_alive = g
    return drbar, dact


class Pool:
    """A serving pool (include/viper.h, viper_pool_*) over one torch workspace."""

    def __init__(self, nbytes, max_scenes=256, precision="f32", device="cuda:0", stream=None):
        import torch
        self.device = torch.device(device)
        self.precision = precision
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        check(lib().viper_pool_create(ctypes.c_void_p(self.workspace.data_ptr()), ctypes.c_size_t(int(nbytes)),
                                      int(max_scenes), F64 if precision in ("f64", F64) else F32,
                                      _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h
        self.descs = {}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                lib().viper_pool_destroy(h)
            except Exception:
                pass
            self.handle = None

    def admit(self, desc, stream=None, capacity=16):
        """Slot id, or None when the pool has no room (VIPER_ERR_NO_CAPACITY)."""
        hd = _DescHolder(desc, self.precision, None, capacity)
        slot = ctypes.c_int32(-1)
        st = lib().viper_pool_admit(self.handle, ctypes.byref(hd.c), _stream_ptr(stream), ctypes.byref(slot))
        if st == ERR_NO_CAPACITY:
            return None
        check(st)
        self.descs[int(slot.value)] = desc
        return int(slot.value)

    def step(self, dt, substeps, iterations, stream=None, classes=None):
        """One frame of every resident scene (classes=None), or of one class: 1 = collision-free,
        2 = with contacts, 3 = both on `stream`."""
        if classes is None:
            check(lib().viper_pool_step(self.handle, float(dt), int(substeps), int(iterations), _stream_ptr(stream)))
        else:
            check(lib().viper_pool_step_ex(self.handle, float(dt), int(substeps), int(iterations), int(classes),
                                           _stream_ptr(stream)))

    def retire(self, slot, stream=None):
        check(lib().viper_pool_retire(self.handle, int(slot), _stream_ptr(stream)))
        self.descs.pop(int(slot), None)

    def status(self, slot):
        """Condition of a resident scene as of its class's last completed step (include/viper.h,
        viper_pool_status): OK, ERR_NAN or ERR_CAPACITY; no synchronisation."""
        v = ctypes.c_int32(-1)
        check(lib().viper_pool_status(self.handle, int(slot), ctypes.byref(v)))
        return int(v.value)

    def scene(self, slot):
        h = ctypes.c_void_p()
        check(lib().viper_pool_scene(self.handle, int(slot), ctypes.byref(h)))
        return Scene.attach(h, self.descs[int(slot)], self.precision, self.device)

    def info(self):
        fb, lf = ctypes.c_size_t(), ctypes.c_size_t()
        n, pills = ctypes.c_int32(), ctypes.c_int64()
        check(lib().viper_pool_info(self.handle, ctypes.byref(fb), ctypes.byref(lf), ctypes.byref(n),
                                    ctypes.byref(pills)))
        return dict(free_bytes=int(fb.value), largest_free=int(lf.value), resident=int(n.value),
                    resident_pills=int(pills.value))
