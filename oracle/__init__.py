"""VIPER rod-solver ORACLE -- test infrastructure only.

ctypes binding of ``viper_oracle.cpp``: a serial CPU implementation of the
VIPER substep (Sec. 6 prediction and per-constraint dual update, Sec. 5
energies as constraints, Sec. 7 collision handling and skinning), templated on
FP64 (reference), FP32 (rounding floor) and dual numbers (gradients).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "viper_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, no FP contraction, no intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-ffp-contract=off", "-std=c++17", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        D = ctypes.c_double
        I = ctypes.c_int
        L.orc_create.restype = P
        L.orc_create.argtypes = [I, I, P, P, P, P, P, P, P, D, P]
        L.orc_destroy.argtypes = [P]
        L.orc_set_state.argtypes = [P] * 7
        L.orc_get_state.argtypes = [P] * 7
        L.orc_step.restype = ctypes.c_int64
        L.orc_step.argtypes = [P, D, I, I, I, I, D, I]
        L.orc_get_rest.argtypes = [P] * 9
        L.orc_project_one.argtypes = [P, I, I, D]
        L.orc_substep_residuals.argtypes = [P, D, I, P]
        L.orc_num_pairs.restype = I
        L.orc_num_pairs.argtypes = [P]
        L.orc_get_pairs.argtypes = [P, P]
        L.orc_get_active_count.argtypes = [P, P]
        L.orc_brute_pairs.restype = I
        L.orc_brute_pairs.argtypes = [I, P, P, P, P, P, P, I]
        L.orc_pill_project.restype = D
        L.orc_pill_project.argtypes = [P, P, D, P, D]
        L.orc_coll_gap.restype = D
        L.orc_coll_gap.argtypes = [P, D, P, D, P, D, P, D, D]
        L.orc_dichotomous.restype = D
        L.orc_dichotomous.argtypes = [P, D, P, D, P, D, P, D, I, D]
        L.orc_skin.argtypes = [P, I, P, P, P, P]
        L.orc_capsule_transforms.argtypes = [P, P]
        L.orc_set_masses.argtypes = [P, P, P, P]
        L.orc_contact_pass.argtypes = [P, I, D]
        L.orc_set_sections.argtypes = [P, I, P, P]
        L.orc_set_floor.argtypes = [P, P, D]
        L.orc_floor_pass.argtypes = [P]
        L.orc_set_solver.argtypes = [P, I]
        L.orc_set_cross_stretch.argtypes = [P, P]
        L.orc_set_surface_bending.argtypes = [P, P]
        L.orc_set_volume_bending.argtypes = [P, I]
        L.orc_set_bones.argtypes = [P, I, P, P, P]
        L.orc_bone_frame.argtypes = [P, P]
        L.orc_skin_weights.argtypes = [P, I, P, P, P]
        L.orc_skin_weights_faired.argtypes = [P, I, P, I, P, I, D, P, P]
        L.orc_rod_iteration.restype = ctypes.c_int64
        L.orc_rod_iteration.argtypes = [P, D, I]
        L.orc_section_fit.argtypes = [P, I, P]
        L.orc_bundle.argtypes = [P]
        L.orc_extract_rotation.argtypes = [P, P, P]
        L.orc_grad.restype = D
        L.orc_grad.argtypes = [I, P, P, P, P, P, P, P, D, P, D, I, I, I, P, P, P, I, I]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def extract_rotation(A, q0=(0.0, 0.0, 0.0, 1.0)):
    """The oracle's rotation extraction (Mueller et al. 2016 iteration) of a 3x3 matrix."""
    A = np.ascontiguousarray(A, dtype=np.float64).reshape(9)
    q0 = np.ascontiguousarray(q0, dtype=np.float64)
    q = np.zeros(4)
    lib().orc_extract_rotation(_p(A), _p(q0), _p(q))
    return q


class OracleScene:
    """One oracle scene (precision 'f64' or 'f32') built from a scene description."""

    def __init__(self, desc, precision: str = "f64"):
        L = lib()
        self.desc = desc
        self._keep = [
            np.ascontiguousarray(desc.rod_offsets, dtype=np.int32),
            _f64(desc.rest_pos).reshape(-1),
            _f64(desc.rest_radius),
            np.ascontiguousarray(desc.pinned, dtype=np.uint8),
            _f64(desc.activation),
            _f64(desc.compliance).reshape(-1),
            np.ascontiguousarray(desc.group, dtype=np.int32),
            _f64(desc.gravity),
        ]
        off, rp, rr, pn, ac, co, gr, g = self._keep
        self.P = int(off[-1])
        self.num_rods = int(desc.num_rods)
        self.h = L.orc_create(1 if precision == "f64" else 0, self.num_rods, _p(off), _p(rp), _p(rr), _p(pn),
                              _p(ac), _p(co), _p(gr), float(desc.density), _p(g))

        if getattr(desc, "section_offsets", None) is not None:
            self._sec = (np.ascontiguousarray(desc.section_offsets, dtype=np.int32),
                         np.ascontiguousarray(desc.section_pills, dtype=np.int32))
            L.orc_set_sections(self.h, int(self._sec[0].shape[0] - 1), _p(self._sec[0]), _p(self._sec[1]))
        if getattr(desc, "solver", "gauss_seidel") == "jacobi":
            L.orc_set_solver(self.h, 1)
        if getattr(desc, "floor", None) is not None:
            n = np.ascontiguousarray(desc.floor[:3], dtype=np.float64)
            L.orc_set_floor(self.h, _p(n), float(desc.floor[3]))
        if getattr(desc, "bone_rest", None) is not None:
            self._bones = (_f64(desc.bone_rest).reshape(-1), np.ascontiguousarray(desc.pill_bones, np.int32).reshape(-1),
                           _f64(desc.pill_bone_weights).reshape(-1))
            L.orc_set_bones(self.h, int(self._bones[0].shape[0] // 12), *[_p(a) for a in self._bones])
        if getattr(desc, "cross_compliance", None) is not None:
            self._sr = _f64(desc.cross_compliance).reshape(-1)
            L.orc_set_cross_stretch(self.h, _p(self._sr))
        if getattr(desc, "volume_bending", False):
            L.orc_set_volume_bending(self.h, 1)
        if getattr(desc, "bending_compliance", None) is not None:
            self._sb = _f64(desc.bending_compliance).reshape(-1)
            L.orc_set_surface_bending(self.h, _p(self._sb))

    def skin_weights(self, rest_v):
        """Initial skinning weights (Sec. 7.4) of rest vertices: (capsule ids [V,4], weights [V,4])."""
        v = np.ascontiguousarray(rest_v, dtype=np.float64).reshape(-1, 3)
        caps = np.zeros((v.shape[0], 4), np.int32)
        w = np.zeros((v.shape[0], 4))
        lib().orc_skin_weights(self.h, int(v.shape[0]), _p(v), _p(caps), _p(w))
        return caps, w

    def skin_weights_faired(self, rest_v, tris, iterations, lam=0.5):
        """Initial skinning weights faired over the mesh (Sec. 7.4; readings in the source):
        (capsule ids [V,4], weights [V,4])."""
        v = np.ascontiguousarray(rest_v, dtype=np.float64).reshape(-1, 3)
        t = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
        caps = np.zeros((v.shape[0], 4), np.int32)
        w = np.zeros((v.shape[0], 4))
        lib().orc_skin_weights_faired(self.h, int(v.shape[0]), _p(v), int(t.shape[0]), _p(t), int(iterations),
                                      float(lam), _p(caps), _p(w))
        return caps, w

    def rod_iterations(self, h, iters=1):
        """`iters` iterations of the rod constraints at the current state (substep h), from
        zero multipliers (as project_one)."""
        return int(lib().orc_rod_iteration(self.h, float(h), int(iters)))

    def set_floor(self, plane):
        """Move the half-plane floor to plane = (nx, ny, nz, d) (Sec. 7, kinematic proxy)."""
        n = np.ascontiguousarray(plane[:3], dtype=np.float64)
        lib().orc_set_floor(self.h, _p(n), float(plane[3]))

    def set_bones(self, transforms):
        """The bones' transforms of a new frame ([nb, 3, 4]): warm start of the pills (Sec. 8.2)."""
        t = _f64(transforms).reshape(-1)
        lib().orc_bone_frame(self.h, _p(t))

    def floor_pass(self):
        """One projection of every pill against the half-plane floor (Sec. 7)."""
        lib().orc_floor_pass(self.h)

    def section_fit(self, k):
        """Bundling fit of section k at the current state (Sec. 7.3): (R*, s*, c*, q*)."""
        out = np.zeros(17)
        lib().orc_section_fit(self.h, int(k), _p(out))
        return out[:9].reshape(3, 3), float(out[9]), out[10:13].copy(), out[13:17].copy()

    def bundle(self):
        """One bundling projection of every section at the current state."""
        lib().orc_bundle(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            try:
                lib().orc_destroy(self.h)
            except Exception:      # interpreter shutdown
                pass
            self.h = None

    def set_state(self, x=None, v=None, s=None, sd=None, q=None, om=None):
        arrs = [None if a is None else _f64(a).reshape(-1) for a in (x, v, s, sd, q, om)]
        lib().orc_set_state(self.h, *[_p(a) for a in arrs])

    def get_state(self):
        P = self.P
        x = np.zeros((P, 3)); v = np.zeros((P, 3)); s = np.zeros(P); sd = np.zeros(P)
        q = np.zeros((P, 4)); om = np.zeros((P, 3))
        lib().orc_get_state(self.h, _p(x), _p(v), _p(s), _p(sd), _p(q), _p(om))
        return dict(x=x, v=v, s=s, sd=sd, q=q, om=om)

    def step(self, dt, substeps, iters, collide=False, search_iters=10, delta=1e-4, threads=1):
        return int(lib().orc_step(self.h, float(dt), int(substeps), int(iters), int(bool(collide)),
                                  int(search_iters), float(delta), int(threads)))

    def rest(self):
        P = self.P
        out = dict(l0=np.zeros(P), lbar=np.zeros(P), qrest=np.zeros((P, 4)), darb=np.zeros((P, 3)),
                   winv=np.zeros(P), wsinv=np.zeros(P), inert=np.zeros(P), comp=np.zeros((P, 4)))
        lib().orc_get_rest(self.h, *[_p(out[k]) for k in ("l0", "lbar", "qrest", "darb", "winv", "wsinv",
                                                          "inert", "comp")])
        return out

    def project_one(self, kind: int, p: int, h: float):
        lib().orc_project_one(self.h, int(kind), int(p), float(h))

    def set_masses(self, winv=None, wsinv=None, inert=None):
        arrs = [None if a is None else _f64(a) for a in (winv, wsinv, inert)]
        lib().orc_set_masses(self.h, *[_p(a) for a in arrs])

    def contact_pass(self, search_iters=10, delta=1e-4):
        lib().orc_contact_pass(self.h, int(search_iters), float(delta))

    def substep_residuals(self, h, iters):
        out = np.zeros(iters)
        lib().orc_substep_residuals(self.h, float(h), int(iters), _p(out))
        return out

    def pairs(self):
        n = lib().orc_num_pairs(self.h)
        out = np.zeros((n, 2), dtype=np.int32)
        if n:
            lib().orc_get_pairs(self.h, _p(out))
        return out

    def active_count(self):
        out = np.zeros(self.P, dtype=np.int32)
        lib().orc_get_active_count(self.h, _p(out))
        return out

    def skin(self, rest_v, caps, w):
        rest_v = _f64(rest_v).reshape(-1)
        caps = np.ascontiguousarray(caps, dtype=np.int32).reshape(-1)
        w = _f64(w).reshape(-1)
        V = rest_v.size // 3
        out = np.zeros((V, 3))
        lib().orc_skin(self.h, V, _p(rest_v), _p(caps), _p(w), _p(out))
        return out

    def capsule_transforms(self):
        out = np.zeros((self.P, 3, 4))
        lib().orc_capsule_transforms(self.h, _p(out))
        return out


def brute_pairs(desc, x, s, rbar):
    """Exact FP64 candidate pair set from explicit values, sorted (a, b)."""
    off = np.ascontiguousarray(desc.rod_offsets, dtype=np.int32)
    grp = np.ascontiguousarray(desc.group, dtype=np.int32)
    x = _f64(x).reshape(-1); s = _f64(s); rbar = _f64(rbar)
    cap = 1 << 16
    while True:
        out = np.zeros((cap, 2), dtype=np.int32)
        n = lib().orc_brute_pairs(int(desc.num_rods), _p(off), _p(grp), _p(x), _p(s), _p(rbar), _p(out), cap)
        if n <= cap:
            return out[:n].copy()
        cap = n


def pill_project(x, c1, r1, c2, r2):
    a = [_f64(v) for v in (x, c1, c2)]
    return lib().orc_pill_project(_p(a[0]), _p(a[1]), float(r1), _p(a[2]), float(r2))


def coll_gap(a1, ra1, a2, ra2, b1, rb1, b2, rb2, al):
    a = [_f64(v) for v in (a1, a2, b1, b2)]
    return lib().orc_coll_gap(_p(a[0]), float(ra1), _p(a[1]), float(ra2), _p(a[2]), float(rb1), _p(a[3]),
                              float(rb2), float(al))


def dichotomous(a1, ra1, a2, ra2, b1, rb1, b2, rb2, iters=10, delta=1e-4):
    a = [_f64(v) for v in (a1, a2, b1, b2)]
    return lib().orc_dichotomous(_p(a[0]), float(ra1), _p(a[1]), float(ra2), _p(a[2]), float(rb1), _p(a[3]),
                                 float(rb2), int(iters), float(delta))


def grad(desc, dt, substeps, iters, frames, targets, threads=8, precision="f64"):
    """Gradient (dual numbers) of L = sum |x_free_end - target|^2 w.r.t. rest radii and activations:
    exact derivatives of the discrete algorithm in FP64, or the same in FP32 arithmetic
    (precision="f32", the rounding floor of an FP32 gradient)."""
    L = lib()
    off = np.ascontiguousarray(desc.rod_offsets, dtype=np.int32)
    arrs = [_f64(desc.rest_pos).reshape(-1), _f64(desc.rest_radius), np.ascontiguousarray(desc.pinned, np.uint8),
            _f64(desc.activation), _f64(desc.compliance).reshape(-1), np.ascontiguousarray(desc.group, np.int32),
            _f64(desc.gravity)]
    tg = _f64(targets).reshape(-1)
    drb = np.zeros(int(off[-1])); dac = np.zeros(int(desc.num_rods))
    loss = L.orc_grad(int(desc.num_rods), _p(off), _p(arrs[0]), _p(arrs[1]), _p(arrs[2]), _p(arrs[3]), _p(arrs[4]),
                      _p(arrs[5]), float(desc.density), _p(arrs[6]), float(dt), int(substeps), int(iters), int(frames),
                      _p(tg), _p(drb), _p(dac), int(threads), 1 if precision == "f64" else 0)
    return loss, drb, dac


def loss(desc, dt, substeps, iters, frames, targets, threads=8):
    """Forward-only FP64 loss (for finite differences)."""
    o = OracleScene(desc, "f64")
    for _ in range(frames):
        o.step(dt, substeps, iters, threads=threads)
    x = o.get_state()["x"]
    last = np.asarray(desc.rod_offsets[1:]) - 1
    e = x[last] - np.asarray(targets).reshape(-1, 3)
    return float((e * e).sum())
