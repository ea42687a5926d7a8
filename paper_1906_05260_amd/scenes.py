"""Seeded synthetic scene generators (inputs only).

This module builds the host-side scene descriptions and skinning meshes that
both the GPU library and the oracle consume.  It holds none of the solver's
arithmetic: only rest geometry, per-rod parameters and random draws.  The
paper's own assets (octopus, anatomical muscles, elastic band; Sec. 7-8) are
not available, so these seeded scenes stand in for them with the shapes and
sizes of the paper's workloads.

All lengths are metres, compliances Pa^-1, density kg/m^3.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

DENSITY = 1000.0               # muscle is mostly water (Sec. 1)
GRAVITY = (0.0, -9.81, 0.0)


@dataclass
class SceneDesc:
    """Host description of a rod scene (one entry per pill / rod)."""
    rod_offsets: np.ndarray            # int32 [R+1]
    rest_pos: np.ndarray               # float64 [P,3]
    rest_radius: np.ndarray            # float64 [P]
    pinned: np.ndarray                 # uint8 [P]
    activation: np.ndarray             # float64 [R]
    compliance: np.ndarray             # float64 [R,4]: stretch-shear, volume, scale-gradient, bend-twist
    group: np.ndarray                  # int32 [R]
    density: float = DENSITY
    gravity: tuple = GRAVITY
    collisions: bool = False
    name: str = ""
    extra: dict = field(default_factory=dict)
    # bundling cross-sections (Sec. 7.3): section k = pills section_pills[section_offsets[k]:section_offsets[k+1]]
    section_offsets: np.ndarray = None  # int32 [S+1]
    section_pills: np.ndarray = None    # int32
    # half-plane floor (Sec. 7): (nx, ny, nz, d), pills stay in n . x >= d; None = no floor
    floor: tuple = None
    # rod-constraint solver: "gauss_seidel" (coloured) or "jacobi" (with averaging, Sec. 7)
    solver: str = "gauss_seidel"
    # cross-section stretch (eq. stretch_xy) compliance per rod [num_rods]; None or +inf = off
    cross_compliance: np.ndarray = None
    # surface bending (Laplacian of the scale along the rod, Sec. 5) compliance per rod
    # [num_rods]; None or +inf = off
    bending_compliance: np.ndarray = None
    # volume-bending coupling (the s^3 Omega^{u,v} terms of the volume energy, Sec. 5) on rods
    # with the volume constraint, at the volume compliance
    volume_bending: bool = False
    # kinematic bones (Sec. 8.2): rest transforms [nb, 3, 4] (the bones' pose at rest_pos) and
    # two (bone, weight) influences per pill, [P, 2] int32 and [P, 2] float64; None = no bones
    bone_rest: np.ndarray = None
    pill_bones: np.ndarray = None
    pill_bone_weights: np.ndarray = None

    @property
    def num_rods(self) -> int:
        return int(self.rod_offsets.shape[0] - 1)

    @property
    def num_pills(self) -> int:
        return int(self.rod_offsets[-1])

    def subset(self, rods) -> "SceneDesc":
        """Scene made of the given rods only (rods are independent without contacts)."""
        rods = np.asarray(rods, dtype=np.int64)
        offs = [0]
        idx = []
        for k in rods:
            a, b = int(self.rod_offsets[k]), int(self.rod_offsets[k + 1])
            idx.append(np.arange(a, b))
            offs.append(offs[-1] + b - a)
        idx = np.concatenate(idx)
        return SceneDesc(np.asarray(offs, np.int32), self.rest_pos[idx].copy(), self.rest_radius[idx].copy(),
                         self.pinned[idx].copy(), self.activation[rods].copy(), self.compliance[rods].copy(),
                         self.group[rods].copy(), self.density, self.gravity, self.collisions,
                         self.name + "[subset]")

    def pill_index(self, rods):
        return np.concatenate([np.arange(self.rod_offsets[k], self.rod_offsets[k + 1]) for k in rods])


@dataclass
class SkinMesh:
    rest_v: np.ndarray     # float32 [V,3]
    caps: np.ndarray       # int32 [V,4]  capsule id = global index of the capsule's first pill
    w: np.ndarray          # float32 [V,4], rows sum to 1
    tris: Optional[np.ndarray] = None   # int32 [F,3] triangles (meshes with connectivity)


def _log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


def straight_rod(n_pills=32, spacing=0.01, radius=0.005, compliance=1e-6) -> SceneDesc:
    """One straight rod along +x, pill 0 pinned (the 32-pill FP64 single-rod case)."""
    x = np.zeros((n_pills, 3))
    x[:, 0] = spacing * np.arange(n_pills)
    pinned = np.zeros(n_pills, np.uint8)
    pinned[0] = 1
    return SceneDesc(np.asarray([0, n_pills], np.int32), x, np.full(n_pills, radius), pinned,
                     np.ones(1), np.full((1, 4), compliance), np.zeros(1, np.int32), name="single_rod_%d" % n_pills)


def helix_rods(num_rods=4096, n_pills=64, seed=1, grid_spacing=0.1, arc=0.01) -> SceneDesc:
    """Independent random helices along +x on a square grid, pill 0 pinned.

    Helix radius U[0.5,2] cm, pitch U[1,4] cm, pills 1 cm apart in arc length,
    pill radii U[0.2,0.8] cm, compliances log-uniform 1e-8..1e-4 per type and rod.
    """
    rng = np.random.default_rng(seed)
    side = int(np.ceil(np.sqrt(num_rods)))
    R = rng.uniform(0.005, 0.02, num_rods)
    pitch = rng.uniform(0.01, 0.04, num_rods)
    rbar = rng.uniform(0.002, 0.008, num_rods * n_pills)
    comp = _log_uniform(rng, 1e-8, 1e-4, (num_rods, 4))
    phase = rng.uniform(0, 2 * np.pi, num_rods)
    k = np.arange(num_rods)
    gy = (k // side) * grid_spacing
    gz = (k % side) * grid_spacing
    c = pitch / (2 * np.pi)
    dt = arc / np.sqrt(R ** 2 + c ** 2)
    t = dt[:, None] * np.arange(n_pills)[None, :]
    x = np.empty((num_rods, n_pills, 3))
    x[:, :, 0] = c[:, None] * t
    x[:, :, 1] = gy[:, None] + R[:, None] * np.cos(t + phase[:, None])
    x[:, :, 2] = gz[:, None] + R[:, None] * np.sin(t + phase[:, None])
    pinned = np.zeros((num_rods, n_pills), np.uint8)
    pinned[:, 0] = 1
    offs = np.arange(num_rods + 1, dtype=np.int32) * n_pills
    return SceneDesc(offs, x.reshape(-1, 3), rbar, pinned.reshape(-1), np.ones(num_rods), comp,
                     np.arange(num_rods, dtype=np.int32), name="helix_%dx%d" % (num_rods, n_pills))


def straight_rods(num_rods=1024, n_pills=32, seed=4, grid_spacing=0.1):
    """Straight rods along +x (1 cm spacing), random radii, compliances and activations,
    plus per-rod targets near the free end (the differentiation workload)."""
    rng = np.random.default_rng(seed)
    side = int(np.ceil(np.sqrt(num_rods)))
    rbar = rng.uniform(0.002, 0.008, num_rods * n_pills)
    comp = _log_uniform(rng, 1e-8, 1e-4, (num_rods, 4))
    act = rng.uniform(0.8, 1.2, num_rods)
    k = np.arange(num_rods)
    x = np.zeros((num_rods, n_pills, 3))
    x[:, :, 0] = 0.01 * np.arange(n_pills)[None, :]
    x[:, :, 1] = ((k // side) * grid_spacing)[:, None]
    x[:, :, 2] = ((k % side) * grid_spacing)[:, None]
    pinned = np.zeros((num_rods, n_pills), np.uint8)
    pinned[:, 0] = 1
    offs = np.arange(num_rods + 1, dtype=np.int32) * n_pills
    desc = SceneDesc(offs, x.reshape(-1, 3), rbar, pinned.reshape(-1), act, comp,
                     np.arange(num_rods, dtype=np.int32), name="straight_%dx%d" % (num_rods, n_pills))
    targets = x[:, -1, :] + rng.normal(0.0, 0.01, (num_rods, 3))
    return desc, targets


def _vogel_disc(n, radius):
    i = np.arange(n) + 0.5
    r = radius * np.sqrt(i / n)
    th = i * np.pi * (3.0 - np.sqrt(5.0))
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


MUSCLE_COMPLIANCE = (1e-7, 1e-8, 1e-8, 1e-5)     # stretch-shear, volume, scale gradient, bend-twist


def muscle_scene(num_muscles=64, seed=2, target_pills=(45000, 55000), rods_range=(16, 48), pills_range=(8, 24),
                 mesh_vertices=200000, spacing=0.01, compliance=MUSCLE_COMPLIANCE, bundling=False, capsule_order=True):
    """Bundles of parallel rods ("muscles") packed side by side so that neighbours touch.

    Each muscle has U{16..48} rods of U{8..24} pills (all rods of a muscle share the
    pill count, so its cross-sections are aligned).  Sizes are then grown one unit at
    a time at random muscles until the total lies in ``target_pills`` (the plain
    draws average ~33k pills; the workload asks for ~50k).  Both rod ends are
    pinned (bone attachments), activation U[0.8,1.2] per muscle, collision group =
    muscle.  Compliances default to ``MUSCLE_COMPLIANCE`` for every rod: a muscle keeps
    its volume, and with volume or scale-gradient compliances near 1e-4 the activation
    step drives some scales through zero (negative radii) within the first frames;
    ``compliance="loguniform"`` draws them log-uniform 1e-8..1e-4 per type and rod as
    in the helix scene.  ``capsule_order``: mesh vertices numbered by first capsule (see
    ``muscle_mesh``).  With ``bundling`` every muscle gets one cross-section per pill
    index (that pill of each of its rods) for the shape matching of Sec. 7.3.  Returns (desc, mesh) with a skinning mesh of ``mesh_vertices`` vertices
    on the muscles' envelopes, 4 nearest capsules each, Dirichlet(1,1,1,1) weights.
    """
    rng = np.random.default_rng(seed)
    nr = rng.integers(rods_range[0], rods_range[1] + 1, num_muscles)
    npl = rng.integers(pills_range[0], pills_range[1] + 1, num_muscles)
    if target_pills is not None:
        lo, hi = target_pills
        while int((nr * npl).sum()) < lo:
            m = int(rng.integers(num_muscles))
            if rng.random() < 0.5 and nr[m] < rods_range[1]:
                nr[m] += 1
            elif npl[m] < pills_range[1]:
                npl[m] += 1
        assert int((nr * npl).sum()) <= hi
    act = rng.uniform(0.8, 1.2, num_muscles)
    side = int(np.ceil(np.sqrt(num_muscles)))
    # per-muscle rod radii and bundle radius
    xs, rbs, pins, acts, comps, groups, offs = [], [], [], [], [], [], [0]
    muscle_info = []
    rmax = 0.008
    bundle_r = 1.2 * np.sqrt(nr) * 0.005
    cell = 2.0 * bundle_r.max()
    for m in range(num_muscles):
        gy = (m // side) * cell
        gz = (m % side) * cell
        centres = _vogel_disc(int(nr[m]), bundle_r[m] - rmax)
        L = (npl[m] - 1) * spacing
        x0 = -0.5 * L
        tilt = rng.normal(0.0, 0.02, 2)
        rod_ids = []
        for r in range(int(nr[m])):
            n = int(npl[m])
            x = np.zeros((n, 3))
            x[:, 0] = x0 + spacing * np.arange(n)
            x[:, 1] = gy + centres[r, 0] + tilt[0] * x[:, 0]
            x[:, 2] = gz + centres[r, 1] + tilt[1] * x[:, 0]
            xs.append(x)
            rbs.append(rng.uniform(0.002, 0.008, n))
            pn = np.zeros(n, np.uint8)
            pn[0] = 1
            pn[-1] = 1
            pins.append(pn)
            acts.append(act[m])
            drawn = _log_uniform(rng, 1e-8, 1e-4, 4)       # drawn either way: the other draws stay put
            comps.append(drawn if isinstance(compliance, str) and compliance == "loguniform"
                         else np.asarray(compliance, dtype=np.float64))
            groups.append(m)
            rod_ids.append(len(offs) - 1)
            offs.append(offs[-1] + n)
        muscle_info.append(dict(rods=rod_ids, centre=(gy, gz), radius=bundle_r[m], x0=x0, L=L, tilt=tilt))
    desc = SceneDesc(np.asarray(offs, np.int32), np.concatenate(xs), np.concatenate(rbs), np.concatenate(pins),
                     np.asarray(acts), np.asarray(comps), np.asarray(groups, np.int32), collisions=True,
                     name="muscles_%d" % num_muscles)
    mesh = muscle_mesh(desc, muscle_info, mesh_vertices, rng, capsule_order) if mesh_vertices else None
    desc.extra["muscles"] = muscle_info
    if bundling:
        # one cross-section per pill index of each muscle: pill k of every rod of the muscle
        offs = np.asarray(desc.rod_offsets)
        so, sp = [0], []
        for mi in muscle_info:
            for k in range(int(offs[mi["rods"][0] + 1] - offs[mi["rods"][0]])):
                sp.extend(int(offs[r]) + k for r in mi["rods"])
                so.append(len(sp))
        desc.section_offsets = np.asarray(so, np.int32)
        desc.section_pills = np.asarray(sp, np.int32)
    return desc, mesh


def muscle_mesh(desc: SceneDesc, muscle_info, V, rng, capsule_order=True) -> SkinMesh:
    """Vertices on each muscle's envelope cylinder (count proportional to its pills);
    influences = the 4 nearest capsules of that muscle at rest, Dirichlet(1,1,1,1) weights.
    Each muscle's vertices are numbered in the order of their first capsule (capsule_order;
    otherwise along the muscle's axis, random around it)."""
    offs = desc.rod_offsets
    pills = np.array([sum(int(offs[k + 1] - offs[k]) for k in mi["rods"]) for mi in muscle_info], dtype=np.float64)
    counts = np.floor(V * pills / pills.sum()).astype(np.int64)
    counts[: V - int(counts.sum())] += 1
    rv, cp, ww = [], [], []
    for m, mi in enumerate(muscle_info):
        nv = int(counts[m])
        if nv == 0:
            continue
        caps = np.concatenate([np.arange(offs[k], offs[k + 1] - 1) for k in mi["rods"]])
        mids = 0.5 * (desc.rest_pos[caps] + desc.rest_pos[caps + 1])
        u = np.sort(rng.uniform(0.0, 1.0, nv))      # vertex order runs along the axis, as a mesh's rings do
        th = rng.uniform(0.0, 2 * np.pi, nv)
        xx = mi["x0"] + u * mi["L"]
        rr = mi["radius"] + 0.004
        p = np.stack([xx, mi["centre"][0] + mi["tilt"][0] * xx + rr * np.cos(th),
                      mi["centre"][1] + mi["tilt"][1] * xx + rr * np.sin(th)], axis=1)
        mc = []
        for c0 in range(0, nv, 4096):
            pc = p[c0:c0 + 4096]
            d2 = ((pc[:, None, :] - mids[None, :, :]) ** 2).sum(-1)
            nn = np.argsort(d2, axis=1, kind="stable")[:, :4]
            mc.append(caps[nn])
        mc = np.concatenate(mc)
        wm = rng.dirichlet(np.ones(4), nv)
        # vertices renumbered in the order of their first capsule (stable), as a mesh pipeline
        # orders vertices for the skinning pass: neighbouring vertices then share transforms
        o = np.argsort(mc[:, 0], kind="stable") if capsule_order else np.arange(nv)
        rv.append(p[o])
        cp.append(mc[o])
        ww.append(wm[o])
    return SkinMesh(np.concatenate(rv).astype(np.float32), np.concatenate(cp).astype(np.int32),
                    np.concatenate(ww).astype(np.float32))


def tube_mesh(desc: SceneDesc, vertices=200000, seed=0, offset=0.004, jitter=0.0) -> SkinMesh:
    """A closed-surface triangle mesh on each muscle's envelope (a muscle scene's
    ``extra["muscles"]``): a tube of rings around the muscle axis, ring count and ring size
    chosen so that the muscle's share of ``vertices`` is proportional to its pills, capped by
    a fan at each end; ``offset`` m outside the bundle radius, optional radial ``jitter``
    (fraction of the radius, seeded).  Influences and weights are left empty (caps -1, w 0):
    they come from the skinning-weight computation."""
    rng = np.random.default_rng(seed)
    offs = desc.rod_offsets
    mus = desc.extra["muscles"]
    pills = np.array([sum(int(offs[k + 1] - offs[k]) for k in mi["rods"]) for mi in mus], dtype=np.float64)
    share = vertices * pills / pills.sum()
    pos, tri, base = [], [], 0
    for m, mi in enumerate(mus):
        n = max(int(share[m]), 10)
        # rings of `ar` vertices, `al` rings, aspect about the tube's length / circumference
        rr = mi["radius"] + offset
        circ, L = 2 * np.pi * rr, max(mi["L"], 1e-3)
        ar = max(3, int(round(np.sqrt(n * circ / L))))
        al = max(2, (n - 2) // ar)
        u = np.linspace(0.0, 1.0, al)
        th = 2 * np.pi * np.arange(ar) / ar
        xx = mi["x0"] + u[:, None] * L + 0 * th[None, :]
        r = rr * (1.0 + jitter * rng.uniform(-1.0, 1.0, (al, ar)))
        cy = mi["centre"][0] + mi["tilt"][0] * xx + r * np.cos(th)[None, :]
        cz = mi["centre"][1] + mi["tilt"][1] * xx + r * np.sin(th)[None, :]
        ring = np.stack([xx, cy, cz], -1).reshape(-1, 3)
        ends = np.array([[mi["x0"], mi["centre"][0] + mi["tilt"][0] * mi["x0"], mi["centre"][1] + mi["tilt"][1] * mi["x0"]],
                         [mi["x0"] + L, mi["centre"][0] + mi["tilt"][0] * (mi["x0"] + L),
                          mi["centre"][1] + mi["tilt"][1] * (mi["x0"] + L)]])
        pos.append(np.vstack([ring, ends]))
        i = np.arange(al - 1)[:, None] * ar
        j = np.arange(ar)[None, :]
        a, b = i + j, i + (j + 1) % ar
        c, d = a + ar, b + ar
        t = np.concatenate([np.stack([a, b, c], -1).reshape(-1, 3), np.stack([b, d, c], -1).reshape(-1, 3)])
        c0, c1 = al * ar, al * ar + 1
        f0 = np.stack([np.full(ar, c0), (np.arange(ar) + 1) % ar, np.arange(ar)], -1)
        f1 = np.stack([np.full(ar, c1), (al - 1) * ar + np.arange(ar), (al - 1) * ar + (np.arange(ar) + 1) % ar], -1)
        tri.append(np.concatenate([t, f0, f1]) + base)
        base += al * ar + 2
    v = np.concatenate(pos).astype(np.float32)
    V = v.shape[0]
    return SkinMesh(v, np.full((V, 4), -1, np.int32), np.zeros((V, 4), np.float32),
                    np.concatenate(tri).astype(np.int32))


def octopus_scene(num_models=100, seed=5, mesh_vertices_per_model=6500, spacing=0.2):
    """Models shaped like the paper's octopus example (Sec. 8): a 5-pill body hanging from
    a pinned top pill and 8 arms of 4 pills leaving the body's lowest pill, 37 pills per
    model, on a square grid close enough for neighbouring arms to collide (collision group =
    model).  The body's top pill and each arm's root are pinned.  Radii 1.5 cm (body) and
    1.2 -> 0.6 cm (arms); compliances 1e-7 (stretch-shear), 1e-8 (volume, scale gradient),
    1e-5 (bend-twist): stiff enough in volume that scales stay near 1 (with the log-uniform
    compliances of the helix scene, the soft volume and scale-gradient terms let bend-twist
    drive scales through zero within a frame); activation 1.  Each model gets a skinning mesh of ``mesh_vertices_per_model``
    vertices on its capsules' surfaces, influences = its 4 nearest capsules at rest with
    Dirichlet(1,1,1,1) weights.  Returns (desc, mesh)."""
    rng = np.random.default_rng(seed)
    side = int(np.ceil(np.sqrt(num_models)))
    pos, rad, pin, offs, grp, comp = [], [], [], [0], [], []
    model_rods = []
    for m in range(num_models):
        base = np.array([(m % side) * spacing, 0.5, (m // side) * spacing])
        rods = []
        body = base + np.outer(np.arange(5), [0.0, -0.025, 0.0])
        pos.append(body)
        rad.append(np.full(5, 0.015))
        pn = np.zeros(5, np.uint8)
        pn[0] = 1
        pin.append(pn)
        rods.append(len(offs) - 1)
        offs.append(offs[-1] + 5)
        grp.append(m)
        foot = body[-1]
        for a in range(8):
            th = 2 * np.pi * a / 8 + rng.uniform(-0.1, 0.1)
            d = np.array([np.cos(th), -0.35, np.sin(th)])
            d /= np.linalg.norm(d)
            arm = foot + np.outer(np.arange(1, 5), 0.03 * d)
            pos.append(arm)
            rad.append(np.linspace(0.012, 0.006, 4))
            pa = np.zeros(4, np.uint8)
            pa[0] = 1                     # the arm's root is held at the body
            pin.append(pa)
            rods.append(len(offs) - 1)
            offs.append(offs[-1] + 4)
            grp.append(m)
        model_rods.append(rods)
    R = len(grp)
    comp = np.tile([1e-7, 1e-8, 1e-8, 1e-5], (R, 1))
    desc = SceneDesc(np.asarray(offs, np.int32), np.concatenate(pos), np.concatenate(rad), np.concatenate(pin),
                     np.ones(R), comp, np.asarray(grp, np.int32), collisions=True,
                     name="octopus%dx37" % num_models)
    rv, cp, ww = [], [], []
    V = int(mesh_vertices_per_model)
    for m in range(num_models if V > 0 else 0):
        caps = np.concatenate([np.arange(offs[k], offs[k + 1] - 1) for k in model_rods[m]])
        a, b = desc.rest_pos[caps], desc.rest_pos[caps + 1]
        ra, rb = desc.rest_radius[caps], desc.rest_radius[caps + 1]
        L = np.linalg.norm(b - a, axis=1)
        pick = rng.choice(len(caps), V, p=L / L.sum())
        t = rng.uniform(0.0, 1.0, V)
        axis = (b - a)[pick] / L[pick, None]
        helper = np.where(np.abs(axis[:, 1:2]) < 0.9, [[0.0, 1.0, 0.0]], [[1.0, 0.0, 0.0]])
        e1 = np.cross(axis, helper)
        e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
        e2 = np.cross(axis, e1)
        th = rng.uniform(0.0, 2 * np.pi, V)
        r = (1 - t) * ra[pick] + t * rb[pick] + 0.002
        p = a[pick] + t[:, None] * (b - a)[pick] + r[:, None] * (np.cos(th)[:, None] * e1 + np.sin(th)[:, None] * e2)
        mids = 0.5 * (a + b)
        d2 = ((p[:, None, :] - mids[None, :, :]) ** 2).sum(-1)
        cp.append(caps[np.argsort(d2, axis=1, kind="stable")[:, :4]])
        rv.append(p)
        ww.append(rng.dirichlet(np.ones(4), V))
    mesh = None
    if rv:
        mesh = SkinMesh(np.concatenate(rv).astype(np.float32), np.concatenate(cp).astype(np.int32),
                        np.concatenate(ww).astype(np.float32))
    return desc, mesh


def scene_of_size(n_pills: int, kind: str, seed: int):
    """A serving request: helix rods of 64 pills or a muscle scene, about n_pills pills.
    Returns (desc, mesh or None)."""
    if kind == "helix":
        nrods = max(1, int(round(n_pills / 64)))
        return helix_rods(nrods, 64, seed=seed), None
    nm = max(1, int(round(n_pills / 512)))
    desc, mesh = muscle_scene(num_muscles=nm, seed=seed, target_pills=None, mesh_vertices=4 * n_pills)
    return desc, mesh


def capsule_mesh(desc: SceneDesc, per_pill=4, seed=0, offset=0.004) -> SkinMesh:
    """A skinning mesh of ``per_pill`` vertices per pill, built without a nearest-capsule
    search (the serving workload's meshes): the vertices of a pill sit ``offset`` outside the
    surface of its capsule (a rod's last pill uses its incoming capsule), at a uniform point
    along it and a uniform angle around it; the influences are that capsule and its
    neighbours along the rod (the capsule itself again past a rod end), with
    Dirichlet(1,1,1,1) weights."""
    rng = np.random.default_rng(seed)
    offs = np.asarray(desc.rod_offsets)
    P = desc.num_pills
    rod = np.repeat(np.arange(desc.num_rods), np.diff(offs))
    first, last = offs[rod], offs[rod + 1] - 1
    cap = np.where(np.arange(P) < last, np.arange(P), np.arange(P) - 1)      # capsule of each pill
    prev_c = np.where(cap > first, cap - 1, cap)
    next_c = np.where(cap + 1 < last, cap + 1, cap)
    c = np.repeat(cap, per_pill)
    infl = np.stack([c, np.repeat(prev_c, per_pill), np.repeat(next_c, per_pill), c], axis=1)
    a, b = desc.rest_pos[c], desc.rest_pos[c + 1]
    ra, rb = desc.rest_radius[c], desc.rest_radius[c + 1]
    V = c.shape[0]
    t = rng.uniform(0.0, 1.0, V)
    th = rng.uniform(0.0, 2 * np.pi, V)
    axis = b - a
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    helper = np.where(np.abs(axis[:, 1:2]) < 0.9, [[0.0, 1.0, 0.0]], [[1.0, 0.0, 0.0]])
    e1 = np.cross(axis, helper)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(axis, e1)
    r = (1 - t) * ra + t * rb + offset
    p = a + t[:, None] * (b - a) + r[:, None] * (np.cos(th)[:, None] * e1 + np.sin(th)[:, None] * e2)
    return SkinMesh(p.astype(np.float32), infl.astype(np.int32), rng.dirichlet(np.ones(4), V).astype(np.float32))


@dataclass
class Request:
    arrival: float          # seconds after the start of the run
    desc: SceneDesc
    frames: int
    kind: str
    mesh: Optional[SkinMesh] = None   # skinned after every frame (muscle requests)


def serving_requests(rate=200.0, duration=2.0, seed=3, min_pills=1000, max_pills=200000, frames=60,
                     kinds=("helix", "muscle"), skin_per_pill=4):
    """Poisson arrivals (exponential gaps of mean 1/rate) over `duration` seconds of scenes
    with log-uniform sizes in [min_pills, max_pills], kind drawn uniformly from `kinds`
    (64-pill helix rods, or muscle bundles with contacts and a skinning mesh of
    `skin_per_pill` vertices per pill, `capsule_mesh`; 0 = no mesh)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    k = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        n = int(np.exp(rng.uniform(np.log(min_pills), np.log(max_pills))))
        kind = kinds[int(rng.integers(len(kinds)))]
        mesh = None
        if kind == "helix":
            desc = helix_rods(max(1, int(round(n / 64))), 64, seed=seed * 100003 + k)
        else:
            desc, _ = muscle_scene(num_muscles=max(1, int(round(n / 512))), seed=seed * 100003 + k,
                                   target_pills=None, mesh_vertices=0)
            if skin_per_pill:
                mesh = capsule_mesh(desc, skin_per_pill, seed=seed * 100003 + k)
        out.append(Request(t, desc, frames, kind, mesh))
        k += 1
    return out
