"""The optional terms together on a contact scene, on the GPU against the oracle.

Workload: 8 muscles (3,860 pills, 231 rods, log-uniform compliances, seed 2) with pill-pill
contacts, cross-section stretch on every other rod, surface bending on every third, the
volume-bending coupling on, and two bones driving every pill (weights by position along its
rod; both rod ends pinned, so attached) turning and translating gently (0.6 rad/s, 12 cm/s:
the oracle rerun from a 1e-14 perturbation, collisions on, stays within 3e-12 of itself over
these frames).
Checks:
- FP64: four frames of set_bones then 4 substeps x 4 iterations, stepped as a captured graph
  (the default for contact scenes, the rod kernels with the optional terms compiled in),
  equal the oracle's (collisions on) to rounding, with the same number of candidate pairs
  every frame (the first appear in the third frame);
- FP32: the captured-graph frames equal eager ITERATION launches bit for bit.
"""
import dataclasses
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1906_05260_amd import scenes, viper  # noqa: E402

sys.path.insert(0, __file__.rsplit("/", 1)[0])
from test_gpu_rods import errors  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rot(axis, ang):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def combined(seed=2, n=8):
    d, _ = scenes.muscle_scene(num_muscles=n, seed=seed, target_pills=None, mesh_vertices=4000,
                               compliance="loguniform")
    R = d.num_rods
    sr = np.full(R, np.inf)
    sr[::2] = 1e-6
    sb = np.full(R, np.inf)
    sb[::3] = 1e-6
    off = d.rod_offsets
    u = np.zeros(d.num_pills)
    for k in range(R):
        u[off[k]:off[k + 1]] = np.linspace(0.0, 1.0, off[k + 1] - off[k])
    rest = np.stack([np.hstack([np.eye(3), np.zeros((3, 1))])] * 2)
    return dataclasses.replace(d, cross_compliance=sr, bending_compliance=sb, volume_bending=True, bone_rest=rest,
                               pill_bones=np.tile(np.array([[0, 1]], np.int32), (d.num_pills, 1)),
                               pill_bone_weights=np.stack([1.0 - u, u], 1))


def bones_at(f):
    T0 = np.hstack([rot((0, 0, 1), 0.01 * f), np.array([[0.0], [0.002 * f], [0.0]])])
    T1 = np.hstack([rot((1, 0, 0), -0.008 * f), np.array([[0.001 * f], [0.0], [0.002 * f]])])
    return np.stack([T0, T1])


def test_fp64_graph_frames_match_oracle():
    d = combined()
    assert d.collisions
    say("case: combined options fp64", d.num_pills, "pills")
    sc = viper.Scene(d, "f64")
    o = oracle.OracleScene(d, "f64")
    seen = 0
    for f in (1, 2, 3, 4):
        sc.set_bones(bones_at(f))
        o.set_bones(bones_at(f))
        sc.step(1 / 60, 4, 4)
        o.step(1 / 60, 4, 4, collide=True)
        sc.sync()
        ex, es, eq = errors(d, sc.state(), o.get_state())
        n = len(sc.contacts())
        say("frame", f, "errors", ex, es, eq, "contacts", n)
        assert n == len(o.pairs())
        seen += n
        assert ex < 1e-9 and es < 1e-9 and eq < 1e-9
    assert seen > 0


def test_fp32_graph_equals_eager():
    d = combined()
    a, b = viper.Scene(d, "f32"), viper.Scene(d, "f32")
    for f in (1, 2, 3, 4):
        for sc in (a, b):
            sc.set_bones(bones_at(f))
        a.step(1 / 60, 4, 4)                                 # default: captured graph
        b.step(1 / 60, 4, 4, mode=viper.MODE_ITERATION)
        a.sync()
        b.sync()
    sa, sb = a.state(), b.state()
    for k in ("x", "v", "s", "q"):
        assert np.array_equal(sa[k], sb[k]), k


def test_fp32_frames_within_the_fp32_rounding_floor():
    """FP32 GPU over the same four frames against the FP64 oracle, bounded by 4x the distance of
    the oracle's own FP32 run from FP64 (its rounding floor on this scene: ~5e-5 in scale by the
    fourth frame), with the same candidate-pair counts."""
    d = combined()
    sc = viper.Scene(d, "f32")
    o64, o32 = oracle.OracleScene(d, "f64"), oracle.OracleScene(d, "f32")
    for f in (1, 2, 3, 4):
        sc.set_bones(bones_at(f))
        for o in (o64, o32):
            o.set_bones(bones_at(f))
            o.step(1 / 60, 4, 4, collide=True)
        sc.step(1 / 60, 4, 4)
    sc.sync()
    g, r, r32 = sc.state(), o64.get_state(), o32.get_state()
    fx, fs, fq = errors(d, r32, r)
    ex, es, eq = errors(d, g, r)
    say("fp32 floor", fx, fs, fq, "gpu", ex, es, eq, "contacts", len(sc.contacts()), len(o64.pairs()))
    assert len(sc.contacts()) == len(o64.pairs())
    assert ex <= 4 * fx + 1e-7 and es <= 4 * fs + 1e-7 and eq <= 4 * fq + 1e-7
