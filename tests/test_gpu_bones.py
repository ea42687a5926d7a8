"""Kinematic bones with the linear-blend warm start (Sec. 8.2) on the GPU against the oracle.

Workload: helix rods of 13 pills (24 rods, seed 2) with two bones, each pill blended between
them by its position along its rod, rod ends pinned (attached); four frames in which both
bones turn and translate (a different motion each, 0.6 rad/s and 12 cm/s), set_bones then one frame of 10 substeps x
4 iterations.  Checks:
- FP64: the state right after each set_bones and after each frame equals the oracle's to
  rounding; FP32 within the 1e-4 bound of the other parity tests after the four frames;
- 70 bones (three launches of bone transforms) with random pill influences: the warm start
  equals the oracle's;
- rejections: a scene without bones, a singular transform (nothing moves), the pool, the
  adjoint.
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


def affine(R, t):
    return np.hstack([R, np.asarray(t, float)[:, None]])


def compose(M, T):
    return np.hstack([M[:, :3] @ T[:, :3], (M[:, :3] @ T[:, 3] + M[:, 3])[:, None]])


def two_bone_scene():
    d = scenes.helix_rods(24, 13, seed=2)
    off = d.rod_offsets
    u = np.zeros(d.num_pills)
    for k in range(d.num_rods):
        n = off[k + 1] - off[k]
        u[off[k]:off[k + 1]] = np.linspace(0.0, 1.0, n)
        d.pinned[off[k]] = 1
        d.pinned[off[k + 1] - 1] = 1
    rest = np.stack([affine(rot((1, 2, 3), 0.4), (0.1, -0.2, 0.05)), affine(rot((0, 1, 0), -0.7), (0.3, 0.0, 0.2))])
    return dataclasses.replace(d, bone_rest=rest, pill_bones=np.tile(np.array([[0, 1]], np.int32), (d.num_pills, 1)),
                               pill_bone_weights=np.stack([1.0 - u, u], 1))


def frame_transforms(d, f):
    # about 0.6 rad/s and 12 cm/s: the oracle rerun from a 1e-14 perturbation stays within
    # 1e-11 of itself over these frames (five times faster, it does not: the forced rods lose
    # reproducibility within three frames in any implementation)
    M0 = affine(rot((0, 0, 1), 0.01 * f), (0.0, 0.002 * f, 0.0))
    M1 = affine(rot((1, 0, 1), -0.008 * f), (0.001 * f, 0.0, 0.002 * f))
    return np.stack([compose(M0, d.bone_rest[0]), compose(M1, d.bone_rest[1])])


def test_fp64_frames_match_oracle():
    d = two_bone_scene()
    say("case: bones fp64, 4 frames", d.num_pills)
    sc = viper.Scene(d, "f64")
    o = oracle.OracleScene(d, "f64")
    for f in range(1, 5):
        T = frame_transforms(d, f)
        g0, r0 = sc.state(), o.get_state()
        sc.set_bones(T)
        o.set_bones(T)
        sc.sync()
        g1, r1 = sc.state(), o.get_state()
        # the warm start alone: the same displacement, scales and rotations untouched
        dd = np.abs((g1["x"] - g0["x"]) - (r1["x"] - r0["x"])).max()
        assert dd < 1e-13 and np.abs(g1["x"] - g0["x"]).max() > 1e-4, (f, dd)
        assert np.array_equal(g1["s"], g0["s"]) and np.array_equal(g1["q"], g0["q"])
        sc.step(1 / 60, 10, 4)
        o.step(1 / 60, 10, 4)
        sc.sync()
        ex, es, eq = errors(d, sc.state(), o.get_state())
        say("frame", f, "errors", ex, es, eq)
        assert ex < 1e-10 and es < 1e-10 and eq < 1e-10


def test_fp32_frames_within_tolerance():
    d = two_bone_scene()
    sc = viper.Scene(d, "f32")
    o = oracle.OracleScene(d, "f64")
    for f in range(1, 5):
        T = frame_transforms(d, f)
        sc.set_bones(T)
        o.set_bones(T)
        sc.step(1 / 60, 10, 4)
        o.step(1 / 60, 10, 4)
    sc.sync()
    ex, es, eq = errors(d, sc.state(), o.get_state())
    say("fp32 errors after 4 frames", ex, es, eq)
    assert ex < 1e-4 and es < 1e-4 and eq < 1e-4


def test_many_bones_warm_start():
    d = scenes.helix_rods(24, 13, seed=2)
    rng = np.random.default_rng(7)
    nb = 70
    rest = np.stack([affine(rot(rng.normal(size=3), rng.uniform(-1, 1)), rng.normal(0, 0.1, 3)) for _ in range(nb)])
    pb = rng.integers(0, nb, (d.num_pills, 2)).astype(np.int32)
    pw = rng.uniform(0.0, 1.0, (d.num_pills, 2))
    pw[::5, 1] = 0.0
    pw[::11] = 0.0
    d = dataclasses.replace(d, bone_rest=rest, pill_bones=pb, pill_bone_weights=pw)
    say("case: 70 bones warm start", d.num_pills)
    cur = np.stack([compose(affine(rot(rng.normal(size=3), 0.3), rng.normal(0, 0.05, 3)), T) for T in rest])
    sc = viper.Scene(d, "f64")
    o = oracle.OracleScene(d, "f64")
    x0 = sc.state()["x"]
    sc.set_bones(cur)
    o.set_bones(cur)
    sc.sync()
    g, r = sc.state(), o.get_state()
    assert np.abs(g["x"] - r["x"]).max() < 1e-13
    assert np.array_equal(g["x"][::11], x0[::11])          # no weight: not moved
    assert np.abs(g["x"] - x0).max() > 1e-2


def test_rejections():
    plain = viper.Scene(scenes.helix_rods(4, 8, seed=1), "f32")
    with pytest.raises(viper.ViperError) as ei:
        plain.set_bones(np.zeros((1, 3, 4)))
    assert ei.value.status == viper.ERR_INVALID
    d = two_bone_scene()
    sc = viper.Scene(d, "f32")
    x0 = sc.state()["x"]
    T = frame_transforms(d, 1)
    T[1, :, :3] = 0.0
    with pytest.raises(viper.ViperError) as ei:
        sc.set_bones(T)
    assert ei.value.status == viper.ERR_INVALID
    assert np.array_equal(sc.state()["x"], x0)
    with pytest.raises(viper.ViperError) as ei:
        sc.step_checkpointed(1 / 60, 1, 4, 4)
    assert ei.value.status == viper.ERR_INVALID
    pool = viper.Pool(16 << 20, precision="f32")
    with pytest.raises(viper.ViperError) as ei:
        pool.admit(d)
    assert ei.value.status == viper.ERR_INVALID
