"""GPU parity of the collision-free rod path (HIP kernels via the C ABI) against the oracle.

Tolerance (the stated target): max over pills of |x_gpu - x_ref| divided by the
rest length of the longest rod <= 1e-4; the same bound on the scale s (absolute,
rest value 1) and on the edge quaternions up to sign.
"""
import math
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1906_05260_amd import scenes, viper  # noqa: E402

TOL = 1e-4


def rod_length(desc):
    off = desc.rod_offsets
    best = 0.0
    for k in range(desc.num_rods):
        x = desc.rest_pos[off[k]:off[k + 1]]
        best = max(best, float(np.linalg.norm(np.diff(x, axis=0), axis=1).sum()))
    return best


def edge_mask(desc):
    m = np.ones(desc.num_pills, bool)
    m[np.asarray(desc.rod_offsets[1:]) - 1] = False
    return m


def errors(desc, g, r, pills=None):
    """Relative position error, scale error, quaternion error (up to sign) on the given pills."""
    idx = np.arange(desc.num_pills) if pills is None else pills
    L = rod_length(desc)
    ex = np.abs(g["x"][idx] - r["x"]).max() / L
    es = np.abs(g["s"][idx] - r["s"]).max()
    m = edge_mask(desc)[idx]
    qg, qr = g["q"][idx][m], r["q"][m]
    eq = np.minimum(np.abs(qg - qr).max(1), np.abs(qg + qr).max(1)).max() if m.any() else 0.0
    return ex, es, eq


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_single_rod_fp64_120_frames():
    """32-pill rod, FP64 on both sides, 10 substeps x 4 iterations, 120 frames."""
    desc = scenes.straight_rod(32)
    say("case: single rod fp64, 120 frames")
    sc = viper.Scene(desc, "f64")
    o = oracle.OracleScene(desc, "f64")
    for _ in range(120):
        sc.step(1 / 60, 10, 4)
        o.step(1 / 60, 10, 4)
    sc.sync()
    ex, es, eq = errors(desc, sc.state(), o.get_state())
    say("fp64 errors", ex, es, eq)
    assert ex < 1e-9 and es < 1e-9 and eq < 1e-9


def test_mixed_lengths_ragged_fp32_and_fp64():
    """Rods of 2..64 pills packed several per wave (ragged wave tails), both precisions,
    all four constraint types, a few frames; every pill compared."""
    rng = np.random.default_rng(21)
    lens = [2, 3, 64, 5, 17, 31, 32, 33, 63, 4, 9, 12, 2, 40, 24, 7]
    lens += list(rng.integers(2, 65, 40))
    base = scenes.helix_rods(len(lens), 64, seed=22)
    offs = [0]
    pos, rad, pin = [], [], []
    for k, n in enumerate(lens):
        a = base.rod_offsets[k]
        pos.append(base.rest_pos[a:a + n]); rad.append(base.rest_radius[a:a + n])
        p = np.zeros(n, np.uint8); p[0] = 1
        pin.append(p)
        offs.append(offs[-1] + n)
    act = rng.uniform(0.8, 1.2, len(lens))
    desc = scenes.SceneDesc(np.asarray(offs, np.int32), np.concatenate(pos), np.concatenate(rad),
                            np.concatenate(pin), act, base.compliance[:len(lens)].copy(),
                            np.arange(len(lens), dtype=np.int32))
    for prec, tol in (("f64", 1e-9), ("f32", TOL)):
        say("case: mixed lengths", prec)
        sc = viper.Scene(desc, prec)
        o = oracle.OracleScene(desc, "f64")
        for _ in range(3):
            sc.step(1 / 60, 20, 8)
            o.step(1 / 60, 20, 8)
        sc.sync()
        ex, es, eq = errors(desc, sc.state(), o.get_state())
        say(prec, "errors", ex, es, eq)
        assert ex < tol and es < tol and eq < tol


def test_helix_4096x64_fp32_sampled_full_horizon():
    """The 4096 x 64 FP32 helix scene for 100 frames of 20 x 8, in the launch
    configuration the benchmark times; 8 sampled rods compared with the FP64 oracle
    (rods are independent) and with the FP32 oracle (rounding floor)."""
    desc = scenes.helix_rods(4096, 64, seed=1)
    say("case: helix 4096x64 fp32 100 frames")
    sc = viper.Scene(desc, "f32")
    t0 = time.time()
    for _ in range(100):
        sc.step(1 / 60, 20, 8)
    sc.sync()
    g = sc.state()
    say("gpu done", time.time() - t0)
    rods = [0, 1, 777, 1500, 2048, 3001, 4000, 4095]
    sub = desc.subset(rods)
    o = oracle.OracleScene(sub, "f64")
    of = oracle.OracleScene(sub, "f32")
    for _ in range(100):
        o.step(1 / 60, 20, 8, threads=8)
        of.step(1 / 60, 20, 8, threads=8)
    idx = desc.pill_index(rods)
    ex, es, eq = errors(desc, g, o.get_state(), idx)
    fx, fs, fq = errors(sub, of.get_state(), o.get_state())
    say("gpu-vs-fp64", ex, es, eq, "fp32-oracle floor", fx, fs, fq)
    assert ex < TOL and es < TOL and eq < TOL


def test_modes_agree():
    """One launch per frame, one per substep, and per-stage launches give the same result."""
    desc = scenes.helix_rods(64, 64, seed=5)
    res = []
    for mode in (viper.MODE_FRAME, viper.MODE_SUBSTEP, viper.MODE_ITERATION):
        say("case: mode", mode)
        sc = viper.Scene(desc, "f32")
        for _ in range(3):
            sc.step(1 / 60, 20, 8, mode=mode)
        sc.sync()
        res.append(sc.state())
    for r in res[1:]:
        for k in ("x", "s", "q"):
            assert np.abs(r[k] - res[0][k]).max() < 1e-5


def test_deterministic_and_state_roundtrip():
    desc = scenes.helix_rods(128, 64, seed=6)
    a = viper.Scene(desc, "f32")
    b = viper.Scene(desc, "f32")
    for _ in range(2):
        a.step(1 / 60, 20, 8)
        b.step(1 / 60, 20, 8)
    sa, sb = a.state(), b.state()
    for k in sa:
        assert np.array_equal(sa[k], sb[k])
    # resume: copy a's full state into a fresh scene and continue both
    c = viper.Scene(desc, "f32")
    for k in ("x", "v", "s", "sd", "q", "om"):
        c.set(k, a.get(k))
    a.step(1 / 60, 20, 8)
    c.step(1 / 60, 20, 8)
    sa, sc = a.state(), c.state()
    for k in sa:
        assert np.array_equal(sa[k], sc[k]), k


def test_unit_quaternions_and_nan_flag():
    desc = scenes.helix_rods(256, 64, seed=8)
    sc = viper.Scene(desc, "f32")
    for _ in range(5):
        sc.step(1 / 60, 20, 8)
    sc.sync()
    q = sc.state()["q"][edge_mask(desc)]
    assert np.abs(np.linalg.norm(q, axis=1) - 1).max() < 1e-6
    x = sc.get("x").clone()
    x[17, 1] = float("nan")
    sc.set("x", x)
    sc.step(1 / 60, 2, 2)
    with pytest.raises(viper.ViperError) as ei:
        sc.sync()
    assert ei.value.status == viper.ERR_NAN
    sc.sync()   # cleared


def test_empty_and_tiny_scenes():
    desc = scenes.straight_rod(2)
    sc = viper.Scene(desc, "f32")
    o = oracle.OracleScene(desc, "f64")
    for _ in range(10):
        sc.step(1 / 60, 5, 3)
        o.step(1 / 60, 5, 3)
    sc.sync()
    ex, es, eq = errors(desc, sc.state(), o.get_state())
    assert ex < TOL and es < TOL and eq < TOL
    # zero iterations: prediction + velocity only
    sc.step(1 / 60, 3, 0)
    sc.sync()
