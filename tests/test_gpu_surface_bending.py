"""Surface bending (Sec. 5: the Laplacian of the scale along the rod) on the GPU against the
oracle.

Workloads: helix rods of 13 pills (24 rods, seed 2: rods start on odd and even wave slots, so
owners of all three colours sit in both slots of a lane and at lane boundaries) and 64-pill
rods (a subset of the 4096 x 64 helix scene), the constraint on every other rod (lanes of one
wavefront differ), compliance 1e-6.  Checks:
- FP64: one frame (20 substeps x 8 iterations) in the fused frame kernel and in the split
  ITERATION launches equals the oracle's to rounding, also together with the cross-section
  stretch; the constraint changes the result;
- FP32: one frame within the 1e-4 bound of the other parity tests;
- rejections: the pool and the adjoint.
"""
import dataclasses
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1906_05260_amd import scenes, viper  # noqa: E402

sys.path.insert(0, __file__.rsplit("/", 1)[0])
from test_gpu_rods import errors, local_subset  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def with_sb(desc, comp=1e-6, sr=False):
    c = np.full(desc.num_rods, np.inf)
    c[::2] = comp
    desc = dataclasses.replace(desc, bending_compliance=c)
    if sr:
        c2 = np.full(desc.num_rods, np.inf)
        c2[1::3] = 1e-7
        desc = dataclasses.replace(desc, cross_compliance=c2)
    return desc


def frame_pair(desc, prec, mode, sub=20, iters=8):
    sc = viper.Scene(desc, prec)
    sc.step(1 / 60, sub, iters, mode=mode)
    sc.sync()
    o = oracle.OracleScene(desc, "f64")
    o.step(1 / 60, sub, iters)
    return sc.state(), o.get_state()


@pytest.mark.parametrize("case,mode,sr", [("helix24x13", "substep", False), ("helix24x13", "iteration", False),
                                          ("helix24x13", "substep", True), ("helix4096x64_subset", "substep", False)])
def test_fp64_frame_matches_oracle(case, mode, sr):
    if case == "helix24x13":
        base = scenes.helix_rods(24, 13, seed=2)
    else:
        base = local_subset(scenes.helix_rods(4096, 64, seed=1), list(range(0, 4096, 128)))
    desc = with_sb(base, sr=sr)
    say("case: surface bending fp64", case, mode, "with cross stretch" if sr else "", desc.num_pills)
    m = viper.MODE_SUBSTEP if mode == "substep" else viper.MODE_ITERATION
    g, r = frame_pair(desc, "f64", m)
    ex, es, eq = errors(desc, g, r)
    say("fp64 errors", ex, es, eq)
    assert ex < 1e-10 and es < 1e-10 and eq < 1e-10
    o = oracle.OracleScene(dataclasses.replace(desc, bending_compliance=None), "f64")
    o.step(1 / 60, 20, 8)
    diff = np.abs(o.get_state()["s"] - r["s"]).max()
    say("scale change made by the constraint", diff)
    assert diff > 1e-8


def test_fp32_frame_within_tolerance():
    desc = with_sb(scenes.helix_rods(24, 13, seed=2))
    g, r = frame_pair(desc, "f32", viper.MODE_SUBSTEP)
    ex, es, eq = errors(desc, g, r)
    say("fp32 errors", ex, es, eq)
    assert ex < 1e-4 and es < 1e-4 and eq < 1e-4


def test_rejections():
    desc = with_sb(scenes.helix_rods(4, 8, seed=1))
    sc = viper.Scene(desc, "f32")
    with pytest.raises(viper.ViperError) as ei:
        sc.step_checkpointed(1 / 60, 1, 4, 4)
    assert ei.value.status == viper.ERR_INVALID
    pool = viper.Pool(16 << 20, precision="f32")
    with pytest.raises(viper.ViperError) as ei:
        pool.admit(desc)
    assert ei.value.status == viper.ERR_INVALID
