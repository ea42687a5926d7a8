"""Cross-section stretch (eq. stretch_xy) on the GPU against the oracle.

Workload: helix rods of 13 pills (24 rods, seed 2, rods starting on odd and even wave slots)
with the constraint on every other rod (so lanes of one wavefront differ), compliance 1e-7.
Checks:
- FP64: one frame (20 substeps x 8 iterations) in the fused frame kernel (SUBSTEP mode) and
  in the split ITERATION launches equals the oracle's frame to rounding, with the Gauss-Seidel
  and with the Jacobi solver; the constraint changes the result (the oracle without it
  differs);
- FP32: one frame within the 1e-4 bound of the other parity tests;
- the pool and the adjoint reject a scene that turns it on; all +inf equals no array.
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
from test_gpu_rods import errors  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def with_sr(desc, comp=1e-7):
    c = np.full(desc.num_rods, np.inf)
    c[::2] = comp
    return dataclasses.replace(desc, cross_compliance=c)


def frame_pair(desc, prec, mode, sub=20, iters=8):
    sc = viper.Scene(desc, prec)
    sc.step(1 / 60, sub, iters, mode=mode)
    sc.sync()
    o = oracle.OracleScene(desc, "f64")
    o.step(1 / 60, sub, iters)
    return sc.state(), o.get_state()


@pytest.mark.parametrize("solver,mode", [("gauss_seidel", "substep"), ("gauss_seidel", "iteration"),
                                         ("jacobi", "iteration")])
def test_fp64_frame_matches_oracle(solver, mode):
    desc = with_sr(dataclasses.replace(scenes.helix_rods(24, 13, seed=2), solver=solver))
    say("case: cross stretch fp64", solver, mode, desc.num_pills)
    m = viper.MODE_SUBSTEP if mode == "substep" else viper.MODE_ITERATION
    g, r = frame_pair(desc, "f64", m)
    ex, es, eq = errors(desc, g, r)
    say("fp64 errors", ex, es, eq)
    assert ex < 1e-10 and es < 1e-10 and eq < 1e-10
    o = oracle.OracleScene(dataclasses.replace(desc, cross_compliance=None), "f64")
    o.step(1 / 60, 20, 8)
    diff = np.abs(o.get_state()["s"] - r["s"]).max()
    say("scale change made by the constraint", diff)
    assert diff > 1e-8


def test_fp32_frame_within_tolerance():
    desc = with_sr(scenes.helix_rods(24, 13, seed=2))
    g, r = frame_pair(desc, "f32", viper.MODE_SUBSTEP)
    ex, es, eq = errors(desc, g, r)
    say("fp32 errors", ex, es, eq)
    assert ex < 1e-4 and es < 1e-4 and eq < 1e-4


def test_all_off_equals_no_array_and_rejections():
    base = scenes.helix_rods(4, 8, seed=1)
    a = viper.Scene(base, "f32")
    b = viper.Scene(dataclasses.replace(base, cross_compliance=np.full(4, np.inf)), "f32")
    for sc in (a, b):
        sc.step(1 / 60, 10, 4)
        sc.sync()
    sa, sb = a.state(), b.state()
    for k in ("x", "s", "q"):
        assert np.array_equal(sa[k], sb[k]), k
    desc = with_sr(base)
    sc = viper.Scene(desc, "f32")
    with pytest.raises(viper.ViperError) as ei:
        sc.step_checkpointed(1 / 60, 1, 4, 4)
    assert ei.value.status == viper.ERR_INVALID
    pool = viper.Pool(16 << 20, precision="f32")
    with pytest.raises(viper.ViperError) as ei:
        pool.admit(desc)
    assert ei.value.status == viper.ERR_INVALID
