"""Jacobi solver with averaging (Sec. 7, the paper's engine) for the rod constraints on the GPU
against the oracle's Jacobi mode.

Workloads: helix rods of 13 pills (24 rods, seed 2: rods start on odd wave slots as well as
even ones) and of 64 pills (a subset of the 4096 x 64 helix scene), and the stretched-rod
scenario of the paper's convergence experiment.  Checks:
- FP64: one frame (20 substeps x 8 iterations) equals the oracle's Jacobi frame to rounding,
  and differs from the Gauss-Seidel frame (the solvers are distinct);
- FP32: one frame within the 1e-4 bound of the other parity tests;
- stretched rod: the state after 1, 10 and 100 Jacobi iterations of one substep equals the
  oracle's;
- the captured-graph frame equals the eager launches bit for bit;
- the single-kernel modes, the pool and the adjoint reject a Jacobi scene.
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


def jacobi(desc):
    return dataclasses.replace(desc, solver="jacobi")


def frame_pair(desc, prec, sub=20, iters=8):
    sc = viper.Scene(desc, prec)
    sc.step(1 / 60, sub, iters, mode=viper.MODE_ITERATION)
    sc.sync()
    o = oracle.OracleScene(desc, "f64")
    o.step(1 / 60, sub, iters)
    return sc.state(), o.get_state()


@pytest.mark.parametrize("case", ["helix24x13", "helix4096x64_subset"])
def test_fp64_frame_matches_oracle(case):
    if case == "helix24x13":
        desc = scenes.helix_rods(24, 13, seed=2)
    else:
        desc = local_subset(scenes.helix_rods(4096, 64, seed=1), list(range(0, 4096, 128)))
    desc = jacobi(desc)
    say("case: jacobi fp64", case, desc.num_pills)
    g, r = frame_pair(desc, "f64")
    ex, es, eq = errors(desc, g, r)
    say("fp64 jacobi errors", ex, es, eq)
    assert ex < 1e-10 and es < 1e-10 and eq < 1e-10
    o = oracle.OracleScene(dataclasses.replace(desc, solver="gauss_seidel"), "f64")
    o.step(1 / 60, 20, 8)
    assert np.abs(o.get_state()["x"] - r["x"]).max() > 1e-6


def test_fp32_frame_within_tolerance():
    desc = jacobi(scenes.helix_rods(24, 13, seed=2))
    g, r = frame_pair(desc, "f32")
    ex, es, eq = errors(desc, g, r)
    say("fp32 jacobi errors", ex, es, eq)
    assert ex < 1e-4 and es < 1e-4 and eq < 1e-4


@pytest.mark.parametrize("iters", [1, 10, 100])
def test_stretched_rod_iterations(iters):
    """The convergence scenario (a rod stretched instantly to twice its length between two
    pinned bars): one substep of `iters` Jacobi iterations, GPU FP64 vs oracle."""
    n = 12
    pos = np.zeros((n, 3))
    pos[:, 0] = 0.01 * np.arange(n)
    desc = scenes.SceneDesc(np.asarray([0, n], np.int32), pos, np.full(n, 0.004), np.zeros(n, np.uint8), np.ones(1),
                            np.asarray([[1e-6, 1e-7, 1e-7, 1e-5]]), np.zeros(1, np.int32), name="stretched",
                            solver="jacobi")
    desc.pinned[[0, n - 1]] = 1
    x = pos.copy()
    x[-1, 0] *= 2.0
    sc = viper.Scene(desc, "f64")
    sc.set("x", x)
    o = oracle.OracleScene(desc, "f64")
    o.set_state(x=x)
    sc.step(1 / 600, 1, iters, mode=viper.MODE_ITERATION)
    sc.sync()
    o.step(1 / 600, 1, iters)
    ex, es, eq = errors(desc, sc.state(), o.get_state())
    say("stretched rod", iters, "iterations:", ex, es, eq)
    assert ex < 1e-10 and es < 1e-10 and eq < 1e-10


def test_graph_equals_eager():
    desc = jacobi(scenes.helix_rods(24, 13, seed=2))
    a, b = viper.Scene(desc, "f32"), viper.Scene(desc, "f32")
    for _ in range(3):
        a.step(1 / 60, 20, 8)                              # default: captured graph
        b.step(1 / 60, 20, 8, mode=viper.MODE_ITERATION)
    a.sync()
    b.sync()
    sa, sb = a.state(), b.state()
    for k in ("x", "v", "s", "q"):
        assert np.array_equal(sa[k], sb[k]), k


def test_rejections():
    desc = jacobi(scenes.helix_rods(4, 8, seed=1))
    sc = viper.Scene(desc, "f32")
    for mode in (viper.MODE_FRAME, viper.MODE_SUBSTEP):
        with pytest.raises(viper.ViperError) as ei:
            sc.step(1 / 60, 4, 4, mode=mode)
        assert ei.value.status == viper.ERR_INVALID
    with pytest.raises(viper.ViperError) as ei:
        sc.step_checkpointed(1 / 60, 1, 4, 4)
    assert ei.value.status == viper.ERR_INVALID
    pool = viper.Pool(16 << 20, precision="f32")
    with pytest.raises(viper.ViperError) as ei:
        pool.admit(desc)
    assert ei.value.status == viper.ERR_INVALID
