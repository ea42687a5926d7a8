"""Serving pool (continuous batching) on the GPU.

- Each scene's result is the same alone and in the mix (staggered admissions and
  retirements, collision-free and contact scenes together), within the stated tolerance
  (1e-4 relative position error; in practice bit-identical: every scene runs the same
  per-wave / per-block arithmetic whatever else shares the launch).
- Admission is refused when no free range fits the footprint and succeeds after a
  retirement frees one.
- A pooled scene matches the FP64 oracle: a collision-free scene stepped in the shared
  launch over frames (FP64 1e-9, FP32 1e-4), a contact scene over one substep from the
  same state (candidate pairs equal, FP64 1e-9, FP32 1e-4).
- The batched server beats the plain per-scene path on the same requests.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1906_05260_amd import scenes, serve, viper  # noqa: E402
from test_gpu_rods import errors  # noqa: E402

DT, SUB, IT = 1 / 60, 20, 8


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_alone(desc, frames, prec="f32"):
    sc = viper.Scene(desc, prec)
    for _ in range(frames):
        sc.step(DT, SUB, IT)
    sc.sync()
    return sc.state()


@pytest.mark.parametrize("prec,split", [("f32", False), ("f64", False), ("f32", True)])
def test_alone_equals_mix(prec, split):
    """split: the two classes (collision-free, with contacts) stepped separately on two
    streams, as the serving loop does, instead of one joint pool step."""
    A = scenes.helix_rods(37, 64, seed=11)
    B, _ = scenes.muscle_scene(num_muscles=6, seed=12, target_pills=None, mesh_vertices=0)
    C = scenes.helix_rods(5, 64, seed=13)
    D, _ = scenes.muscle_scene(num_muscles=3, seed=14, target_pills=None, mesh_vertices=0)
    pool = viper.Pool(512 << 20, max_scenes=8, precision=prec)
    plan = {}                                    # slot -> (desc, frames stepped)
    frames = {}

    def admit(desc, name):
        s = pool.admit(desc)
        assert s is not None
        plan[name] = s
        frames[name] = 0

    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

    def step(n):
        for _ in range(n):
            if split:
                pool.step(DT, SUB, IT, stream=s1, classes=1)
                pool.step(DT, SUB, IT, stream=s2, classes=2)
                torch.cuda.synchronize()
            else:
                pool.step(DT, SUB, IT)
            for k in frames:
                if k not in retired:
                    frames[k] += 1

    retired = {}
    admit(A, "A")
    step(2)
    admit(B, "B")
    admit(C, "C")
    step(3)
    st = pool.scene(plan["A"]).state()
    retired["A"] = st
    pool.retire(plan["A"])
    admit(D, "D")
    step(2)
    for name in ("B", "C", "D"):
        retired[name] = pool.scene(plan[name]).state()
    descs = {"A": A, "B": B, "C": C, "D": D}
    for name, desc in descs.items():
        alone = run_alone(desc, frames[name], prec)
        e = errors(desc, retired[name], alone)
        same = all(np.array_equal(retired[name][k], alone[k]) for k in ("x", "s", "q"))
        say(prec, "split" if split else "joint", name, "frames", frames[name], "errors", e, "bit-identical", same)
        assert max(e) < 1e-4
    for name in ("B", "C", "D"):
        pool.scene(plan[name]).sync()


@pytest.mark.parametrize("prec,tol,frames", [("f64", 1e-9, 3), ("f32", 1e-4, 2)])
def test_pooled_collision_free_scene_matches_oracle(prec, tol, frames):
    A = scenes.helix_rods(16, 64, seed=1)
    B, _ = scenes.muscle_scene(num_muscles=3, seed=52, target_pills=None, mesh_vertices=0)
    C = scenes.helix_rods(24, 64, seed=53)
    pool = viper.Pool(256 << 20, max_scenes=4, precision=prec)
    sc_, sa, sb = pool.admit(C), pool.admit(A), pool.admit(B)
    o = oracle.OracleScene(A, "f64")
    for _ in range(frames):
        pool.step(DT, SUB, IT)
        o.step(DT, SUB, IT)
    e = errors(A, pool.scene(sa).state(), o.get_state())
    say("pooled collision-free scene vs oracle", prec, frames, "frames:", e)
    assert max(e) < tol
    for s in (sa, sb, sc_):
        pool.scene(s).sync()


@pytest.mark.parametrize("prec,tol,seed", [("f64", 1e-9, 3), ("f32", 1e-4, 4)])
def test_pooled_contact_substep_matches_oracle(prec, tol, seed):
    """The scenes of the single-scene contact substep tests (seed 3 in FP64, seed 4 in FP32:
    the soft log-uniform scale compliances of seed 3 amplify FP32 rounding of the scales to
    ~1e-3, in the FP32 oracle as much as on the GPU), stepped in a pool beside others."""
    B, _ = scenes.muscle_scene(num_muscles=8, seed=seed, target_pills=None, mesh_vertices=0, compliance="loguniform")
    A = scenes.helix_rods(8, 64, seed=54)
    D, _ = scenes.muscle_scene(num_muscles=4, seed=55, target_pills=None, mesh_vertices=0, compliance="loguniform")
    pool = viper.Pool(256 << 20, max_scenes=4, precision=prec)
    sa, sb, sd = pool.admit(A), pool.admit(B), pool.admit(D)
    for _ in range(5):                      # until contacts are active (as the single-scene test)
        pool.step(DT, 4, 4)
    scene = pool.scene(sb)
    st0 = scene.state()
    o = oracle.OracleScene(B, "f64")
    o.set_state(**st0)
    pool.step(DT, 1, 8)
    o.step(DT, 1, 8, collide=True)
    torch.cuda.synchronize()
    assert np.array_equal(scene.contacts(), o.pairs())
    assert (o.active_count() > 0).any()
    e = errors(B, scene.state(), o.get_state())
    o32 = oracle.OracleScene(B, "f32")          # the FP32 rounding floor of the same substep
    o32.set_state(**st0)
    o32.step(DT, 1, 8, collide=True)
    floor = errors(B, o32.get_state(), o.get_state())
    say("pooled contact substep vs oracle", prec, e, "FP32 oracle floor", floor, "pairs", len(o.pairs()))
    assert max(e) < tol
    for s in (sa, sb, sd):
        pool.scene(s).sync()


def test_admission_by_footprint():
    big = scenes.helix_rods(1024, 64, seed=21)
    small = scenes.helix_rods(8, 64, seed=22)
    fp_big = viper.footprint(big)
    pool = viper.Pool(int(fp_big * 1.3) + (4 << 20), max_scenes=4)
    s1 = pool.admit(big)
    assert s1 is not None
    assert pool.admit(big) is None          # no free range fits a second one
    s2 = pool.admit(small)
    assert s2 is not None                   # but a small one still fits
    pool.step(DT, SUB, IT)
    pool.retire(s1)
    s3 = pool.admit(big)                    # the freed range is reused
    assert s3 is not None
    pool.step(DT, SUB, IT)
    pool.scene(s3).sync()
    info = pool.info()
    assert info["resident"] == 2


def test_batched_beats_plain():
    reqs = scenes.serving_requests(rate=200, duration=0.25, seed=31, min_pills=1000, max_pills=30000, frames=10)
    say("requests", len(reqs), "pills", sum(r.desc.num_pills for r in reqs))
    b = serve.serve_batched(reqs, pool_bytes=4 << 30)
    p = serve.serve_plain(reqs)
    say("batched", b)
    say("plain", p)
    # a scene that fails (here a marginally stable FP32 muscle scene whose scales the rod
    # iterations drive through zero; the FP64 oracle does the same from its state) fails at
    # the same frame on both paths: a scene's arithmetic is the same alone and in the mix
    key = lambda f: (f["arrival"], f["frames_done"], f["status"])
    assert sorted(map(key, b["failed"])) == sorted(map(key, p["failed"]))
    lost = sum(next(r.frames for r in reqs if r.arrival == f["arrival"]) - f["frames_done"] for f in b["failed"])
    assert b["frames"] == p["frames"] == sum(r.frames for r in reqs) - lost
    assert b["pill_frames_per_s"] > p["pill_frames_per_s"]
    assert b["latency_ms_p99"] < p["latency_ms_p99"]
