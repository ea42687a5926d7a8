"""Synthetic workload generators: sizes and structure as the workloads state them."""
import numpy as np

from paper_1906_05260_amd import scenes


def _capsule_ok(desc, caps):
    """A capsule id is the first pill of an edge: not the last pill of its rod."""
    last = set((np.asarray(desc.rod_offsets[1:]) - 1).tolist())
    return all(int(c) not in last for c in np.asarray(caps).reshape(-1))


def test_helix_scene_shape():
    d = scenes.helix_rods(64, 64, seed=1)
    assert d.num_rods == 64 and d.num_pills == 64 * 64
    assert np.all(d.pinned[d.rod_offsets[:-1]] == 1) and d.pinned.sum() == 64
    assert d.rest_radius.min() >= 0.002 and d.rest_radius.max() <= 0.008
    assert d.compliance.min() >= 1e-8 and d.compliance.max() <= 1e-4
    # pills 1 cm apart in arc length along each helix (chord slightly shorter)
    seg = np.linalg.norm(np.diff(d.rest_pos.reshape(64, 64, 3), axis=1), axis=2)
    assert np.all(seg > 0.009) and np.all(seg <= 0.01 + 1e-12)     # chords of 1 cm arcs


def test_straight_rods_and_targets():
    d, t = scenes.straight_rods(16, 32, seed=4)
    assert d.num_pills == 512 and t.shape == (16, 3)
    assert np.all((d.activation >= 0.8) & (d.activation <= 1.2))
    ends = d.rest_pos[np.asarray(d.rod_offsets[1:]) - 1]
    assert np.abs(t - ends).max() < 0.06


def test_muscle_scene_size_and_mesh():
    d, mesh = scenes.muscle_scene(num_muscles=4, seed=2, target_pills=None, mesh_vertices=2000)
    assert d.collisions
    assert np.all(d.pinned[d.rod_offsets[:-1]] == 1) and np.all(d.pinned[np.asarray(d.rod_offsets[1:]) - 1] == 1)
    assert mesh.rest_v.shape == (2000, 3) and mesh.caps.shape == (2000, 4)
    assert np.allclose(mesh.w.sum(1), 1.0, atol=1e-6) and _capsule_ok(d, mesh.caps)


def test_muscle_scene_target_pill_range():
    d, _ = scenes.muscle_scene(num_muscles=64, seed=2, mesh_vertices=0)
    assert 45000 <= d.num_pills <= 55000


def test_octopus_scene():
    d, mesh = scenes.octopus_scene(num_models=9, mesh_vertices_per_model=500)
    assert d.num_pills == 9 * 37 and d.num_rods == 9 * 9
    assert np.all(np.bincount(d.group) == 9)                  # 1 body + 8 arms per model
    assert d.pinned.sum() == 9 * 9                            # body top + 8 arm roots
    assert mesh.rest_v.shape == (9 * 500, 3) and _capsule_ok(d, mesh.caps)
    # influences stay within the vertex's own model
    cap_model = np.repeat(d.group, np.diff(d.rod_offsets))
    vm = np.repeat(np.arange(9), 500)
    assert np.all(cap_model[mesh.caps] == vm[:, None])


def test_serving_requests_poisson_and_sizes():
    reqs = scenes.serving_requests(rate=200, duration=0.2, seed=3, min_pills=1000, max_pills=20000, frames=5)
    assert 20 <= len(reqs) <= 70
    arr = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(arr) > 0) and arr[-1] <= 0.2
    sizes = np.array([r.desc.num_pills for r in reqs])
    assert sizes.min() >= 900 and sizes.max() <= 30000
    assert {r.kind for r in reqs} <= {"helix", "muscle"}
