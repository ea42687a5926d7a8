"""Host-only checks of the C ABI: the library loads, exports every declared symbol, and
validates descriptions / computes footprints without touching a GPU."""
import ctypes
import dataclasses
import os
import re

import numpy as np
import pytest

from paper_1906_05260_amd import scenes, viper

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "viper.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(viper_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = viper.lib()
    names = declared_symbols()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert sorted(viper.ABI_SYMBOLS) == names


def test_footprint_scales_and_validates():
    d = scenes.helix_rods(16, 64, seed=1)
    f32 = viper.footprint(d, "f32")
    f64 = viper.footprint(d, "f64")
    assert f64 > f32 > 16 * 64 * 4 * 30
    d2 = scenes.helix_rods(32, 64, seed=1)
    assert viper.footprint(d2, "f32") > f32
    # collisions add the contact buffers
    assert viper.footprint(d, "f32", collisions=True) > f32


@pytest.mark.parametrize("mutate,msg", [
    (lambda d: d.rest_radius.__setitem__(3, 0.0), "rest_radius"),
    (lambda d: d.rest_radius.__setitem__(3, np.nan), "rest_radius"),
    (lambda d: d.compliance.__setitem__((0, 1), -1.0), "compliance"),
    (lambda d: d.activation.__setitem__(0, 0.0), "activation"),
    (lambda d: d.rest_pos.__setitem__(1, d.rest_pos[0]), "coincide"),
])
def test_invalid_descriptions_rejected(mutate, msg):
    d = scenes.helix_rods(4, 8, seed=2)
    mutate(d)
    with pytest.raises(viper.ViperError) as ei:
        viper.footprint(d)
    assert ei.value.status == viper.ERR_INVALID
    assert msg in str(ei.value)


def test_rod_length_limits():
    """A rod lives in one wavefront: 2..128 pills (two slots per lane)."""
    for n in (2, 64, 65, 128):
        viper.footprint(scenes.straight_rod(n))
    for n in (1, 129):
        d = scenes.straight_rod(max(n, 2))
        if n == 1:
            d.rod_offsets = np.asarray([0, 1], np.int32)
            d.rest_pos = d.rest_pos[:1]
        else:
            d = scenes.straight_rod(129)
        with pytest.raises(viper.ViperError) as ei:
            viper.footprint(d)
        assert ei.value.status == viper.ERR_INVALID


def test_infinite_compliance_disables_type():
    d = scenes.helix_rods(4, 8, seed=2)
    d.compliance[:, 3] = np.inf
    viper.footprint(d)


def test_create_requires_workspace_and_alignment():
    L = viper.lib()
    d = scenes.helix_rods(2, 8, seed=2)
    h = viper._DescHolder(d, "f32")
    out = ctypes.c_void_p()
    assert L.viper_create_scene(ctypes.byref(h.c), None, 0, None, ctypes.byref(out)) == viper.ERR_INVALID
    assert L.viper_create_scene(ctypes.byref(h.c), ctypes.c_void_p(0x1001), 1 << 30, None,
                                ctypes.byref(out)) == viper.ERR_INVALID
    assert L.viper_create_scene(ctypes.byref(h.c), ctypes.c_void_p(0x100000), 16, None,
                                ctypes.byref(out)) == viper.ERR_NO_CAPACITY
    assert b"workspace" in L.viper_last_error()


def test_step_rejects_bad_arguments_without_gpu():
    L = viper.lib()
    assert L.viper_step(None, 1 / 60, 1, 1, None) == viper.ERR_INVALID
    assert L.viper_sync(None, None) == viper.ERR_INVALID


def test_bundling_sections_footprint_and_validation():
    """Bundling sections (Sec. 7.3) add their buffers to the footprint; empty sections,
    out-of-range pills and a pill in two sections are rejected on the host."""
    d, _ = scenes.muscle_scene(num_muscles=2, seed=5, target_pills=None, mesh_vertices=0)
    base = viper.footprint(d)
    b, _ = scenes.muscle_scene(num_muscles=2, seed=5, target_pills=None, mesh_vertices=0, bundling=True)
    assert viper.footprint(b) > base
    for offs, pills, msg in (([0, 0, 2], [0, 1], "empty"), ([0, 2], [0, b.num_pills], "range"),
                             ([0, 2, 4], [0, 1, 1, 2], "two sections"), ([1, 2], [0, 1], "section_offsets[0]")):
        bad = dataclasses.replace(b, section_offsets=np.asarray(offs, np.int32), section_pills=np.asarray(pills, np.int32))
        with pytest.raises(viper.ViperError) as ei:
            viper.footprint(bad)
        assert ei.value.status == viper.ERR_INVALID and msg in str(ei.value), str(ei.value)


def test_floor_validation():
    """The half-plane floor (Sec. 7) needs a finite nonzero normal and a finite offset."""
    d = scenes.helix_rods(2, 8, seed=1)
    viper.footprint(dataclasses.replace(d, floor=(0.0, 2.0, 0.0, -0.1)))
    for fl in ((0.0, 0.0, 0.0, 0.0), (np.nan, 1.0, 0.0, 0.0), (0.0, 1.0, 0.0, np.inf)):
        with pytest.raises(viper.ViperError) as ei:
            viper.footprint(dataclasses.replace(d, floor=fl))
        assert ei.value.status == viper.ERR_INVALID and "floor" in str(ei.value)


def test_cross_stretch_validation():
    """Cross-section stretch compliances (eq. stretch_xy): one per rod, >= 0 or +inf; the
    footprint grows by one per-edge rest array and one multiplier array when it is off or on
    alike (the layout does not depend on it)."""
    d = scenes.helix_rods(2, 8, seed=1)
    base = viper.footprint(d)
    assert viper.footprint(dataclasses.replace(d, cross_compliance=np.array([1e-6, np.inf]))) == base
    for bad in (np.array([-1.0, 0.0]), np.array([np.nan, 0.0])):
        with pytest.raises(viper.ViperError) as ei:
            viper.footprint(dataclasses.replace(d, cross_compliance=bad))
        assert ei.value.status == viper.ERR_INVALID and "cross_compliance" in str(ei.value)
    with pytest.raises(ValueError):
        viper.footprint(dataclasses.replace(d, cross_compliance=np.zeros(3)))


def _with_bones(d, nb=2):
    P = d.num_pills
    rest = np.tile(np.hstack([np.eye(3), np.zeros((3, 1))])[None], (nb, 1, 1))
    pb = np.tile(np.array([[0, nb - 1]], np.int32), (P, 1))
    pw = np.tile(np.array([[0.25, 0.75]]), (P, 1))
    return dataclasses.replace(d, bone_rest=rest, pill_bones=pb, pill_bone_weights=pw)


def test_bone_validation():
    """Bones (Sec. 8.2): rest transforms finite with an invertible linear part, weights finite
    and >= 0, a bone id in range wherever its weight is positive (ignored where it is zero);
    the workspace grows by the bone and influence arrays."""
    d = scenes.helix_rods(2, 8, seed=1)
    base = viper.footprint(d)
    assert viper.footprint(_with_bones(d)) > base
    ok = _with_bones(d)
    ok.pill_bones[3] = (-1, 1)
    ok.pill_bone_weights[3] = (0.0, 1.0)
    viper.footprint(ok)
    bad = []
    b = _with_bones(d)
    b.bone_rest[1, :, :3] = 0.0
    bad.append((b, "bone_rest"))
    b = _with_bones(d)
    b.bone_rest[0, 1, 3] = np.nan
    bad.append((b, "bone_rest"))
    b = _with_bones(d)
    b.pill_bone_weights[5, 0] = -0.1
    bad.append((b, "pill_bone_weights"))
    b = _with_bones(d)
    b.pill_bones[2, 1] = 2
    bad.append((b, "pill_bones"))
    for b, msg in bad:
        with pytest.raises(viper.ViperError) as ei:
            viper.footprint(b)
        assert ei.value.status == viper.ERR_INVALID and msg in str(ei.value), str(ei.value)


def test_surface_bending_validation():
    """Surface bending compliances: one per rod, >= 0 or +inf, and only with the Gauss-Seidel
    solver (the Jacobi path does not carry it)."""
    d = scenes.helix_rods(2, 8, seed=1)
    viper.footprint(dataclasses.replace(d, bending_compliance=np.array([1e-6, np.inf])))
    for bad in (np.array([-1.0, 0.0]), np.array([np.nan, 0.0])):
        with pytest.raises(viper.ViperError) as ei:
            viper.footprint(dataclasses.replace(d, bending_compliance=bad))
        assert ei.value.status == viper.ERR_INVALID and "bending_compliance" in str(ei.value)
    with pytest.raises(viper.ViperError) as ei:
        viper.footprint(dataclasses.replace(d, bending_compliance=np.array([1e-6, np.inf]), solver="jacobi"))
    assert ei.value.status == viper.ERR_INVALID and "Gauss-Seidel" in str(ei.value)
    viper.footprint(dataclasses.replace(d, bending_compliance=np.array([np.inf, np.inf]), solver="jacobi"))
    with pytest.raises(ValueError):
        viper.footprint(dataclasses.replace(d, bending_compliance=np.zeros(3)))


def test_volume_bending_validation():
    """The volume-bending coupling is a Gauss-Seidel-only option: a Jacobi scene that turns it
    on is rejected; the footprint does not depend on it."""
    d = scenes.helix_rods(2, 8, seed=1)
    assert viper.footprint(dataclasses.replace(d, volume_bending=True)) == viper.footprint(d)
    with pytest.raises(viper.ViperError) as ei:
        viper.footprint(dataclasses.replace(d, volume_bending=True, solver="jacobi"))
    assert ei.value.status == viper.ERR_INVALID and "volume_bending" in str(ei.value)


@pytest.mark.parametrize("cname,mirror", [("viper_scene_desc", "SceneDescC"), ("viper_contact_info", "ContactInfoC")])
def test_desc_layout_matches_header(tmp_path, cname, mirror):
    """The binding's mirrors of viper_scene_desc and viper_contact_info have the header's size
    and every field at the header's offset (a C program compiled here prints sizeof and
    offsetof)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    M = getattr(viper, mirror)
    fields = [f[0] for f in M._fields_]
    root = __file__.rsplit("/", 2)[0]
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "include/viper.h"', "int main(void) {",
           '  printf("%%zu\\n", sizeof(%s));' % cname]
    src += ['  printf("%%zu\\n", offsetof(%s, %s));' % (cname, f) for f in fields]
    src += ["  return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", root, str(c), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert got[0] == ctypes.sizeof(M)
    for name, off in zip(fields, got[1:]):
        assert getattr(M, name).offset == off, name
