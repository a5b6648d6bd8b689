"""The C-ABI library loads, exports what include/ugks.h declares, and rejects bad input.

These run without a GPU: only validation paths that fail before any HIP call
are exercised.
"""

import ctypes as C
import os
import re

import numpy as np
import pytest

import ugks_cases as uc
from paper_2606_15720_amd import ugks

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "ugks.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ugks_[a-z_]+)\s*\(", txt)))


def test_header_declares_what_the_binding_lists():
    assert _declared() == sorted(ugks.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = ugks.load_library()
    for name in _declared():
        assert hasattr(lib, name), name
    out = os.popen(f"nm -D --defined-only {ugks.LIB_PATH}").read()
    for name in _declared():
        assert re.search(rf"\bT {name}\b", out), name


def test_library_is_built_for_gfx950():
    blob = open(ugks.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


def _create(case, **kw):
    return ugks.ugks_create(case.mesh, case.vel, case.gas, case.bcs, case.W0, **kw)


def test_rejects_negative_internal_degrees_of_freedom():
    case = uc.cavity2d(n=4, nv=4)
    case.gas.K = -1
    with pytest.raises(ugks.UGKSError) as e:
        _create(case)
    assert e.value.code == ugks.UGKS_EINVAL and "gas.K" in str(e.value)


@pytest.mark.parametrize("what", ["volume", "normal", "weight", "bcid", "state", "precision", "open"])
def test_rejects_invalid_input(what):
    case = uc.cavity2d(n=4, nv=4)
    m = case.mesh
    kw = {}
    if what == "volume":
        m.cell_volume[3] = -1.0
    elif what == "normal":
        m.face_normal[5] *= 2.0
    elif what == "weight":
        case.vel.w[0] = 0.0
    elif what == "bcid":
        m.face_bc_id[m.face_bc == 1] = 9
    elif what == "state":
        case.W0[2, 3] = 0.0
    elif what == "precision":
        kw["precision"] = 16
    elif what == "open":
        m.face_area[7] *= 1.5
    with pytest.raises(ugks.UGKSError) as e:
        _create(case, **kw)
    assert e.value.code == ugks.UGKS_EINVAL
    assert ugks.ugks_last_error(None)


def test_rejects_empty_mesh_and_velocity_set():
    import dataclasses
    case = uc.cavity2d(n=4, nv=4)
    m = case.mesh
    empty = dataclasses.replace(
        m, cell_volume=m.cell_volume[:0], cell_centroid=m.cell_centroid[:0],
        face_cells=m.face_cells[:0], face_area=m.face_area[:0], face_normal=m.face_normal[:0],
        face_centroid=m.face_centroid[:0], face_shift=m.face_shift[:0], face_bc=m.face_bc[:0],
        face_bc_id=m.face_bc_id[:0])
    with pytest.raises(ugks.UGKSError) as e:
        ugks.ugks_create(empty, case.vel, case.gas, case.bcs, case.W0[:0])
    assert e.value.code == ugks.UGKS_EINVAL
    v = case.vel
    novel = dataclasses.replace(v, u=v.u[:0], w=v.w[:0])
    with pytest.raises(ugks.UGKSError) as e:
        ugks.ugks_create(m, novel, case.gas, case.bcs, case.W0)
    assert e.value.code == ugks.UGKS_EINVAL


def test_autotune_cache_file_round_trip(tmp_path):
    """The tuning cache is host-side: save / load / clear need no GPU."""
    lib = ugks.load_library()
    lib.ugks_autotune_clear()
    empty = tmp_path / "empty.txt"
    assert lib.ugks_autotune_save(str(empty).encode()) == 0
    assert empty.read_text() == "ugks-autotune 1\n"
    good = tmp_path / "good.txt"
    good.write_text("ugks-autotune 1\ncase 2 64 128 100 256 : 128 64 12.5\n"
                    "batch 2 64 0 100 256 : 128\n")
    assert lib.ugks_autotune_load(str(good).encode()) == 0
    out = tmp_path / "out.txt"
    assert lib.ugks_autotune_save(str(out).encode()) == 0
    text = out.read_text().splitlines()
    assert text[0] == "ugks-autotune 1"
    assert "case 2 64 128 100 256 : 128 64 12.5" in text
    assert "batch 2 64 0 100 256 : 128" in text
    for bad in ("not-a-cache\n", "ugks-autotune 1\ncase 2 64 128 100 256 : 0 64 1\n",
                "ugks-autotune 1\nbatch x : 96\n", "ugks-autotune 1\nother : 1\n"):
        p = tmp_path / "bad.txt"
        p.write_text(bad)
        assert lib.ugks_autotune_load(str(p).encode()) == -1
    lib.ugks_autotune_clear()


def test_batch_create_rejects_empty_batch():
    from paper_2606_15720_amd import ugks as U
    with pytest.raises(U.UGKSError) as e:
        U.ugks_batch_create([])
    assert e.value.code == U.UGKS_EINVAL
