"""Host-side checks of the C-ABI library (no GPU needed): symbols, argument and mesh
errors, and the library's tent pitcher against the oracle's independent one (the tent
list is integer/index work plus quantised times: bit-exact)."""
import ctypes
import os
import re

import numpy as np
import pytest

from mtp_inputs import meshes
from oracle.mesh import Mesh as OMesh
from oracle.pitch import pitch as opitch, validate
from paper_1906_11029_amd import mtp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "mtp.h")).read()
    names = set(re.findall(r"^(?:mtp_status|void|const char\*)\s+(mtp_[a-z_]+)\s*\(", hdr, re.M))
    assert len(names) >= 20
    lib = ctypes.CDLL(mtp.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n


@pytest.mark.parametrize("dim,n,T", [(2, 4, 0.5), (2, 8, 0.5), (3, 2, 0.4), (3, 4, 0.3)])
def test_pitch_matches_oracle_bit_exact(dim, n, T):
    mm = meshes.cube_kuhn(n) if dim == 3 else meshes.square_tri(n)
    M = mtp.Mesh(mm["coords"], mm["cells"])
    tents = mtp.Tents(M, T, 0.5)
    ex = tents.export()
    om = OMesh(mm["coords"], mm["cells"])
    ot = opitch(om, T, 0.5)
    order = np.argsort(ot["layer"], kind="stable")
    for k in ("vertex", "t_bot", "t_top", "layer"):
        assert np.array_equal(ex[k], ot[k][order]), k
    assert tents.n_layers == ot["layer"].max() + 1
    assert np.array_equal(np.diff(tents.layer_ptr), np.bincount(ex["layer"]))
    # and the library's list passes the oracle's validator
    validate(om, {k: np.asarray(v) for k, v in ex.items()}, T, 0.5)


def test_pitch_graded_materials_matches_oracle():
    mm = meshes.cube_kuhn(3, axis_map=lambda g: 0.3 * g + 0.7 * g * g)
    eps, mu = meshes.materials_split(mm)
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu)
    ex = mtp.Tents(M, 0.2, 0.5).export()
    om = OMesh(mm["coords"], mm["cells"], eps=eps, mu=mu)
    ot = opitch(om, 0.2, 0.5)
    order = np.argsort(ot["layer"], kind="stable")
    for k in ("vertex", "t_bot", "t_top", "layer"):
        assert np.array_equal(ex[k], ot[k][order]), k


def _colour_meshes():
    graded = meshes.cube_kuhn(3, axis_map=lambda g: 0.3 * g + 0.7 * g * g)
    return {"square6": (meshes.square_tri(6), None), "disk8": (meshes.disk_tri(8), None),
            "fan32": (meshes.fan_disk(32), None), "kuhn3": (meshes.cube_kuhn(3), None),
            "graded3_eps": (graded, meshes.materials_split(graded))}


@pytest.mark.parametrize("name", ["square6", "disk8", "fan32", "kuhn3", "graded3_eps"])
def test_colour_pitch_matches_oracle_bit_exact(name):
    """The colour rule: the library's table equals the oracle's, entry for entry."""
    mm, mat = _colour_meshes()[name]
    eps, mu = mat if mat else (None, None)
    T = 0.2
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu)
    tents = mtp.Tents(M, T, 0.5, rule=mtp.MTP_PITCH_COLOUR)
    ex = tents.export()
    om = OMesh(mm["coords"], mm["cells"], eps=eps, mu=mu)
    ot = opitch(om, T, 0.5, rule="colour")
    order = np.argsort(ot["layer"], kind="stable")
    for k in ("vertex", "t_bot", "t_top", "layer"):
        assert np.array_equal(ex[k], ot[k][order]), k
    assert tents.n_layers == ot["layer"].max() + 1
    validate(om, {k: np.asarray(v) for k, v in ex.items()}, T, 0.5)
    # the explicit min-vertex rule is mtp_pitch_layers' table
    a = mtp.Tents(M, T, 0.5).export()
    b = mtp.Tents(M, T, 0.5, rule=mtp.MTP_PITCH_MIN_VERTEX).export()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_colour_pitch_refuses_unknown_rule():
    mm = meshes.square_tri(2)
    M = mtp.Mesh(mm["coords"], mm["cells"])
    for rule in (-1, 3):
        with pytest.raises(mtp.MTPError) as e:
            mtp.Tents(M, 0.5, 0.5, rule=rule)
        assert e.value.code == -1


def test_mesh_info_patch_sizes():
    mm = meshes.cube_kuhn(3)
    info = mtp.Mesh(mm["coords"], mm["cells"]).info
    assert info == {"dim": 3, "nv": 64, "ne": 162, "max_patch": 24}
    mm = meshes.square_tri(3)
    assert mtp.Mesh(mm["coords"], mm["cells"]).info["max_patch"] == 6


def test_mesh_errors():
    with pytest.raises(mtp.MTPError) as e:   # degenerate (collinear) triangle
        mtp.Mesh(np.array([[0, 0], [1, 0], [2, 0.0]]), np.array([[0, 1, 2]]))
    assert e.value.code == -2
    with pytest.raises(mtp.MTPError) as e:   # vertex id out of range
        mtp.Mesh(np.array([[0, 0], [1, 0], [0, 1.0]]), np.array([[0, 1, 3]]))
    assert e.value.code == -2
    with pytest.raises(mtp.MTPError) as e:   # face shared by three triangles
        X = np.array([[0, 0], [1, 0], [0, 1.0], [0, -1.0], [-1, 0.5]])
        mtp.Mesh(X, np.array([[0, 1, 2], [0, 3, 1], [0, 1, 4]]))
    assert e.value.code == -2
    with pytest.raises(mtp.MTPError) as e:   # non-positive material
        mtp.Mesh(np.array([[0, 0], [1, 0], [0, 1.0]]), np.array([[0, 1, 2]]), eps=np.array([0.0]))
    assert e.value.code == -2


def test_pitch_errors():
    mm = meshes.square_tri(2)
    M = mtp.Mesh(mm["coords"], mm["cells"])
    for s in (0.0, 1.0, 1.5):
        with pytest.raises(mtp.MTPError) as e:
            mtp.Tents(M, 0.5, s)
        assert e.value.code == -3
    with pytest.raises(mtp.MTPError) as e:
        mtp.Tents(M, -1.0, 0.5)
    assert e.value.code == -1


def test_workspace_size_and_unsupported_degree():
    mm = meshes.square_tri(2)
    M = mtp.Mesh(mm["coords"], mm["cells"])
    T = mtp.Tents(M, 0.5)
    assert mtp.mtp_solver_workspace_size(M.h, T.h, 2, 3, 4) > 0
    with pytest.raises(mtp.MTPError) as e:
        mtp.mtp_solver_workspace_size(M.h, T.h, 9, 3, 4)
    assert e.value.code == -9
    with pytest.raises(mtp.MTPError) as e:
        mtp.mtp_solver_workspace_size(M.h, T.h, 2, 3, 4, precision=7)
    assert e.value.code == -9


def test_acoustic_system_selection_errors():
    """Host-side checks of the second system: unknown system, and the vector-ALU kernel
    (Maxwell only) refused at the workspace query."""
    mm = meshes.cube_kuhn(2)
    M = mtp.Mesh(mm["coords"], mm["cells"], system=mtp.MTP_SYSTEM_ACOUSTIC)
    with pytest.raises(mtp.MTPError) as e:
        mtp.mtp_mesh_set_system(M.h, 7)
    assert e.value.code == -1
    T = mtp.Tents(M, 0.2, 0.5)
    with pytest.raises(mtp.MTPError) as e:
        mtp.mtp_solver_workspace_size(M.h, T.h, 2, 3, 4, mtp.MTP_FP64_VALU)
    assert e.value.code == -9
    # acoustics has d + 1 fields: a smaller workspace than Maxwell on the same mesh
    Mm = mtp.Mesh(mm["coords"], mm["cells"])
    Tm = mtp.Tents(Mm, 0.2, 0.5)
    assert mtp.mtp_solver_workspace_size(M.h, T.h, 2, 3, 4) < mtp.mtp_solver_workspace_size(Mm.h, Tm.h, 2, 3, 4)


def test_pitch_from_t_start():
    """A table pitched from the flat front t_start holds the same tents as one pitched from
    0, shifted by t_start (times are kept relative to t_start, so the slab pattern is the
    same bit for bit); t_end <= t_start is refused."""
    mm = meshes.square_tri(4)
    M = mtp.Mesh(mm["coords"], mm["cells"])
    a = mtp.Tents(M, 0.3, 0.5).export()
    b = mtp.Tents(M, 2.3, 0.5, t_start=2.0).export()
    assert np.array_equal(a["vertex"], b["vertex"]) and np.array_equal(a["layer"], b["layer"])
    assert np.array_equal(b["t_top"], 2.0 + a["t_top"]) and np.array_equal(b["t_bot"], 2.0 + a["t_bot"])
    with pytest.raises(mtp.MTPError) as e:
        mtp.Tents(M, 1.0, 0.5, t_start=1.0)
    assert e.value.code == -1


def test_binding_checks_array_sizes_before_calling_the_library():
    """The library reads ne*Np*nc field values and nc amplitudes / dim wave-vector entries:
    the binding refuses arrays of another shape before any call is made (handle None)."""
    with pytest.raises(ValueError, match="shape"):
        mtp.mtp_set_fields(None, np.zeros((4, 6, 3)), (4, 10, 3))
    with pytest.raises(ValueError, match="amplitudes"):
        mtp.mtp_set_planewave_bc(None, np.zeros(3), np.zeros(2), 1.0, 0.0, nc=6, dim=3)
    with pytest.raises(ValueError, match="amplitudes"):
        mtp.mtp_set_planewave_bc(None, np.zeros(3), np.zeros(3), 1.0, 0.0, nc=3, dim=2)


def test_split_bf16_precision_is_reserved():
    mm = meshes.cube_kuhn(2)
    M = mtp.Mesh(mm["coords"], mm["cells"])
    T = mtp.Tents(M, 0.2, 0.5)
    with pytest.raises(mtp.MTPError) as e:
        mtp.mtp_solver_workspace_size(M.h, T.h, 2, 3, 4, mtp.MTP_BF16X3)
    assert e.value.code == -9


def star_mesh(nfaces_min=50, seed=4):
    """One interior vertex at the origin whose patch is the cone over the convex hull of
    points on the unit sphere: 2 n - 4 tets around it."""
    from scipy.spatial import ConvexHull
    rng = np.random.default_rng(seed)
    n = (nfaces_min + 4 + 1) // 2
    x = rng.normal(size=(n, 3))
    x /= np.linalg.norm(x, axis=1)[:, None]
    hull = ConvexHull(x)
    coords = np.vstack([np.zeros((1, 3)), x])
    cells = np.hstack([np.zeros((len(hull.simplices), 1), np.int64), hull.simplices + 1]).astype(np.int32)
    return {"coords": coords, "cells": meshes._orient(coords, cells)}


def test_p4_patch_classes_accept_up_to_48_tets():
    """P4 in 3D: patches of up to 48 tets run on the matrix-core kernels (FP64 and mixed).  The
    36-tet class keeps its operator block in device memory, the 48-tet class the tent's F/R
    (1024 workgroup slots, which the workspace includes); larger patches, and the vector-ALU
    kernel beyond its LDS, are refused."""
    from cases import build_mesh
    mm = build_mesh(("delaunay", 3))
    M = mtp.Mesh(mm["coords"], mm["cells"])
    assert M.info["max_patch"] == 36
    T = mtp.Tents(M, 0.05, 0.5)
    w64 = mtp.mtp_solver_workspace_size(M.h, T.h, 4, 5, 8, mtp.MTP_FP64)
    wmx = mtp.mtp_solver_workspace_size(M.h, T.h, 4, 5, 8, mtp.MTP_MIXED_FP32)
    assert wmx > w64 > 0          # the mixed operator block adds its FP32 copy
    with pytest.raises(mtp.MTPError) as e:
        mtp.mtp_solver_workspace_size(M.h, T.h, 4, 5, 8, mtp.MTP_FP64_VALU)
    assert e.value.code == -9
    m48 = build_mesh(("delaunay48", 4))
    M48 = mtp.Mesh(m48["coords"], m48["cells"])
    assert M48.info["max_patch"] == 48
    T48 = mtp.Tents(M48, 0.04, 0.5)
    slot = 45 * (6 * 48 + 1) * 8   # F/R rows (3 x 15 face nodes) x (288 columns + 1) doubles
    for prec in (mtp.MTP_FP64, mtp.MTP_MIXED_FP32):
        assert mtp.mtp_solver_workspace_size(M48.h, T48.h, 4, 5, 8, prec) > 1024 * slot
    # a workspace without the slots: the same mesh at P3 (48-tet class in LDS)
    assert mtp.mtp_solver_workspace_size(M48.h, T48.h, 3, 4, 6, mtp.MTP_FP64) < 1024 * slot
    star = star_mesh()
    Ms = mtp.Mesh(star["coords"], star["cells"])
    assert Ms.info["max_patch"] > 48
    Ts = mtp.Tents(Ms, 0.02, 0.5)
    for prec in (mtp.MTP_FP64, mtp.MTP_MIXED_FP32):
        with pytest.raises(mtp.MTPError) as e:
            mtp.mtp_solver_workspace_size(Ms.h, Ts.h, 4, 5, 8, prec)
        assert e.value.code == -9
    # P3 keeps its 48-tet class
    big = meshes.graded_delaunay_cube(n=8, a=2.0 / 9.0, jitter=0.15, seed=11029)
    Mb = mtp.Mesh(big["coords"], big["cells"])
    assert 36 < Mb.info["max_patch"] <= 48
    Tb = mtp.Tents(Mb, 0.02, 0.5)
    assert mtp.mtp_solver_workspace_size(Mb.h, Tb.h, 3, 4, 6, mtp.MTP_MIXED_FP32) > 0


def test_auto_pitch_stops_the_losing_colour_table():
    """On a jittered Delaunay cube the colour table makes more work (761 against 484 tents
    at slab 0.05); the library stops its colour pitch once that work reaches the minimum-vertex
    table's, and still returns the oracle's choice, bit for bit."""
    from cases import build_mesh
    mm = build_mesh(("delaunay48", 4))
    om = OMesh(mm["coords"], mm["cells"])
    ot = opitch(om, 0.05, 0.5, rule="auto")
    assert ot["rule"] == "min_vertex"
    assert len(opitch(om, 0.05, 0.5, rule="colour")["vertex"]) > len(ot["vertex"])
    M = mtp.Mesh(mm["coords"], mm["cells"])
    tents = mtp.Tents(M, 0.05, 0.5, rule=mtp.MTP_PITCH_AUTO)
    assert tents.rule == mtp.MTP_PITCH_MIN_VERTEX
    ex = tents.export()
    order = np.argsort(ot["layer"], kind="stable")
    for k in ("vertex", "t_bot", "t_top", "layer"):
        assert np.array_equal(ex[k], ot[k][order]), k


@pytest.mark.parametrize("name", ["square6", "disk8", "kuhn3", "graded3_eps"])
def test_auto_pitch_matches_oracle_bit_exact(name):
    """MTP_PITCH_AUTO: the library picks the same ordering as the oracle and the same table,
    and reports the ordering it chose."""
    mm, mat = _colour_meshes()[name]
    eps, mu = mat if mat else (None, None)
    T = 0.2
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu)
    tents = mtp.Tents(M, T, 0.5, rule=mtp.MTP_PITCH_AUTO)
    ot = opitch(OMesh(mm["coords"], mm["cells"], eps=eps, mu=mu), T, 0.5, rule="auto")
    assert tents.rule == {"min_vertex": mtp.MTP_PITCH_MIN_VERTEX, "colour": mtp.MTP_PITCH_COLOUR}[ot["rule"]]
    ex = tents.export()
    order = np.argsort(ot["layer"], kind="stable")
    for k in ("vertex", "t_bot", "t_top", "layer"):
        assert np.array_equal(ex[k], ot[k][order]), k
    assert mtp.Tents(M, T, 0.5).rule == mtp.MTP_PITCH_MIN_VERTEX
