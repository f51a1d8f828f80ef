"""Host-side checks of the curved-element interface (no GPU needed): the library's pitcher on
meshes with quadratic boundary triangles against the oracle's curved pitcher (bit-exact tent
lists), and the refusals of mtp_mesh_set_curved_p2."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from cases import CURVED_CASES, setup  # noqa: E402
from mtp_inputs import meshes  # noqa: E402
from oracle import curved  # noqa: E402
from oracle.pitch import pitch as opitch  # noqa: E402
from paper_1906_11029_amd import mtp  # noqa: E402


@pytest.mark.parametrize("name", list(CURVED_CASES))
def test_curved_pitch_matches_the_oracle_bit_exact(name):
    c, mm, dim, eps, mu, bc, ex, u0 = setup(name)
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc, curved=mm["geo"])
    ex_t = mtp.Tents(M, c["T"], 0.5).export()
    cm = curved.CurvedMesh(mm["coords"], mm["cells"], mm["geo"], eps=eps, mu=mu, face_bc=bc)
    ot = opitch(cm.base, c["T"], 0.5, k_elem=cm.step_bounds(0.5))
    order = np.argsort(ot["layer"], kind="stable")
    for k in ("vertex", "t_bot", "t_top", "layer"):
        assert np.array_equal(ex_t[k], ot[k][order]), k


def test_curved_colour_pitch_matches_the_oracle_bit_exact():
    from cases import setup as csetup
    c, mm, dim, eps, mu, bc, ex, u0 = csetup("disk_curved_p3_colour")
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc, curved=mm["geo"])
    ex_t = mtp.Tents(M, c["T"], 0.5, rule=mtp.MTP_PITCH_COLOUR).export()
    cm = curved.CurvedMesh(mm["coords"], mm["cells"], mm["geo"], eps=eps, mu=mu, face_bc=bc)
    ot = opitch(cm.base, c["T"], 0.5, k_elem=cm.step_bounds(0.5), rule="colour")
    order = np.argsort(ot["layer"], kind="stable")
    for k in ("vertex", "t_bot", "t_top", "layer"):
        assert np.array_equal(ex_t[k], ot[k][order]), k


def _mesh():
    mm = meshes.disk_tri(2)
    return mm, meshes.p2_geometry(mm, on_circle=1.0)


def test_set_curved_refusals():
    mm, geo = _mesh()
    M = mtp.Mesh(mm["coords"], mm["cells"])
    bad = geo.copy()
    bad[0, 0, 0] += 1e-3      # a vertex node that is not the mesh's vertex
    with pytest.raises(mtp.MTPError) as e:
        mtp.mtp_mesh_set_curved_p2(M.h, bad, M.info["ne"])
    assert e.value.code == mtp.MTP_OK - 1
    # an interior edge whose two elements disagree on its midpoint
    bad = geo.copy()
    e0 = 0
    # move the midpoint of an interior edge of element 0 in element 0 only
    mid_for_face = {2: 3, 0: 4, 1: 5}
    from oracle.mesh import Mesh as OMesh
    om = OMesh(mm["coords"], mm["cells"])
    f = next(f for f in range(3) if om.nbr[e0, f] >= 0)
    bad[e0, mid_for_face[f]] += np.array([1e-3, 0.0])
    with pytest.raises(mtp.MTPError) as e:
        mtp.mtp_mesh_set_curved_p2(M.h, bad, M.info["ne"])
    assert e.value.code == -2
    # a boundary element folded over (midpoint pushed past the opposite vertex)
    bnd = next(i for i in range(len(geo)) if np.any(om.nbr[i] < 0))
    fb = next(f for f in range(3) if om.nbr[bnd, f] < 0)
    bad = geo.copy()
    opp = mm["coords"][mm["cells"][bnd, fb]]
    bad[bnd, mid_for_face[fb]] = opp + 2.0 * (opp - bad[bnd, mid_for_face[fb]])
    with pytest.raises(mtp.MTPError) as e:
        mtp.mtp_mesh_set_curved_p2(M.h, bad, M.info["ne"])
    assert e.value.code == -2
    # 3D meshes have no curved elements here
    k = meshes.cube_kuhn(1)
    M3 = mtp.Mesh(k["coords"], k["cells"])
    with pytest.raises(mtp.MTPError) as e:
        mtp.mtp_mesh_set_curved_p2(M3.h, np.zeros((M3.info["ne"], 6, 2)), M3.info["ne"])
    assert e.value.code == -1
    with pytest.raises(ValueError):
        mtp.mtp_mesh_set_curved_p2(M.h, geo[:-1], M.info["ne"])
    # a valid call after the refusals
    mtp.mtp_mesh_set_curved_p2(M.h, geo, M.info["ne"])
