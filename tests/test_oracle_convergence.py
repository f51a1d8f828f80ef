"""Pins of the oracle against closed-form Maxwell solutions: optimal h-convergence of
q = p+1 stage SAT with m = 2p (section "Numerical Results", 2D study), the order loss of
classical RK4 on Y = MU, and non-increasing front energy with the upwind flux."""
import numpy as np
import pytest

from mtp_inputs import fields, meshes
from oracle.mesh import Mesh
from oracle.pitch import pitch
from oracle.solve import OracleSolver


def run(case, n, p, method="sat", T=0.5, energy=False):
    if case == "planewave":     # 2D TE plane wave, exact-solution ghost on all sides
        mm, kind, ex = meshes.square_tri(n), meshes.DATA, fields.PlaneWaveTE()
    elif case == "pmc":         # TE dual of the paper's cavity on [0, pi]^2
        mm, kind, ex = meshes.square_tri(n, length=np.pi), meshes.PMC, fields.CavityTE_PMC()
    elif case == "pec2":
        mm, kind, ex = meshes.square_tri(n), meshes.PEC, fields.CavityTE_PEC()
    else:
        mm, kind, ex = meshes.cube_kuhn(n), meshes.PEC, fields.Cavity3D_PEC()
    d = mm["coords"].shape[1]
    mesh = Mesh(mm["coords"], mm["cells"], face_bc=meshes.uniform_bc(len(mm["cells"]), d, kind))
    tents = pitch(mesh, T, sigma=0.5)
    S = OracleSolver(mesh, p, p + 1, 2 * p, data=ex if kind == meshes.DATA else None, method=method)
    S.set_nodal_u(ex.u(meshes.equispaced_nodes(mm, p), 0.0))
    en = S.run(tents, energy_trace=energy)
    err, ref = S.l2_error(ex, T)
    return err, en


def rate(e0, e1):
    return np.log2(e0 / e1)


@pytest.mark.parametrize("case,p,ns", [("pmc", 1, (4, 8)), ("pmc", 3, (2, 4)), ("planewave", 2, (4, 8)),
                                       ("pmc", 4, (4, 8))])
def test_sat_optimal_order_2d(case, p, ns):
    e0, _ = run(case, ns[0], p)
    e1, _ = run(case, ns[1], p)
    assert rate(e0, e1) > p + 1 - 0.3, (e0, e1)


@pytest.mark.parametrize("p", [1, 2])
def test_sat_order_3d_cavity(p):
    """3D PEC cavity mode on 2^3 and 4^3 Kuhn cubes: rate > p + 1 - 0.3 (measured 1.80
    at p = 1, 3.21 at p = 2)."""
    e0, _ = run("pec3", 2, p, T=0.25)
    e1, _ = run("pec3", 4, p, T=0.25)
    assert rate(e0, e1) > p + 1 - 0.3, (e0, e1)


def test_rk4_loses_order():
    """Classical RK4 on dY/dth = A M^{-1} Y falls behind SAT once the error is small
    (the paper reports first-order stagnation; the magnitude is parity unpinned)."""
    s0, _ = run("pmc", 4, 4)
    s1, _ = run("pmc", 8, 4)
    r0, _ = run("pmc", 4, 4, method="rk4")
    r1, _ = run("pmc", 8, 4, method="rk4")
    assert rate(s0, s1) > 4.7
    assert rate(r0, r1) < rate(s0, s1) - 0.5
    assert r1 > 1.5 * s1


@pytest.mark.parametrize("p", [2, 3])
def test_energy_nonincreasing_pec(p):
    _, en = run("pec2", 4, p, T=0.3, energy=True)
    en = np.asarray(en)
    assert np.all(np.diff(en) <= 1e-12 * en[0])
    assert en[-1] < en[0]


def test_energy_nonincreasing_impedance_flux_two_materials():
    """The impedance-matched flux is dissipative across the material jump too."""
    mm = meshes.square_tri(4)
    eps, mu = meshes.materials_split(mm)
    mesh = Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu,
                face_bc=meshes.uniform_bc(len(mm["cells"]), 2, meshes.PEC))
    tents = pitch(mesh, 0.3, sigma=0.5)
    S = OracleSolver(mesh, 2, 3, 4, flux="impedance")
    S.set_nodal_u(fields.CavityTE_PEC().u(meshes.equispaced_nodes(mm, 2), 0.0))
    en = np.asarray(S.run(tents, energy_trace=True))
    assert np.all(np.diff(en) <= 1e-12 * en[0])
    assert en[-1] < en[0]
