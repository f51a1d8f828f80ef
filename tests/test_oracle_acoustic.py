"""Pins of the oracle's second system, linear acoustics (the method is stated for linear
hyperbolic systems in conservation form): the conservation form against exact acoustic
solutions, causality of the mass form, the fluxes against an independent eigenvector
Riemann solver, optimal h-convergence of SAT and non-increasing energy."""
import numpy as np
import pytest

from mtp_inputs import fields, meshes
from oracle.acoustic import AcousticSystem
from oracle.mesh import Mesh
from oracle.pitch import pitch
from oracle.solve import OracleSolver
from test_oracle_maxwell import _riemann_flux_by_eigenvectors


@pytest.mark.parametrize("dim,exact,mat", [
    (2, fields.AcousticCavity(2), (1.0, 1.0)),
    (3, fields.AcousticCavity(3), (1.0, 1.0)),
    (2, fields.AcousticPlaneWave(direction=(0.3, -1.0), k=5.0, phase=0.4, kappa=2.0, rho=0.7), (2.0, 0.7)),
    (3, fields.AcousticPlaneWave(direction=(1.0, 2.0, -0.5), k=3.0, kappa=0.5, rho=1.5), (0.5, 1.5)),
])
def test_conservation_form_reproduces_acoustics(dim, exact, mat):
    sysm = AcousticSystem(dim)
    rng = np.random.default_rng(3)
    h = 1e-5
    for _ in range(5):
        x, t = rng.uniform(0.1, 0.9, size=dim), rng.uniform(0.0, 1.0)
        dgt = np.diag(sysm.g_diag(*mat)) @ (exact.u(x, t + h) - exact.u(x, t - h)) / (2 * h)
        div = np.zeros(sysm.nc)
        for j in range(dim):
            dx = np.zeros(dim)
            dx[j] = h
            div += sysm.Aj[j] @ (exact.u(x + dx, t) - exact.u(x - dx, t)) / (2 * h)
        assert np.allclose(dgt + div, 0.0, atol=1e-7)


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_form_positive_exactly_inside_the_cone(dim):
    """K(b) = g - f b is symmetric positive definite iff kappa rho > |b|^2."""
    sysm = AcousticSystem(dim)
    rng = np.random.default_rng(5)
    for _ in range(20):
        kappa, rho = rng.uniform(0.5, 2.0, size=2)
        d = rng.normal(size=dim)
        d /= np.linalg.norm(d)
        for f, pos in ((0.95, True), (1.05, False)):
            K = sysm.K(f * np.sqrt(kappa * rho) * d, kappa, rho)
            assert np.allclose(K, K.T)
            assert (np.linalg.eigvalsh(K).min() > 0) == pos


@pytest.mark.parametrize("dim", [2, 3])
def test_acoustic_fluxes_are_the_riemann_flux(dim):
    sysm = AcousticSystem(dim)
    rng = np.random.default_rng(13)
    for _ in range(20):
        n = rng.normal(size=dim)
        n /= np.linalg.norm(n)
        ui, uo = rng.normal(size=sysm.nc), rng.normal(size=sysm.nc)
        mi, mo = rng.uniform(0.5, 3.0, size=2), rng.uniform(0.5, 3.0, size=2)
        zi, zo = np.sqrt(mi[1] / mi[0]), np.sqrt(mo[1] / mo[0])
        want = _riemann_flux_by_eigenvectors(sysm, ui, uo, n, mi, mo)
        assert np.allclose(sysm.flux_impedance(ui, uo, n, zi, zo), want, atol=1e-12)
        unit = _riemann_flux_by_eigenvectors(sysm, ui, uo, n, (1.0, 1.0), (1.0, 1.0))
        assert np.allclose(sysm.flux(ui, uo, n, 0.5), unit, atol=1e-12)
        assert np.allclose(sysm.flux_impedance(ui, uo, n, 1.0, 1.0), unit, atol=1e-12)


def _cavity_run(dim, n, p, T=0.3, energy=False, kind=meshes.PMC, flux="penalty"):
    mm = meshes.square_tri(n) if dim == 2 else meshes.cube_kuhn(n)
    mesh = Mesh(mm["coords"], mm["cells"], face_bc=meshes.uniform_bc(len(mm["cells"]), dim, kind))
    tents = pitch(mesh, T, sigma=0.5)
    ex = fields.AcousticCavity(dim)
    S = OracleSolver(mesh, p, p + 1, 2 * p, system="acoustic", flux=flux)
    S.set_nodal_u(ex.u(meshes.equispaced_nodes(mm, p), 0.0))
    en = S.run(tents, energy_trace=energy)
    return S, ex, en


@pytest.mark.parametrize("p,ns", [(1, (4, 8)), (2, (4, 8)), (3, (2, 4))])
def test_sat_optimal_order_acoustic_cavity_2d(p, ns):
    """Rigid-wall cavity (kind 1 walls), q = p + 1, m = 2p: rate p + 1."""
    errs = []
    for n in ns:
        S, ex, _ = _cavity_run(2, n, p)
        errs.append(S.l2_error(ex, 0.3)[0])
    assert np.log2(errs[0] / errs[1]) > p + 1 - 0.3, errs


def test_energy_nonincreasing_acoustic_pressure_release():
    _, _, en = _cavity_run(2, 4, 2, T=0.3, energy=True, kind=meshes.PEC)
    en = np.asarray(en)
    assert np.all(np.diff(en) <= 1e-12 * en[0])
    assert en[-1] < en[0]
