"""Pins of the oracle's Maxwell system against the paper's closed forms and against
exact solutions of Maxwell's equations."""
import numpy as np
import pytest

from mtp_inputs import fields
from oracle.maxwell import System


def _dt_g_plus_div_f(sysm, exact, x, t, h=1e-5):
    """d_t g(u) + sum_j A_j d_j u by central differences (eps = mu = 1)."""
    dut = (exact.u(x, t + h) - exact.u(x, t - h)) / (2 * h)
    div = np.zeros_like(dut)
    for j in range(sysm.dim):
        dx = np.zeros(sysm.dim)
        dx[j] = h
        duj = (exact.u(x + dx, t) - exact.u(x - dx, t)) / (2 * h)
        div += duj @ sysm.Aj[j].T
    return dut + div


@pytest.mark.parametrize("dim,exact", [
    (3, fields.Cavity3D_PEC()),
    (3, fields.PlaneWave3D(direction=(1.0, 2.0, -0.5), amp_e=(0.3, -0.2, 1.0), k=3.0)),
    (2, fields.CavityTE_PEC()),
    (2, fields.CavityTE_PMC()),
    (2, fields.PlaneWaveTE(direction=(0.3, -1.0), k=5.0, phase=0.4)),
])
def test_conservation_form_reproduces_maxwell(dim, exact):
    # exact Maxwell solutions satisfy d_t g(u) + div f(u) = 0 with the oracle's f
    sysm = System(dim)
    x = np.random.default_rng(3).uniform(0.1, 0.9, size=(10, dim))
    r = _dt_g_plus_div_f(sysm, exact, x, 0.37)
    assert np.max(np.abs(r)) < 1e-7


def _closed_form_inverse(b, eps, mu, w):
    """The paper's pointwise inverse of u -> g(u) - f(u) grad phi (section on SAT)."""
    wE, wH = w[:3], w[3:]
    P = np.eye(3) - np.outer(b, b) / (eps * mu)
    s = 1.0 / (eps * mu - b @ b)
    E = s * P @ (mu * wE + np.cross(wH, b))
    H = s * P @ (eps * wH - np.cross(wE, b))
    return np.concatenate([E, H])


def test_mass_form_matches_paper_closed_form_inverse():
    sysm = System(3)
    rng = np.random.default_rng(4)
    for _ in range(20):
        eps, mu = rng.uniform(0.5, 3.0, 2)
        b = rng.standard_normal(3)
        b *= rng.uniform(0, 0.95) * np.sqrt(eps * mu) / np.linalg.norm(b)
        w = rng.standard_normal(6)
        u = np.linalg.solve(sysm.K(b, eps, mu), w)
        assert np.allclose(u, _closed_form_inverse(b, eps, mu, w), rtol=1e-12, atol=1e-12)


def test_mass_form_te_is_restriction_of_3d():
    s2, s3 = System(2), System(3)
    rng = np.random.default_rng(5)
    b = np.array([0.2, -0.3])
    K2 = s2.K(b, 1.3, 0.7)
    K3 = s3.K(np.array([0.2, -0.3, 0.0]), 1.3, 0.7)
    rows = [0, 1, 5]
    assert np.allclose(K2, K3[np.ix_(rows, rows)])
    # and the closed form of the paper restricted to TE fields
    w = rng.standard_normal(3)
    w6 = np.zeros(6)
    w6[rows] = w
    u6 = _closed_form_inverse(np.array([0.2, -0.3, 0.0]), 1.3, 0.7, w6)
    assert np.allclose(np.linalg.solve(K2, w), u6[rows], rtol=1e-12)


def test_coercivity_bound():
    # a(u,u) >= (1 - |b|/sqrt(eps mu)) (eps|E|^2 + mu|H|^2)   (section on SAT)
    sysm = System(3)
    rng = np.random.default_rng(6)
    for _ in range(50):
        eps, mu = rng.uniform(0.5, 3.0, 2)
        b = rng.standard_normal(3)
        frac = rng.uniform(0, 0.99)
        b *= frac * np.sqrt(eps * mu) / np.linalg.norm(b)
        K = sysm.K(b, eps, mu)
        assert np.allclose(K, K.T)
        G = np.diag(sysm.g_diag(eps, mu))
        lam = np.linalg.eigvalsh(np.linalg.solve(np.sqrt(G), np.linalg.solve(np.sqrt(G), K).T))
        assert lam.min() >= (1 - frac) - 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_flux_consistency_and_godunov(dim):
    sysm = System(dim)
    rng = np.random.default_rng(7)
    for _ in range(10):
        n = rng.standard_normal(dim)
        n /= np.linalg.norm(n)
        u = rng.standard_normal(sysm.nc)
        # consistency: f_n(u, u) = f(u) n
        assert np.allclose(sysm.flux(u, u, n, 0.5), sysm.f(u) @ n)
        # alpha = 1/2 is the Godunov flux A+ u_in + A- u_out (eigen-split of A(n))
        lam, Q = np.linalg.eigh(sysm.A(n))
        Ap = Q @ np.diag(np.maximum(lam, 0)) @ Q.T
        Am = Q @ np.diag(np.minimum(lam, 0)) @ Q.T
        uo = rng.standard_normal(sysm.nc)
        assert np.allclose(sysm.flux(u, uo, n, 0.5), Ap @ u + Am @ uo)
        # flux seen from the other side is the negative (conservation)
        assert np.allclose(sysm.flux(u, uo, n, 0.7), -sysm.flux(uo, u, -n, 0.7))


def test_wall_ghosts():
    sysm = System(3)
    rng = np.random.default_rng(8)
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    u = rng.standard_normal(6)
    for kind in (0, 1):
        uo = sysm.ghost_matrix(kind) @ u
        E_mean = 0.5 * (u[:3] + uo[:3])
        H_mean = 0.5 * (u[3:] + uo[3:])
        if kind == 0:   # PEC: mean tangential E vanishes
            assert np.allclose(np.cross(E_mean, n), 0)
        else:           # PMC: mean tangential H vanishes
            assert np.allclose(np.cross(H_mean, n), 0)


@pytest.mark.parametrize("dim", [2, 3])
def test_impedance_flux_is_godunov_for_unit_impedance(dim):
    """With Z = 1 on both sides the impedance-matched flux is the alpha = 1/2 flux."""
    sysm = System(dim)
    rng = np.random.default_rng(7)
    for _ in range(20):
        n = rng.normal(size=dim)
        n /= np.linalg.norm(n)
        ui, uo = rng.normal(size=sysm.nc), rng.normal(size=sysm.nc)
        assert np.allclose(sysm.flux_impedance(ui, uo, n, 1.0, 1.0), sysm.flux(ui, uo, n, 0.5), atol=1e-13)


def _riemann_flux_by_eigenvectors(sysm, ui, uo, n, mat_in, mat_out):
    """Interface flux of the one-dimensional Riemann problem M du/dt + A(n) du/dxi = 0
    (xi along n) from the characteristic decomposition of each side: the waves of
    negative speed enter the "in" medium, those of positive speed the "out" medium,
    u*_in = u_in + sum a_k r_k, u*_out = u_out + sum b_k r_k, and the normal flux is
    continuous, A u*_in = A u*_out."""
    import scipy.linalg
    A = sysm.A(n)

    def eig(eps, mu):
        lam, R = scipy.linalg.eig(A, np.diag(sysm.g_diag(eps, mu)))
        return lam.real, R.real
    li, Ri = eig(*mat_in)
    lo, Ro = eig(*mat_out)
    Rn, Rp = Ri[:, li < -1e-12], Ro[:, lo > 1e-12]
    coef, *_ = np.linalg.lstsq(np.hstack([A @ Rn, -(A @ Rp)]), A @ (uo - ui), rcond=None)
    ustar = ui + Rn @ coef[:Rn.shape[1]]
    return A @ ustar


@pytest.mark.parametrize("dim", [2, 3])
def test_impedance_flux_is_the_exact_riemann_flux(dim):
    """Against an independent construction from the generalised eigenvectors of
    (A(n), diag(g)) on each side, for random materials, normals and states."""
    sysm = System(dim)
    rng = np.random.default_rng(11)
    for _ in range(20):
        n = rng.normal(size=dim)
        n /= np.linalg.norm(n)
        ui, uo = rng.normal(size=sysm.nc), rng.normal(size=sysm.nc)
        mi, mo = rng.uniform(0.5, 3.0, size=2), rng.uniform(0.5, 3.0, size=2)
        zi, zo = np.sqrt(mi[1] / mi[0]), np.sqrt(mo[1] / mo[0])
        want = _riemann_flux_by_eigenvectors(sysm, ui, uo, n, mi, mo)
        assert np.allclose(sysm.flux_impedance(ui, uo, n, zi, zo), want, atol=1e-12)
        # both sides see the same interface state: swapping sides flips the flux
        assert np.allclose(sysm.flux_impedance(uo, ui, -n, zo, zi), -want, atol=1e-12)
