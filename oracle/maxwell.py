"""Maxwell's equations in the conservation form the paper uses (section "The MTP
discretization"), written out literally, for the oracle.

u = (E, H);  g(u) = (eps E, mu H);  f(u) = [-skew H ; skew E]  (6 x 3), with
skew E = [[0, Ez, -Ey], [-Ez, 0, Ex], [Ey, -Ex, 0]]  so that div skew E = curl E
(divergence taken row-wise).  Then  d_t g(u) + div_x f(u) = 0  is Maxwell's system.

2D TE is the restriction to fields independent of z with E = (Ex, Ey, 0),
H = (0, 0, Hz):  u = (Ex, Ey, Hz), rows (Ex, Ey, Hz) and columns (x, y) of f.

All matrices below are obtained by applying these definitions to unit vectors, so a
reader can check them against the paper's formulas by eye.
"""
import numpy as np


def cross(a, b):
    """a x b for 3-vectors."""
    return np.array([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


def skew(E):
    return np.array([[0.0, E[2], -E[1]],
                     [-E[2], 0.0, E[0]],
                     [E[1], -E[0], 0.0]])


def f3(u6):
    """f(u) in 3D, the 6 x 3 flux matrix of the paper's conservation law."""
    E, H = u6[:3], u6[3:]
    return np.vstack([-skew(H), skew(E)])


_TE_ROWS = [0, 1, 5]  # (Ex, Ey, Hz) inside (Ex, Ey, Ez, Hx, Hy, Hz)


def _embed_te(u3):
    u6 = np.zeros(6)
    u6[0], u6[1], u6[5] = u3
    return u6


class System:
    """One of the two field systems: dim = 3 (E, H) or dim = 2 (TE: Ex, Ey, Hz)."""

    def __init__(self, dim):
        self.dim = dim
        self.nc = 6 if dim == 3 else 3
        # A_j[:, c] = column j of f(e_c):  f(u)[:, j] = A_j u
        self.Aj = np.zeros((dim, self.nc, self.nc))
        for c in range(self.nc):
            e = np.zeros(self.nc)
            e[c] = 1.0
            F = self.f(e)
            for j in range(dim):
                self.Aj[j][:, c] = F[:, j]

    def f(self, u):
        """Flux matrix f(u), nc x dim."""
        if self.dim == 3:
            return f3(u)
        return f3(_embed_te(u))[_TE_ROWS][:, :2]

    def g_diag(self, eps, mu):
        """g(u) = diag(eps.., mu..) u."""
        if self.dim == 3:
            return np.array([eps, eps, eps, mu, mu, mu])
        return np.array([eps, eps, mu])

    def A(self, n):
        """f(u) n = A(n) u."""
        return np.einsum("j,jab->ab", np.asarray(n, dtype=np.float64), self.Aj)

    def K(self, b, eps, mu):
        """Matrix of u -> g(u) - f(u) b  (the mass-form integrand, paper eq. for a(u,v))."""
        return np.diag(self.g_diag(eps, mu)) - self.A(b)

    def split_EH(self, u):
        """(E, H) as 3-vectors for the tangential-part formulas."""
        if self.dim == 3:
            return u[:3], u[3:]
        return np.array([u[0], u[1], 0.0]), np.array([0.0, 0.0, u[2]])

    def join_EH(self, E, H):
        if self.dim == 3:
            return np.concatenate([E, H])
        return np.array([E[0], E[1], H[2]])

    def flux(self, u_in, u_out, n, alpha):
        """Upwind numerical flux on a face with unit normal n pointing from the "in"
        element to the "out" side (section "The MTP discretization"):

            f_n = [ {H} x n + alpha [[E_t]] ;  -{E} x n + alpha [[H_t]] ] ,
            {u} = (u_in + u_out)/2,  E_t = -(E x n) x n,  [[u]] = u_in - u_out.

        Readings: the jump is taken inside-minus-outside with respect to n (with the
        printed outside-minus-inside the printed weak-form sign and the central flux
        disagree, and the scheme would not be energy stable); alpha = 1/2 is the exact
        (Godunov) upwind flux for unit impedance, alpha = 1 is the printed
        coefficient.  Both are dissipative."""
        n3 = np.zeros(3)
        n3[: len(n)] = n
        Ei, Hi = self.split_EH(u_in)
        Eo, Ho = self.split_EH(u_out)
        Em, Hm = 0.5 * (Ei + Eo), 0.5 * (Hi + Ho)
        tang = lambda v: -cross(cross(v, n3), n3)  # noqa: E731
        fE = cross(Hm, n3) + alpha * tang(Ei - Eo)
        fH = -cross(Em, n3) + alpha * tang(Hi - Ho)
        return self.join_EH(fE, fH)

    def flux_impedance(self, u_in, u_out, n, z_in, z_out):
        """Impedance-matched upwind flux across a material interface: the physical flux
        f(u*) n at the interface state u* of the one-dimensional Riemann problem along n
        (tangential E and H continuous; the wave entering each side determined by that
        side's state alone).  With impedances Z = sqrt(mu/eps) of the two sides:

            E*_t = (Z_out E_in + Z_in E_out - Z_in Z_out n x [[H]]) / (Z_in + Z_out)
            H*_t = (Z_in H_in + Z_out H_out + n x [[E]]) / (Z_in + Z_out),

        [[u]] = u_in - u_out.  For Z_in = Z_out = 1 it is the alpha = 1/2 flux above."""
        n3 = np.zeros(3)
        n3[: len(n)] = n
        Ei, Hi = self.split_EH(u_in)
        Eo, Ho = self.split_EH(u_out)
        s = z_in + z_out
        Es = (z_out * Ei + z_in * Eo - z_in * z_out * cross(n3, Hi - Ho)) / s
        Hs = (z_in * Hi + z_out * Ho + cross(n3, Ei - Eo)) / s
        return self.join_EH(cross(Hs, n3), -cross(Es, n3))

    def flux_matrices(self, n, alpha, z=None):
        """(B_in, B_out) with flux(u_in, u_out) = B_in u_in + B_out u_out; z = (Z_in, Z_out)
        selects the impedance-matched flux."""
        Bi = np.zeros((self.nc, self.nc))
        Bo = np.zeros((self.nc, self.nc))
        zero = np.zeros(self.nc)
        f = (lambda a, b: self.flux(a, b, n, alpha)) if z is None else \
            (lambda a, b: self.flux_impedance(a, b, n, z[0], z[1]))
        for c in range(self.nc):
            e = np.zeros(self.nc)
            e[c] = 1.0
            Bi[:, c] = f(e, zero)
            Bo[:, c] = f(zero, e)
        return Bi, Bo

    def ghost_matrix(self, kind):
        """Mirror ghost state u_out = R u_in on a wall:
        PEC (kind 0): E_out = -E_in, H_out = H_in;  PMC (kind 1): E_out = E_in, H_out = -H_in."""
        if self.dim == 3:
            sE, sH = (-1.0, 1.0) if kind == 0 else (1.0, -1.0)
            return np.diag([sE] * 3 + [sH] * 3)
        sE, sH = (-1.0, 1.0) if kind == 0 else (1.0, -1.0)
        return np.diag([sE, sE, sH])
