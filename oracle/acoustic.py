"""Linear acoustics in the same conservation form d_t g(u) + div f(u) = 0 (the method is
stated for linear hyperbolic systems of this form; this is the second system it is run
on), written out literally for the oracle.

u = (p, v);  g(u) = (kappa p, rho v);  f(u) = [v^T ; p I]  ((1 + d) x d),  so that
d_t g(u) + div f(u) = 0 reads  kappa p_t + div v = 0,  rho v_t + grad p = 0.
The per-element coefficients (kappa, rho) sit where Maxwell has (eps, mu): the wave speed
is 1/sqrt(kappa rho), the impedance Z = sqrt(rho/kappa).

Walls: kind 0 is pressure release (ghost p_out = -p_in), kind 1 is rigid (ghost
v_out = -v_in; only v.n enters the flux).  The interface has the same structure as the
Maxwell System class (matrices from unit vectors, generic solves elsewhere).
"""
import numpy as np


class AcousticSystem:
    def __init__(self, dim):
        self.dim = dim
        self.nc = dim + 1
        self.Aj = np.zeros((dim, self.nc, self.nc))
        for c in range(self.nc):
            e = np.zeros(self.nc)
            e[c] = 1.0
            F = self.f(e)
            for j in range(dim):
                self.Aj[j][:, c] = F[:, j]

    def f(self, u):
        """Flux matrix f(u), nc x dim: first row v^T, then p I."""
        p, v = u[0], u[1:]
        return np.vstack([v[None, :], p * np.eye(self.dim)])

    def g_diag(self, kappa, rho):
        return np.array([kappa] + [rho] * self.dim)

    def A(self, n):
        """f(u) n = A(n) u = (v.n, p n)."""
        return np.einsum("j,jab->ab", np.asarray(n, dtype=np.float64), self.Aj)

    def K(self, b, kappa, rho):
        """u -> g(u) - f(u) b."""
        return np.diag(self.g_diag(kappa, rho)) - self.A(b)

    def flux(self, u_in, u_out, n, alpha):
        """Upwind flux on a face with unit normal n (in -> out):
        1/2 A(n)(u_in + u_out) + alpha ([[p]], ([[v]].n) n),  [[u]] = u_in - u_out;
        alpha = 1/2 is the exact upwind flux for unit impedance."""
        n = np.asarray(n, dtype=np.float64)
        d = np.asarray(u_in) - np.asarray(u_out)
        pen = np.concatenate([[d[0]], (d[1:] @ n) * n])
        return 0.5 * self.A(n) @ (np.asarray(u_in) + np.asarray(u_out)) + alpha * pen

    def flux_impedance(self, u_in, u_out, n, z_in, z_out):
        """f(u*) n at the interface state of the Riemann problem along n between media of
        impedance z_in, z_out:
            p*   = (z_out p_in + z_in p_out + z_in z_out ([[v]].n)) / (z_in + z_out)
            v*.n = (z_in v_in.n + z_out v_out.n + [[p]]) / (z_in + z_out)."""
        n = np.asarray(n, dtype=np.float64)
        pi, po = u_in[0], u_out[0]
        vi, vo = np.asarray(u_in[1:]) @ n, np.asarray(u_out[1:]) @ n
        s = z_in + z_out
        ps = (z_out * pi + z_in * po + z_in * z_out * (vi - vo)) / s
        vs = (z_in * vi + z_out * vo + (pi - po)) / s
        return np.concatenate([[vs], ps * n])

    def flux_matrices(self, n, alpha, z=None):
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
        """kind 0: pressure release (p -> -p); kind 1: rigid wall (v -> -v)."""
        if kind == 0:
            return np.diag([-1.0] + [1.0] * self.dim)
        return np.diag([1.0] + [-1.0] * self.dim)
