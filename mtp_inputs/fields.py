"""Exact solutions and initial fields of Maxwell's equations and of linear acoustics
(problem data only).

Field layouts: Maxwell 3D u = (Ex, Ey, Ez, Hx, Hy, Hz), 2D TE u = (Ex, Ey, Hz);
acoustics u = (p, v_1 .. v_d).
Each exact solution is an object with
  u(x, t)        -> (..., nc) field values at points x (..., d) and time t
  dt(x, t, k)    -> k-th time derivative (plane waves only; used as boundary data)
"""
import numpy as np


class PlaneWaveTE:
    """2D TE plane wave  Hz = amp*sqrt(eps/mu) cos(psi), E = amp*(-dy, dx) cos(psi),
    psi = k (d.x) - omega t + phase, omega = k / sqrt(eps mu)."""

    def __init__(self, direction=(1.0, 1.0), k=2 * np.pi, amp=1.0, phase=0.0, eps=1.0, mu=1.0):
        dvec = np.asarray(direction, dtype=np.float64)
        self.d = dvec / np.linalg.norm(dvec)
        self.k, self.amp, self.phase = float(k), float(amp), float(phase)
        self.eps, self.mu = float(eps), float(mu)
        self.omega = self.k / np.sqrt(self.eps * self.mu)

    def dt(self, x, t, n=0):
        x = np.asarray(x, dtype=np.float64)
        psi = self.k * (x @ self.d) - self.omega * t + self.phase
        s = self.omega ** n * np.cos(psi - n * np.pi / 2)
        out = np.empty(x.shape[:-1] + (3,))
        out[..., 0] = -self.d[1] * self.amp * s
        out[..., 1] = self.d[0] * self.amp * s
        out[..., 2] = self.amp * np.sqrt(self.eps / self.mu) * s
        return out

    def u(self, x, t):
        return self.dt(x, t, 0)


class PlaneWave3D:
    """3D plane wave  E = aE cos(psi), H = sqrt(eps/mu) d x aE cos(psi), aE orthogonal to d."""

    def __init__(self, direction=(1.0, 0.0, 0.0), k=2 * np.pi, amp_e=(0.0, 1.0, 0.0), phase=0.0, eps=1.0, mu=1.0):
        dvec = np.asarray(direction, dtype=np.float64)
        self.d = dvec / np.linalg.norm(dvec)
        a = np.asarray(amp_e, dtype=np.float64)
        self.aE = a - (a @ self.d) * self.d
        self.k, self.phase, self.eps, self.mu = float(k), float(phase), float(eps), float(mu)
        self.omega = self.k / np.sqrt(self.eps * self.mu)
        self.aH = np.sqrt(self.eps / self.mu) * np.cross(self.d, self.aE)

    def dt(self, x, t, n=0):
        x = np.asarray(x, dtype=np.float64)
        psi = self.k * (x @ self.d) - self.omega * t + self.phase
        s = self.omega ** n * np.cos(psi - n * np.pi / 2)
        return np.concatenate([s[..., None] * self.aE, s[..., None] * self.aH], axis=-1)

    def u(self, x, t):
        return self.dt(x, t, 0)


class CavityTE_PMC:
    """TE dual of the paper's 2D TM cavity mode on [0, pi]^2 (eps = mu = 1), exact with
    magnetic walls:  Hz = sin x sin y cos(sqrt2 t),
    Ex = (1/sqrt2) sin x cos y sin(sqrt2 t),  Ey = -(1/sqrt2) cos x sin y sin(sqrt2 t)."""

    def u(self, x, t):
        x = np.asarray(x, dtype=np.float64)
        X, Y = x[..., 0], x[..., 1]
        w = np.sqrt(2.0)
        out = np.empty(x.shape[:-1] + (3,))
        out[..., 0] = np.sin(X) * np.cos(Y) * np.sin(w * t) / w
        out[..., 1] = -np.cos(X) * np.sin(Y) * np.sin(w * t) / w
        out[..., 2] = np.sin(X) * np.sin(Y) * np.cos(w * t)
        return out


class CavityTE_PEC:
    """TE cavity mode on the unit square with perfectly conducting walls (eps = mu = 1):
    Hz = cos(pi x) cos(pi y) cos(w t), w = sqrt2 pi,
    Ex = -(1/sqrt2) cos(pi x) sin(pi y) sin(w t), Ey = (1/sqrt2) sin(pi x) cos(pi y) sin(w t)."""

    def u(self, x, t):
        x = np.asarray(x, dtype=np.float64)
        X, Y = np.pi * x[..., 0], np.pi * x[..., 1]
        w = np.sqrt(2.0) * np.pi
        out = np.empty(x.shape[:-1] + (3,))
        out[..., 0] = -np.cos(X) * np.sin(Y) * np.sin(w * t) / np.sqrt(2.0)
        out[..., 1] = np.sin(X) * np.cos(Y) * np.sin(w * t) / np.sqrt(2.0)
        out[..., 2] = np.cos(X) * np.cos(Y) * np.cos(w * t)
        return out


class Cavity3D_PEC:
    """Unit-cube PEC cavity mode (eps = mu = 1):
    E = (0, 0, sin(pi x) sin(pi y) cos(w t)), w = sqrt2 pi,
    H = (sin(w t)/sqrt2) (-sin(pi x) cos(pi y), cos(pi x) sin(pi y), 0)."""

    def u(self, x, t):
        x = np.asarray(x, dtype=np.float64)
        X, Y = np.pi * x[..., 0], np.pi * x[..., 1]
        w = np.sqrt(2.0) * np.pi
        out = np.zeros(x.shape[:-1] + (6,))
        out[..., 2] = np.sin(X) * np.sin(Y) * np.cos(w * t)
        s = np.sin(w * t) / np.sqrt(2.0)
        out[..., 3] = -s * np.sin(X) * np.cos(Y)
        out[..., 4] = s * np.cos(X) * np.sin(Y)
        return out


class GaussianPulse3D:
    """Initial E = curl(a exp(-|x-x0|^2/(2 s^2))) (divergence free), H = 0;
    a ~ N(0, I) normalised, x0 ~ U[0.35, 0.65]^3, s ~ U[0.06, 0.10]."""

    def __init__(self, seed=11030):
        rng = np.random.default_rng(seed)
        a = rng.standard_normal(3)
        self.a = a / np.linalg.norm(a)
        self.x0 = rng.uniform(0.35, 0.65, size=3)
        self.s = rng.uniform(0.06, 0.10)

    def u(self, x, t=0.0):
        x = np.asarray(x, dtype=np.float64)
        r = x - self.x0
        gfac = np.exp(-np.sum(r * r, axis=-1) / (2 * self.s ** 2))
        grad = -(r / self.s ** 2) * gfac[..., None]   # grad of the Gaussian
        E = np.cross(grad, self.a)                      # curl(a g) = grad g x a
        out = np.zeros(x.shape[:-1] + (6,))
        out[..., :3] = E
        return out


def nodal_fields(exact, nodes, t=0.0):
    """Nodal values u(node, t) of an exact solution, shape (ne, Np, nc)."""
    return exact.u(nodes, t)


# ------------------------------------------------------------------ linear acoustics
# u = (p, v):  kappa p_t + div v = 0,  rho v_t + grad p = 0  (wave speed 1/sqrt(kappa rho),
# impedance sqrt(rho/kappa)).

class AcousticPlaneWave:
    """p = amp cos(psi), v = amp d / Z cos(psi), psi = k (d.x) - omega t + phase."""

    def __init__(self, direction=(1.0, 1.0), k=2 * np.pi, amp=1.0, phase=0.0, kappa=1.0, rho=1.0):
        dvec = np.asarray(direction, dtype=np.float64)
        self.d = dvec / np.linalg.norm(dvec)
        self.k, self.amp, self.phase = float(k), float(amp), float(phase)
        self.kappa, self.rho = float(kappa), float(rho)
        self.omega = self.k / np.sqrt(self.kappa * self.rho)
        self.z = np.sqrt(self.rho / self.kappa)
        self.avec = self.amp * np.concatenate([[1.0], self.d / self.z])

    def dt(self, x, t, n=0):
        x = np.asarray(x, dtype=np.float64)
        psi = self.k * (x @ self.d) - self.omega * t + self.phase
        s = self.omega ** n * np.cos(psi - n * np.pi / 2)
        return s[..., None] * self.avec

    def u(self, x, t):
        return self.dt(x, t, 0)


class AcousticCavity:
    """Rigid-wall (v.n = 0) mode of the unit square / cube, kappa = rho = 1:
    p = prod_i cos(pi x_i) cos(omega t),  v_i = (pi/omega) sin(pi x_i) prod_{j != i} cos(pi x_j)
    sin(omega t),  omega = pi sqrt(d)."""

    def __init__(self, dim):
        self.dim = dim
        self.omega = np.pi * np.sqrt(dim)

    def u(self, x, t):
        x = np.asarray(x, dtype=np.float64)
        c, s = np.cos(np.pi * x), np.sin(np.pi * x)
        out = np.empty(x.shape[:-1] + (self.dim + 1,))
        out[..., 0] = np.prod(c, axis=-1) * np.cos(self.omega * t)
        for i in range(self.dim):
            others = np.prod(np.delete(c, i, axis=-1), axis=-1)
            out[..., 1 + i] = np.pi / self.omega * s[..., i] * others * np.sin(self.omega * t)
        return out


class AcousticPulse:
    """Gaussian pressure pulse at rest: p = exp(-|x - x0|^2 / (2 s^2)), v = 0, with x0 in
    [0.35, 0.65]^d and s in [0.06, 0.10] drawn from the seed."""

    def __init__(self, dim, seed=11031):
        rng = np.random.default_rng(seed)
        self.dim = dim
        self.x0 = rng.uniform(0.35, 0.65, size=dim)
        self.s = rng.uniform(0.06, 0.10)

    def u(self, x, t=0.0):
        x = np.asarray(x, dtype=np.float64)
        r2 = np.sum((x - self.x0) ** 2, axis=-1)
        out = np.zeros(x.shape[:-1] + (self.dim + 1,))
        out[..., 0] = np.exp(-r2 / (2 * self.s ** 2))
        return out


class CircularCavityTE:
    """TE mode of the circular PEC cavity of radius R (eps = mu = 1):
    Hz = J_m(k r) cos(m theta) cos(k t) with J_m'(k R) = 0 (tangential E vanishes on the
    wall), E = (d_y Hz, -d_x Hz) sin(k t) / k; u = (Ex, Ey, Hz).  Default: m = 1 and the
    first root, k R = 1.8412."""

    def __init__(self, m=1, root=1, radius=1.0):
        from scipy.special import jnp_zeros
        self.m, self.R = m, radius
        self.k = float(jnp_zeros(m, root)[-1]) / radius

    def _hz_grad(self, x):
        from scipy.special import jv, jvp
        x = np.asarray(x, dtype=np.float64)
        r = np.hypot(x[..., 0], x[..., 1])
        th = np.arctan2(x[..., 1], x[..., 0])
        k, m = self.k, self.m
        rs = np.maximum(r, 1e-300)
        J, Jp = jv(m, k * r), k * jvp(m, k * r)
        c, s = np.cos(m * th), np.sin(m * th)
        hz = J * c
        dr, dth = Jp * c, -m * J * s / rs            # d/dr and (1/r) d/dtheta
        gx = dr * np.cos(th) - dth * np.sin(th)
        gy = dr * np.sin(th) + dth * np.cos(th)
        if m == 1:   # at the centre J_1(kr)/r -> k/2: grad Hz = (k/2, 0)
            z = r < 1e-12
            gx = np.where(z, k / 2.0, gx)
            gy = np.where(z, 0.0, gy)
        return hz, gx, gy

    def u(self, x, t):
        hz, gx, gy = self._hz_grad(x)
        k = self.k
        out = np.empty(np.shape(x)[:-1] + (3,))
        out[..., 0] = gy * np.sin(k * t) / k
        out[..., 1] = -gx * np.sin(k * t) / k
        out[..., 2] = hz * np.cos(k * t)
        return out
