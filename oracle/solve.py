"""Oracle driver: runs tents layer by layer on the whole mesh (section "Mesh
generation by tent pitching": tents of one layer are independent; the tent-top
function is the next tent's initial condition, no projection), converts to and from
the documented nodal interchange format, and measures L2 errors and energies.

Pins: tests/test_oracle_convergence.py (closed-form solutions, h-convergence orders,
energy decay) and tests/test_oracle_tent.py.
"""
import numpy as np

from .simplex import basis, quadrature, reference_nodes
from .tent import TentDG


class OracleSolver:
    def __init__(self, mesh, p, q, m, alpha=0.5, data=None, method="sat", flux="penalty", system="maxwell"):
        self.mesh, self.p, self.q, self.m = mesh, p, q, m
        self.dg = TentDG(mesh, p, alpha=alpha, data=data, flux=flux, system=system)
        self.nc, self.nb = self.dg.nc, self.dg.nb
        self.method = method
        self.tau = np.zeros(mesh.nv)
        self.cw = np.zeros((mesh.ne, self.nc * self.nb))   # modal coefficients of w
        self.V = basis(mesh.d, p).eval(reference_nodes(mesh.d, p))   # Vandermonde (Np x nb)
        self.Vinv = np.linalg.inv(self.V)

    # ------------------------------------------------------------ interchange format
    def set_nodal_w(self, w_nodal, t0=0.0):
        """w given as nodal values (ne, Np, nc) at the documented equispaced nodes."""
        self.tau[:] = t0
        c = np.einsum("ab,ebc->eca", self.Vinv, np.asarray(w_nodal, dtype=np.float64))
        self.cw = c.reshape(self.mesh.ne, -1)

    def set_nodal_u(self, u_nodal, t0=0.0):
        """Fields u on a flat front: w = g(u) = diag(eps, mu) u."""
        g = np.stack([self.dg.sys.g_diag(self.mesh.eps[e], self.mesh.mu[e]) for e in range(self.mesh.ne)])
        self.set_nodal_w(np.asarray(u_nodal) * g[:, None, :], t0)

    def nodal_w(self):
        c = self.cw.reshape(self.mesh.ne, self.nc, self.nb)
        return np.einsum("ab,ecb->eac", self.V, c)

    def nodal_u(self):
        """u = K(grad tau)^{-1} w, node by node (exact for affine elements)."""
        w = self.nodal_w()
        out = np.empty_like(w)
        m = self.mesh
        for e in range(m.ne):
            g = self.tau[m.cells[e]] @ m.grad_lam[e]
            K = self.dg.sys.K(g, m.eps[e], m.mu[e])
            out[e] = np.linalg.solve(K, w[e].T).T
        return out

    # ------------------------------------------------------------ evolution
    def run_tent(self, v, t_top):
        dg = self.dg
        T = dg.tent(self.tau, v, t_top)
        Y = [T["mass"][i] @ self.cw[e] for i, e in enumerate(T["es"])]
        if self.method == "sat":
            Y = dg.sat(T, Y, self.q, self.m)
        else:
            Y = dg.rk4(T, Y, self.m)
        for i, e in enumerate(T["es"]):
            self.cw[e] = np.linalg.solve(T["mass"][i], Y[i])
        self.tau[v] = t_top

    def run(self, tents, energy_trace=False, t_offset=0.0):
        """Run all tents in layer order (stable within a layer)."""
        order = np.argsort(tents["layer"], kind="stable")
        L = tents["layer"][order]
        energies = []
        for idx, i in enumerate(order):
            self.run_tent(int(tents["vertex"][i]), float(tents["t_top"][i]) + t_offset)
            if energy_trace and (idx + 1 == len(order) or L[idx + 1] != L[idx]):
                energies.append(self.energy())
        return energies

    # ------------------------------------------------------------ diagnostics
    def energy(self):
        """Front energy 1/2 int u.K(grad tau) u = 1/2 int w.K^{-1} w."""
        m, dg = self.mesh, self.dg
        tot = 0.0
        for e in range(m.ne):
            g = self.tau[m.cells[e]] @ m.grad_lam[e]
            Kinv = np.linalg.inv(dg.sys.K(g, m.eps[e], m.mu[e]))
            tot += 0.5 * self.cw[e] @ (np.kron(Kinv, dg.mass(e)) @ self.cw[e])
        return tot

    def l2_error(self, exact, t):
        """Spatial L2 error of all field components on the flat front at time t,
        quadrature of degree >= 2p+4."""
        m, dg = self.mesh, self.dg
        pts, w = quadrature(m.d, self.p + 3)
        Phi = dg.B.eval(pts)
        err2, ref2 = 0.0, 0.0
        for e in range(m.ne):
            g = self.tau[m.cells[e]] @ m.grad_lam[e]
            K = dg.sys.K(g, m.eps[e], m.mu[e])
            wq = Phi @ self.cw[e].reshape(self.nc, self.nb).T     # (nq, nc)
            uq = np.linalg.solve(K, wq.T).T
            ue = exact.u(m.to_phys(e, pts), t)
            ww = w * abs(m.detJ[e])
            err2 += np.sum(ww[:, None] * (uq - ue) ** 2)
            ref2 += np.sum(ww[:, None] * ue ** 2)
        return np.sqrt(err2), np.sqrt(ref2)
