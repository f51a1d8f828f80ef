"""Per-tent DG semi-discretisation and SAT / RK4 time stepping for the oracle.

Follows the paper's sections "The MTP discretization" and "Structure-aware Taylor
time-stepping" in their order:

  tent map     phi(x, th) = (1 - th) phi_b(x) + th phi_t(x),  delta = phi_t - phi_b
  transformed  d_th (g(u) - f(u) grad phi) + div_x(delta f(u)) = 0
  DG on the patch (one element's rows; n = outward normal, "out" = neighbour/ghost):
     d/dth int_T [g(u) - f(u) grad phi].v
        = int_T delta f(u) : grad v  -  int_{F in dT, F contains V} delta f_n(u_in, u_out).v
     (faces of the patch boundary carry delta = 0 and drop out)
  semi-discrete ODE  d/dth (M U) = A U (+ boundary data b(th)),  M affine in th
  SAT(q, m)   Y_{i,n} = A U_{i,n-1} + b^{(n-1)}(th_i),            1 <= n <= q
              M_i U_{i,n} = Y_{i,n} - n M' U_{i,n-1},               1 <= n <= q-1
              M_i U_{i,0} = Y_{i,0} = Y_{i-1}(th_i),  Y_i(th_{i+1}) = sum_n Y_{i,n}/(m^n n!)
  RK4 variant dY/dth = A M(th)^{-1} Y + b(th) with classical RK4 on the same m steps.

Boundary data (faces on the domain boundary that contain V): mirror ghosts for PEC /
PMC walls, and for DATA faces the exact solution as ghost,
u_out(x, th) = u_ex(x, phi(x, th)), whose th-derivatives are
delta(x)^k (d_t^k u_ex)(x, phi(x, th)); the ghost enters the face integral through its
degree-p interpolant at the face's equispaced nodes (a reading: the paper does not say
how data enter a tent).

State: per element the modal coefficients of w = g(u) - f(u) grad tau (the mass form
integrand, continuous from one tent to the next); Y = (I x Mass_T) w.

Pins: tests/test_oracle_tent.py -- energy identity with random U; SAT temporal order
m^-q against a DOP853 reference of the tent ODE; flat-front slab reduces to the
Taylor polynomial of exp; brute-force tiny meshes against independent sympy integrals;
closed-form solutions and convergence orders in tests/test_oracle_convergence.py.
"""
from math import factorial

import numpy as np

from .acoustic import AcousticSystem
from .maxwell import System
from .simplex import basis, quadrature, reference_nodes

PEC, PMC, DATA = 0, 1, 2


class TentDG:
    def __init__(self, mesh, p, alpha=0.5, data=None, flux="penalty", system="maxwell"):
        self.mesh, self.p, self.alpha = mesh, p, alpha
        self.flux_kind = flux   # "penalty" (alpha-weighted, as printed) or "impedance"
        self.d = mesh.d
        self.sys = System(mesh.d) if system == "maxwell" else AcousticSystem(mesh.d)
        self.nc = self.sys.nc
        self.B = basis(self.d, p)
        self.nb = self.B.n
        self.qv_pts, self.qv_w = quadrature(self.d, p + 2)
        self.Phi_v = self.B.eval(self.qv_pts)
        self.Grad_v = self.B.grad(self.qv_pts)
        self.qf_pts, self.qf_w = quadrature(self.d - 1, p + 2)
        fb = basis(self.d - 1, p)
        fn = reference_nodes(self.d - 1, p)
        # face Lagrange interpolation at the equispaced face nodes: I[q, s] = l_s(point q)
        self.face_interp = fb.eval(self.qf_pts) @ np.linalg.inv(fb.eval(fn))
        self.face_nodes_ref = fn
        self.data = data
        self._mass, self._vol, self._face = {}, {}, {}

    # ---------------------------------------------------------------- element integrals
    def mass(self, e):
        """Mass_T[b, a] = int_T phi_b phi_a."""
        if e not in self._mass:
            w = self.qv_w * abs(self.mesh.detJ[e])
            self._mass[e] = self.Phi_v.T @ (w[:, None] * self.Phi_v)
        return self._mass[e]

    def vol(self, e, k):
        """D[j][b, a] = int_T lambda_k d_j phi_b phi_a  (physical derivative j)."""
        key = (e, k)
        if key not in self._vol:
            m = self.mesh
            xq = m.to_phys(e, self.qv_pts)
            lam = m.barycentric(e, xq)[:, k]
            w = self.qv_w * abs(m.detJ[e]) * lam
            gphys = np.einsum("qal,lj->qaj", self.Grad_v, m.Jinv[e])
            self._vol[key] = np.einsum("q,qbj,qa->jba", w, gphys, self.Phi_v)
        return self._vol[key]

    def face(self, e, f, k):
        """Integrals over local face f of element e (opposite local vertex f), weighted by
        lambda_k (k = local index of the tent vertex).  Returns dict with the outward
        unit normal n, Fself[b,a] = int_F lambda_k phi^e_b phi^e_a, Fcross with the
        neighbour's basis (if any), and for boundary data the quadrature data."""
        key = (e, f, k)
        if key in self._face:
            return self._face[key]
        m = self.mesh
        Y = m.X[e][[i for i in range(self.d + 1) if i != f]]
        Bf = (Y[1:] - Y[0]).T                      # d x (d-1)
        meas = np.sqrt(np.linalg.det(Bf.T @ Bf))
        xq = Y[0] + self.qf_pts @ Bf.T
        w = self.qf_w * meas
        lam_e = m.barycentric(e, xq)
        lam = lam_e[:, k]
        # outward normal: orthogonal to the face, pointing away from the opposite vertex
        if self.d == 2:
            t = Y[1] - Y[0]
            n = np.array([t[1], -t[0]])
        else:
            n = np.cross(Y[1] - Y[0], Y[2] - Y[0])
        n = n / np.linalg.norm(n)
        if (m.X[e, f] - Y[0]) @ n > 0:
            n = -n
        phi_e = self.B.eval(m.to_ref(e, xq))
        out = {"n": n, "w": w, "lam": lam, "xq": xq,
               "Fself": phi_e.T @ ((w * lam)[:, None] * phi_e), "phi_e": phi_e}
        nb = m.nbr[e, f]
        if nb >= 0:
            phi_n = self.B.eval(m.to_ref(nb, xq))
            out["Fcross"] = phi_e.T @ ((w * lam)[:, None] * phi_n)
        # equispaced face nodes (physical) for interpolated boundary data
        out["xnodes"] = Y[0] + self.face_nodes_ref @ Bf.T
        out["lam_nodes"] = m.barycentric(e, out["xnodes"])
        self._face[key] = out
        return out

    # ---------------------------------------------------------------- tent operators
    def tent(self, tau, v, t_top):
        """Assemble the operators of the tent at vertex v from the front tau to t_top."""
        m, sys, nc = self.mesh, self.sys, self.nc
        es = m.v2e[v]
        ks = [int(np.where(m.cells[e] == v)[0][0]) for e in es]
        pos = {int(e): i for i, e in enumerate(es)}
        H = t_top - tau[v]
        tau_t = tau.copy()
        tau_t[v] = t_top
        T = {"es": es, "ks": ks, "H": H, "v": v, "tau_b": tau.copy(), "tau_t": tau_t,
             "A": {}, "data_faces": []}
        T["gphi_b"], T["gphi_t"], T["mass"], T["eps"], T["mu"] = [], [], [], [], []
        I = np.eye(nc)
        for i, (e, k) in enumerate(zip(es, ks)):
            gb = tau[m.cells[e]] @ m.grad_lam[e]          # grad of the P1 bottom front
            gt = tau_t[m.cells[e]] @ m.grad_lam[e]        # grad of the P1 top front
            T["gphi_b"].append(gb)
            T["gphi_t"].append(gt)
            T["mass"].append(np.kron(I, self.mass(e)))
            T["eps"].append(m.eps[e])
            T["mu"].append(m.mu[e])
            D = self.vol(e, k)
            Aee = sum(np.kron(sys.Aj[j], H * D[j]) for j in range(self.d))
            T["A"][(i, i)] = Aee
            for f in range(self.d + 1):
                if f == k:
                    continue  # the face opposite V lies on the patch boundary: delta = 0
                fc = self.face(e, f, k)
                nb = m.nbr[e, f]
                if "B" not in fc:
                    z = None
                    if self.flux_kind == "impedance":   # walls and data: the element's own medium
                        o = nb if nb >= 0 else e
                        z = (np.sqrt(m.mu[e] / m.eps[e]), np.sqrt(m.mu[o] / m.eps[o]))
                    fc["B"] = sys.flux_matrices(fc["n"], self.alpha, z)
                Bi, Bo = fc["B"]
                if nb >= 0:
                    j = pos[int(nb)]
                    T["A"][(i, i)] = T["A"][(i, i)] - np.kron(Bi, H * fc["Fself"])
                    T["A"][(i, j)] = T["A"].get((i, j), 0.0) - np.kron(Bo, H * fc["Fcross"])
                else:
                    kind = int(m.face_bc[e, f])
                    if kind == DATA:
                        T["A"][(i, i)] = T["A"][(i, i)] - np.kron(Bi, H * fc["Fself"])
                        T["data_faces"].append((i, e, k, fc, Bo))
                    else:
                        R = sys.ghost_matrix(kind)
                        T["A"][(i, i)] = T["A"][(i, i)] - np.kron(Bi + Bo @ R, H * fc["Fself"])
        return T

    def M_of(self, T, th):
        """Per-element blocks of M(th) = (g - f grad phi(th)) tested against the basis."""
        out = []
        for i, e in enumerate(T["es"]):
            b = (1 - th) * T["gphi_b"][i] + th * T["gphi_t"][i]
            K = self.sys.K(b, T["eps"][i], T["mu"][i])
            out.append(np.kron(K, self.mass(e)))
        return out

    def Mprime(self, T):
        """dM/dth: -f(u) (grad phi_t - grad phi_b) tested against the basis."""
        out = []
        for i, e in enumerate(T["es"]):
            bp = T["gphi_t"][i] - T["gphi_b"][i]
            out.append(np.kron(-self.sys.A(bp), self.mass(e)))
        return out

    def apply_A(self, T, U):
        out = [np.zeros(self.nc * self.nb) for _ in T["es"]]
        for (i, j), blk in T["A"].items():
            out[i] += blk @ U[j]
        return out

    def source(self, T, th, k):
        """k-th th-derivative of the boundary-data term b(th) at th, per element."""
        out = [np.zeros(self.nc * self.nb) for _ in T["es"]]
        if not T["data_faces"]:
            return out
        ex = self.data
        H = T["H"]
        for (i, e, kv, fc, Bo) in T["data_faces"]:
            cells = self.mesh.cells[e]
            lam = fc["lam_nodes"]
            delta = H * lam[:, kv]
            phi = lam @ T["tau_b"][cells] + th * delta      # phi(x, th) at the face nodes
            g_nodes = np.stack([(delta[s] ** k) * ex.dt(fc["xnodes"][s], phi[s], k)
                                for s in range(len(delta))])            # (nfn, nc)
            g_q = self.face_interp @ g_nodes                             # (nq, nc)
            flux = g_q @ Bo.T                                            # (nq, nc)
            wl = fc["w"] * H * fc["lam"]
            contrib = np.einsum("q,qc,qb->cb", wl, flux, fc["phi_e"])    # (nc, nb)
            out[i] = out[i] - contrib.ravel()
        return out

    # ---------------------------------------------------------------- time stepping
    def sat(self, T, Y, q, m):
        """q-stage SAT on m sub-intervals (eqs. coeff_rec and recursion-init)."""
        Mp = self.Mprime(T)
        ne = len(T["es"])
        for i in range(m):
            th = i / m
            Mi = self.M_of(T, th)
            U = [np.linalg.solve(Mi[e], Y[e]) for e in range(ne)]
            Ys = [Y]
            for n in range(1, q + 1):
                AU = self.apply_A(T, U)
                src = self.source(T, th, n - 1)
                Yn = [AU[e] + src[e] for e in range(ne)]
                Ys.append(Yn)
                if n <= q - 1:
                    U = [np.linalg.solve(Mi[e], Yn[e] - n * (Mp[e] @ U[e])) for e in range(ne)]
            Y = [sum(Ys[n][e] / (m ** n * factorial(n)) for n in range(q + 1)) for e in range(ne)]
        return Y

    def rk4(self, T, Y, m):
        """Classical RK4 for dY/dth = A M(th)^{-1} Y + b(th) on m steps."""
        ne = len(T["es"])
        h = 1.0 / m

        def rhs(th, Yc):
            Mt = self.M_of(T, th)
            U = [np.linalg.solve(Mt[e], Yc[e]) for e in range(ne)]
            AU = self.apply_A(T, U)
            src = self.source(T, th, 0)
            return [AU[e] + src[e] for e in range(ne)]

        for i in range(m):
            th = i * h
            k1 = rhs(th, Y)
            k2 = rhs(th + h / 2, [Y[e] + h / 2 * k1[e] for e in range(ne)])
            k3 = rhs(th + h / 2, [Y[e] + h / 2 * k2[e] for e in range(ne)])
            k4 = rhs(th + h, [Y[e] + h * k3[e] for e in range(ne)])
            Y = [Y[e] + h / 6 * (k1[e] + 2 * k2[e] + 2 * k3[e] + k4[e]) for e in range(ne)]
        return Y
