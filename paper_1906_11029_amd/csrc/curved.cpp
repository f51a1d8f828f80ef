// Curved quadratic triangles (section 4: on the few curved elements the projection after the
// pointwise inverse uses an approximation of the inverse mass matrix): checks of the
// geometry, the pitcher's step on a curved element, and the host tables of the curved-element
// tent path.
//
// Geometry: x(xh) = sum_i G_i N_i(xh) with the P2 Lagrange shape functions N_i (vertices
// l_v (2 l_v - 1), midpoints of edges (0,1), (1,2), (0,2): 4 l_a l_b; l the barycentric
// coordinates of xh).  Fronts stay P1 in reference coordinates, so grad lambda_k =
// J^{-T} gradhat lambdahat_k varies inside a curved element.  Quadrature: the n-point
// collapsed Gauss-Jacobi rule of the reference triangle, x = u, y = (1 - u) v with u the
// Gauss-Jacobi points of weight (1 - u) and v the Gauss-Legendre points on [0, 1]; volume
// integrals with n = p + 4, the weight-adjusted mass with n = p + 8, faces with p + 4
// Gauss-Legendre points.  Inverse mass: the weight-adjusted one, Mhat^{-1} M_{1/J} Mhat^{-1}.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace mtp {

namespace {

const double kRefV[3][2] = {{0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}};
const double kHatGrad[3][2] = {{-1.0, -1.0}, {1.0, 0.0}, {0.0, 1.0}};
const int kEdge[3][2] = {{0, 1}, {1, 2}, {0, 2}};     // geometry midpoint nodes 3, 4, 5

void bary(const double* xh, double* l) {
  l[0] = 1.0 - xh[0] - xh[1];
  l[1] = xh[0];
  l[2] = xh[1];
}

void p2_shape(const double* xh, double* N) {
  double l[3];
  bary(xh, l);
  for (int v = 0; v < 3; ++v) N[v] = l[v] * (2.0 * l[v] - 1.0);
  for (int s = 0; s < 3; ++s) N[3 + s] = 4.0 * l[kEdge[s][0]] * l[kEdge[s][1]];
}

// dN_i / dxh_l
void p2_grad(const double* xh, double g[6][2]) {
  double l[3];
  bary(xh, l);
  for (int v = 0; v < 3; ++v)
    for (int x = 0; x < 2; ++x) g[v][x] = (4.0 * l[v] - 1.0) * kHatGrad[v][x];
  for (int s = 0; s < 3; ++s) {
    const int a = kEdge[s][0], b = kEdge[s][1];
    for (int x = 0; x < 2; ++x) g[3 + s][x] = 4.0 * (l[a] * kHatGrad[b][x] + l[b] * kHatGrad[a][x]);
  }
}

// J[r][l] = d x_r / d xh_l
void p2_jac(const double* G, const double* xh, double J[2][2]) {
  double g[6][2];
  p2_grad(xh, g);
  for (int r = 0; r < 2; ++r)
    for (int l = 0; l < 2; ++l) {
      double s = 0.0;
      for (int i = 0; i < 6; ++i) s += G[i * 2 + r] * g[i][l];
      J[r][l] = s;
    }
}

// Jinv[l][r] = d xh_l / d x_r; returns det J
double inv2(const double J[2][2], double Jinv[2][2]) {
  const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  Jinv[0][0] = J[1][1] / det;
  Jinv[0][1] = -J[0][1] / det;
  Jinv[1][0] = -J[1][0] / det;
  Jinv[1][1] = J[0][0] / det;
  return det;
}

// Jacobi polynomial P_n^{(alpha, 0)}(z) and its derivative
void jacobi(int n, int alpha, double z, double& p, double& dp) {
  const double a = alpha;
  double p0 = 1.0, p1 = 0.5 * ((a + 2.0) * z + a);
  if (n == 0) {
    p = 1.0;
    dp = 0.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    const double c1 = 2.0 * k * (k + a) * (2.0 * k + a - 2.0);
    const double c2 = (2.0 * k + a - 1.0) * ((2.0 * k + a) * (2.0 * k + a - 2.0) * z + a * a);
    const double c4 = 2.0 * (k + a - 1.0) * (k - 1.0) * (2.0 * k + a);
    const double p2 = (c2 * p1 - c4 * p0) / c1;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  // (2n + a)(1 - z^2) P_n' = n (a - (2n + a) z) P_n + 2 (n + a) n P_{n-1}
  dp = (n * (a - (2.0 * n + a) * z) * p1 + 2.0 * (n + a) * n * p0) / ((2.0 * n + a) * (1.0 - z * z));
}

// n-point Gauss-Jacobi rule on [0,1] for the weight (1 - u)^alpha (alpha 0 or 1): Newton with
// deflation on P_n^{(alpha, 0)}(z), u = (z + 1) / 2, weights 1 / ((1 - z^2) P_n'(z)^2);
// points ascending
void gauss_jacobi01(int n, int alpha, std::vector<double>& u, std::vector<double>& w) {
  std::vector<double> z(n);
  for (int k = 0; k < n; ++k) {
    double x = -std::cos(M_PI * (k + 0.75) / (n + 0.5));
    for (int it = 0; it < 200; ++it) {
      double p, dp;
      jacobi(n, alpha, x, p, dp);
      double s = 0.0;
      for (int j = 0; j < k; ++j) s += 1.0 / (x - z[j]);
      const double dx = p / (dp - p * s);
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    z[k] = x;
  }
  std::sort(z.begin(), z.end());
  u.resize(n);
  w.resize(n);
  for (int k = 0; k < n; ++k) {
    double p, dp;
    jacobi(n, alpha, z[k], p, dp);
    u[k] = 0.5 * (z[k] + 1.0);
    w[k] = 1.0 / ((1.0 - z[k] * z[k]) * dp * dp);
  }
}

// the collapsed rule of the reference triangle: pts (n*n, 2), weights summing to 1/2
void collapsed_rule(int n, std::vector<double>& pts, std::vector<double>& wts) {
  std::vector<double> u, wu, v, wv;
  gauss_jacobi01(n, 1, u, wu);
  gauss_jacobi01(n, 0, v, wv);
  pts.clear();
  wts.clear();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      pts.push_back(u[i]);
      pts.push_back((1.0 - u[i]) * v[j]);
      wts.push_back(wu[i] * wv[j]);
    }
}

// Lagrange basis at the equispaced nodes (barycentric multi-indices mi, 3 per node) and its
// reference gradient: phi_a = prod_m prod_{r < mi_m} (p l_m - r) / (r + 1)
void lagrange(int p, const std::vector<int32_t>& mi, const double* xh, double* phi, double* grad) {
  const int np = (int)mi.size() / 3;
  double l[3];
  bary(xh, l);
  for (int a = 0; a < np; ++a) {
    double f[3], df[3];
    for (int m = 0; m < 3; ++m) {
      double val = 1.0, der = 0.0;
      for (int r = 0; r < mi[a * 3 + m]; ++r) {
        const double fr = (p * l[m] - r) / (r + 1.0);
        der = der * fr + val * p / (r + 1.0);
        val *= fr;
      }
      f[m] = val;
      df[m] = der;
    }
    phi[a] = f[0] * f[1] * f[2];
    if (grad) {
      const double d0 = df[0] * f[1] * f[2], d1 = f[0] * df[1] * f[2], d2 = f[0] * f[1] * df[2];
      grad[a * 2 + 0] = d1 - d0;
      grad[a * 2 + 1] = d2 - d0;
    }
  }
}

// A := A^{-1} for a symmetric positive definite n x n matrix (Cholesky)
void spd_inverse(int n, std::vector<double>& A) {
  std::vector<double> L(A);
  for (int j = 0; j < n; ++j) {
    double s = L[j * n + j];
    for (int q = 0; q < j; ++q) s -= L[j * n + q] * L[j * n + q];
    if (!(s > 0)) throw Error(MTP_ERR_MESH, "curved element: mass matrix not positive definite");
    const double r = std::sqrt(s);
    L[j * n + j] = r;
    for (int i = j + 1; i < n; ++i) {
      double t = L[i * n + j];
      for (int q = 0; q < j; ++q) t -= L[i * n + q] * L[j * n + q];
      L[i * n + j] = t / r;
    }
  }
  for (int c = 0; c < n; ++c) {
    std::vector<double> x(n, 0.0);
    x[c] = 1.0;
    for (int i = 0; i < n; ++i) {
      double t = x[i];
      for (int q = 0; q < i; ++q) t -= L[i * n + q] * x[q];
      x[i] = t / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = x[i];
      for (int q = i + 1; q < n; ++q) t -= L[q * n + i] * x[q];
      x[i] = t / L[i * n + i];
    }
    for (int i = 0; i < n; ++i) A[i * n + c] = x[i];
  }
}

}  // namespace

void curved_node(const Mesh& m, int64_t e, const double* xh, double* x) {
  double N[6];
  p2_shape(xh, N);
  for (int r = 0; r < 2; ++r) {
    double s = 0.0;
    for (int i = 0; i < 6; ++i) s += m.geo[(e * 6 + i) * 2 + r] * N[i];
    x[r] = s;
  }
}

double curved_step(const Mesh& m, int64_t e, double slope) {
  const int n = 12;
  const double* G = &m.geo[e * 12];
  double worst = 0.0;
  for (int j = 0; j <= n; ++j)
    for (int i = 0; i + j <= n; ++i) {
      const double xh[2] = {(double)i / n, (double)j / n};
      double J[2][2], Ji[2][2];
      p2_jac(G, xh, J);
      inv2(J, Ji);
      double nrm[3], tot = 0.0;
      for (int k = 0; k < 3; ++k) {
        double g[2];
        for (int r = 0; r < 2; ++r) g[r] = Ji[0][r] * kHatGrad[k][0] + Ji[1][r] * kHatGrad[k][1];
        nrm[k] = std::sqrt(g[0] * g[0] + g[1] * g[1]);
        tot += nrm[k];
      }
      double best = 1e300;
      for (int k = 0; k < 3; ++k) best = std::min(best, tot - nrm[k]);
      worst = std::max(worst, best);
    }
  return slope * std::sqrt(m.eps[e] * m.mu[e]) / worst;
}

void set_curved_p2(Mesh& m, const double* nodes) {
  if (m.d != 2) throw Error(MTP_ERR_ARG, "curved elements: 2D meshes only");
  std::vector<double> geo(nodes, nodes + m.ne * 12);
  std::vector<uint8_t> curved(m.ne, 0);
  int64_t nc = 0;
  for (int64_t e = 0; e < m.ne; ++e) {
    const double* G = &geo[e * 12];
    double scale = 1.0;
    for (int v = 0; v < 3; ++v)
      for (int r = 0; r < 2; ++r) {
        const double x = m.coords[m.cells[e * 3 + v] * 2 + r];
        if (!std::isfinite(G[v * 2 + r]) || G[v * 2 + r] != x)
          throw Error(MTP_ERR_ARG, "curved elements: the first three nodes of an element must be its vertices");
        scale = std::max(scale, 1.0 + std::fabs(x));
      }
    for (int s = 0; s < 3; ++s)
      for (int r = 0; r < 2; ++r) {
        const double mid = 0.5 * (G[kEdge[s][0] * 2 + r] + G[kEdge[s][1] * 2 + r]);
        if (!std::isfinite(G[(3 + s) * 2 + r])) throw Error(MTP_ERR_ARG, "curved elements: non-finite node");
        if (std::fabs(G[(3 + s) * 2 + r] - mid) > 1e-14 * scale) curved[e] = 1;
      }
    if (curved[e]) {
      ++nc;
      const int n = 12;
      for (int j = 0; j <= n; ++j)
        for (int i = 0; i + j <= n; ++i) {
          const double xh[2] = {(double)i / n, (double)j / n};
          double J[2][2];
          p2_jac(G, xh, J);
          if (!(J[0][0] * J[1][1] - J[0][1] * J[1][0] > 0.0))
            throw Error(MTP_ERR_MESH, "curved element with a non-positive Jacobian");
        }
    }
  }
  // a shared edge must have one midpoint node: face f of an element is its edge opposite
  // vertex f, i.e. geometry midpoint 3 + s with kEdge[s] the two other vertices
  auto mid_of_face = [&](int64_t e, int f) -> const double* {
    for (int s = 0; s < 3; ++s)
      if (kEdge[s][0] != f && kEdge[s][1] != f) return &geo[e * 12 + (3 + s) * 2];
    return nullptr;
  };
  for (int64_t e = 0; e < m.ne; ++e)
    for (int f = 0; f < 3; ++f) {
      const int32_t nb = m.nbr[e * 3 + f];
      if (nb < 0) continue;
      const double* a = mid_of_face(e, f);
      const double* b = mid_of_face(nb, m.nbr_face[e * 3 + f]);
      if (std::fabs(a[0] - b[0]) > 1e-14 * (1.0 + std::fabs(a[0])) ||
          std::fabs(a[1] - b[1]) > 1e-14 * (1.0 + std::fabs(a[1])))
        throw Error(MTP_ERR_MESH, "curved elements: a shared edge with two different midpoint nodes");
    }
  m.geo.swap(geo);
  m.curved.swap(curved);
  m.n_curved = nc;
}

CurvedPlan curved_plan(const Mesh& m, const Tents& t, int p) {
  CurvedPlan cp;
  cp.p = p;
  cp.np = (p + 1) * (p + 2) / 2;
  cp.nq = (p + 4) * (p + 4);
  cp.nfq = p + 4;
  cp.tent_curved.assign(t.vertex.size(), 0);
  cp.zone.assign(m.ne, -1);
  if (m.n_curved == 0) return cp;
  for (size_t i = 0; i < t.vertex.size(); ++i) {
    const int32_t v = t.vertex[i];
    bool c = false;
    for (int64_t k = m.v2e_ptr[v]; k < m.v2e_ptr[v + 1]; ++k) c = c || m.curved[m.v2e[k]];
    if (!c) continue;
    cp.tent_curved[i] = 1;
    cp.max_patch = std::max(cp.max_patch, (int)(m.v2e_ptr[v + 1] - m.v2e_ptr[v]));
    for (int64_t k = m.v2e_ptr[v]; k < m.v2e_ptr[v + 1]; ++k) {
      const int32_t e = m.v2e[k];
      if (cp.zone[e] < 0) {
        cp.zone[e] = (int32_t)cp.zone_elem.size();
        cp.zone_elem.push_back(e);
      }
    }
  }
  return cp;
}

void curved_tables(const Mesh& m, const CurvedPlan& cp, const std::vector<int32_t>& mi, std::vector<double>& ref,
                   std::vector<double>& geo, std::vector<int32_t>& nbr) {
  const int p = cp.p, np = cp.np, nq = cp.nq, nfq = cp.nfq;
  std::vector<double> qp, qw, qp8, qw8, fs, fw;
  collapsed_rule(p + 4, qp, qw);
  collapsed_rule(p + 8, qp8, qw8);
  gauss_jacobi01(nfq, 0, fs, fw);
  // reference tables
  ref.assign(cp.n_ref(), 0.0);
  double* V = ref.data();
  double* Gr = V + (size_t)nq * np;
  double* Lam = Gr + (size_t)nq * np * 2;
  double* Vf = Lam + (size_t)nq * 3;
  double* Lamf = Vf + 3 * (size_t)nfq * np;
  for (int q = 0; q < nq; ++q) {
    lagrange(p, mi, &qp[q * 2], &V[q * np], &Gr[q * np * 2]);
    bary(&qp[q * 2], &Lam[q * 3]);
  }
  // face f: the edge opposite vertex f, parametrised from its lower to its higher vertex
  auto face_point = [&](int f, double s, double* xh) {
    int a = -1, b = -1;
    for (int i = 0; i < 3; ++i)
      if (i != f) (a < 0 ? a : b) = i;
    for (int r = 0; r < 2; ++r) xh[r] = kRefV[a][r] + s * (kRefV[b][r] - kRefV[a][r]);
    return std::make_pair(a, b);
  };
  for (int f = 0; f < 3; ++f)
    for (int q = 0; q < nfq; ++q) {
      double xh[2];
      face_point(f, fs[q], xh);
      lagrange(p, mi, xh, &Vf[(f * nfq + q) * np], nullptr);
      bary(xh, &Lamf[(f * nfq + q) * 3]);
    }
  // reference Lagrange mass (exact with p + 8 points)
  std::vector<double> phi(np);
  std::vector<double> Mh((size_t)np * np, 0.0);
  const int nq8 = (int)qw8.size();
  std::vector<double> V8((size_t)nq8 * np);
  for (int q = 0; q < nq8; ++q) {
    lagrange(p, mi, &qp8[q * 2], &V8[(size_t)q * np], nullptr);
    for (int a = 0; a < np; ++a)
      for (int b = 0; b < np; ++b) Mh[a * np + b] += qw8[q] * V8[(size_t)q * np + a] * V8[(size_t)q * np + b];
  }
  std::vector<double> Mhi(Mh);
  spd_inverse(np, Mhi);
  // per zone element
  const size_t nz = cp.zone_elem.size();
  const size_t per = (size_t)nq * 5 + (size_t)np * np + 3 * (size_t)nfq * 3;
  geo.assign(nz * per, 0.0);
  nbr.assign(nz * 6, 0);
  for (size_t z = 0; z < nz; ++z) {
    const int32_t e = cp.zone_elem[z];
    std::vector<double> G(12);
    if (m.n_curved > 0) {
      for (int i = 0; i < 12; ++i) G[i] = m.geo[(size_t)e * 12 + i];
    }
    double* Q = &geo[z * per];
    double* Mi = Q + (size_t)nq * 5;
    double* F = Mi + (size_t)np * np;
    for (int q = 0; q < nq; ++q) {
      double J[2][2], Ji[2][2];
      p2_jac(G.data(), &qp[q * 2], J);
      const double det = inv2(J, Ji);
      Q[q * 5 + 0] = qw[q] * std::fabs(det);
      Q[q * 5 + 1] = Ji[0][0];
      Q[q * 5 + 2] = Ji[0][1];
      Q[q * 5 + 3] = Ji[1][0];
      Q[q * 5 + 4] = Ji[1][1];
    }
    // M_{1/J} and the weight-adjusted inverse Mhat^{-1} M_{1/J} Mhat^{-1}
    std::vector<double> Mj((size_t)np * np, 0.0);
    for (int q = 0; q < nq8; ++q) {
      double J[2][2];
      p2_jac(G.data(), &qp8[q * 2], J);
      const double wq = qw8[q] / std::fabs(J[0][0] * J[1][1] - J[0][1] * J[1][0]);
      for (int a = 0; a < np; ++a)
        for (int b = 0; b < np; ++b) Mj[a * np + b] += wq * V8[(size_t)q * np + a] * V8[(size_t)q * np + b];
    }
    std::vector<double> T((size_t)np * np, 0.0);
    for (int a = 0; a < np; ++a)
      for (int b = 0; b < np; ++b) {
        double s = 0.0;
        for (int c = 0; c < np; ++c) s += Mhi[a * np + c] * Mj[c * np + b];
        T[a * np + b] = s;
      }
    for (int a = 0; a < np; ++a)
      for (int b = 0; b < np; ++b) {
        double s = 0.0;
        for (int c = 0; c < np; ++c) s += T[a * np + c] * Mhi[c * np + b];
        Mi[a * np + b] = s;
      }
    // faces: w |dx/ds| and the outward unit normal at each point
    double xc[2];
    {
      const double c3[2] = {1.0 / 3.0, 1.0 / 3.0};
      double N[6];
      p2_shape(c3, N);
      for (int r = 0; r < 2; ++r) {
        double s = 0.0;
        for (int i = 0; i < 6; ++i) s += G[i * 2 + r] * N[i];
        xc[r] = s;
      }
    }
    for (int f = 0; f < 3; ++f) {
      for (int q = 0; q < nfq; ++q) {
        double xh[2];
        const auto ab = face_point(f, fs[q], xh);
        double J[2][2];
        p2_jac(G.data(), xh, J);
        double t[2];
        for (int r = 0; r < 2; ++r)
          t[r] = J[r][0] * (kRefV[ab.second][0] - kRefV[ab.first][0]) +
                 J[r][1] * (kRefV[ab.second][1] - kRefV[ab.first][1]);
        const double len = std::sqrt(t[0] * t[0] + t[1] * t[1]);
        double n[2] = {t[1] / len, -t[0] / len};
        double N[6], x[2];
        p2_shape(xh, N);
        for (int r = 0; r < 2; ++r) {
          double s = 0.0;
          for (int i = 0; i < 6; ++i) s += G[i * 2 + r] * N[i];
          x[r] = s;
        }
        if (n[0] * (xc[0] - x[0]) + n[1] * (xc[1] - x[1]) > 0) {
          n[0] = -n[0];
          n[1] = -n[1];
        }
        double* Fq = &F[(f * nfq + q) * 3];
        Fq[0] = fw[q] * len;
        Fq[1] = n[0];
        Fq[2] = n[1];
      }
      // neighbour: element (or -1 - boundary kind) and its face, reversed when the shared
      // edge's lower-to-higher vertex order differs between the two elements
      const int32_t nb = m.nbr[(size_t)e * 3 + f];
      if (nb < 0) {
        nbr[z * 6 + f] = -1 - m.face_bc[(size_t)e * 3 + f];
        nbr[z * 6 + 3 + f] = 0;
      } else {
        const int fn = m.nbr_face[(size_t)e * 3 + f];
        int a = -1, an = -1;
        for (int i = 0; i < 3; ++i)
          if (i != f) { a = i; break; }
        for (int i = 0; i < 3; ++i)
          if (i != fn) { an = i; break; }
        const bool rev = m.cells[(size_t)e * 3 + a] != m.cells[(size_t)nb * 3 + an];
        nbr[z * 6 + f] = nb;
        nbr[z * 6 + 3 + f] = fn | (rev ? 4 : 0);
      }
    }
  }
}

}  // namespace mtp
