// Mesh topology and affine element geometry (section 2: conforming simplicial mesh,
// vertex patches omega_V).
#include <algorithm>
#include <array>
#include <cmath>

#include "internal.h"

namespace mtp {

namespace {

// Gradients of the barycentric coordinates of one simplex.  With e_l = v_l - v_0 the
// rows of J^{-1} (J = [e_1 .. e_d]) are grad lambda_l; grad lambda_0 = -sum_l grad lambda_l.
// 2D: J^{-1} = adj(J)/det;  3D: rows (e2 x e3, e3 x e1, e1 x e2)/det.
double simplex_gradients(int d, const double* X, double* g) {
  if (d == 2) {
    double a = X[2] - X[0], b = X[4] - X[0];  // x components of e1, e2
    double c = X[3] - X[1], e = X[5] - X[1];  // y components
    double det = a * e - b * c;
    // J = [[a, b], [c, e]]; J^{-1} = [[e, -b], [-c, a]] / det
    g[2] = e / det;  g[3] = -b / det;   // grad lambda_1
    g[4] = -c / det; g[5] = a / det;    // grad lambda_2
    g[0] = -(g[2] + g[4]);
    g[1] = -(g[3] + g[5]);
    return det;
  }
  double e1[3], e2[3], e3[3];
  for (int i = 0; i < 3; ++i) {
    e1[i] = X[3 + i] - X[i];
    e2[i] = X[6 + i] - X[i];
    e3[i] = X[9 + i] - X[i];
  }
  auto cross = [](const double* u, const double* v, double* w) {
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
  };
  double c23[3], c31[3], c12[3];
  cross(e2, e3, c23);
  cross(e3, e1, c31);
  cross(e1, e2, c12);
  double det = e1[0] * c23[0] + e1[1] * c23[1] + e1[2] * c23[2];
  for (int i = 0; i < 3; ++i) {
    g[3 + i] = c23[i] / det;
    g[6 + i] = c31[i] / det;
    g[9 + i] = c12[i] / det;
    g[i] = -(g[3 + i] + g[6 + i] + g[9 + i]);
  }
  return det;
}

}  // namespace

void build_topology(Mesh& m) {
  const int d = m.d, nvert = d + 1;
  if (d != 2 && d != 3) throw Error(MTP_ERR_ARG, "dim must be 2 or 3");
  for (int64_t i = 0; i < m.ne * nvert; ++i)
    if (m.cells[i] < 0 || m.cells[i] >= m.nv) throw Error(MTP_ERR_MESH, "cell vertex id out of range");
  for (int64_t e = 0; e < m.ne; ++e)
    if (!(m.eps[e] > 0.0) || !(m.mu[e] > 0.0)) throw Error(MTP_ERR_MESH, "eps and mu must be positive");
  for (int64_t i = 0; i < m.ne * nvert; ++i)
    if (m.face_bc[i] < MTP_BC_PEC || m.face_bc[i] > MTP_BC_DATA) throw Error(MTP_ERR_MESH, "unknown boundary kind");

  // geometry
  m.grad_lam.assign(m.ne * nvert * d, 0.0);
  m.volume.assign(m.ne, 0.0);
  const double dfact = (d == 2) ? 2.0 : 6.0;
  std::vector<double> X(nvert * d);
  for (int64_t e = 0; e < m.ne; ++e) {
    for (int k = 0; k < nvert; ++k)
      for (int i = 0; i < d; ++i) X[k * d + i] = m.coords[m.cells[e * nvert + k] * d + i];
    double det = simplex_gradients(d, X.data(), &m.grad_lam[e * nvert * d]);
    m.volume[e] = std::fabs(det) / dfact;
    if (!(m.volume[e] > 0.0) || !std::isfinite(det))
      throw Error(MTP_ERR_MESH, "degenerate element " + std::to_string(e));
  }

  // face neighbours: sort (sorted face vertex tuple, element, local face)
  struct FaceRec { std::array<int32_t, 3> key; int32_t e; int8_t j; };
  std::vector<FaceRec> faces;
  faces.reserve(m.ne * nvert);
  for (int64_t e = 0; e < m.ne; ++e)
    for (int j = 0; j < nvert; ++j) {
      FaceRec r{{-1, -1, -1}, (int32_t)e, (int8_t)j};
      int c = 0;
      for (int k = 0; k < nvert; ++k)
        if (k != j) r.key[c++] = m.cells[e * nvert + k];
      std::sort(r.key.begin(), r.key.begin() + d);
      faces.push_back(r);
    }
  std::sort(faces.begin(), faces.end(), [](const FaceRec& a, const FaceRec& b) {
    if (a.key != b.key) return a.key < b.key;
    return a.e < b.e;
  });
  m.nbr.assign(m.ne * nvert, -1);
  m.nbr_face.assign(m.ne * nvert, -1);
  for (size_t i = 0; i < faces.size();) {
    size_t j = i + 1;
    while (j < faces.size() && faces[j].key == faces[i].key) ++j;
    if (j - i > 2) throw Error(MTP_ERR_MESH, "face shared by more than two elements");
    if (j - i == 2) {
      const FaceRec &a = faces[i], &b = faces[i + 1];
      if (a.e == b.e) throw Error(MTP_ERR_MESH, "repeated vertex in an element");
      m.nbr[a.e * nvert + a.j] = b.e;
      m.nbr_face[a.e * nvert + a.j] = b.j;
      m.nbr[b.e * nvert + b.j] = a.e;
      m.nbr_face[b.e * nvert + b.j] = a.j;
    }
    i = j;
  }

  // vertex patches
  m.v2e_ptr.assign(m.nv + 1, 0);
  for (int64_t i = 0; i < m.ne * nvert; ++i) m.v2e_ptr[m.cells[i] + 1]++;
  for (int64_t v = 0; v < m.nv; ++v) m.v2e_ptr[v + 1] += m.v2e_ptr[v];
  m.v2e.assign(m.ne * nvert, 0);
  m.v2e_k.assign(m.ne * nvert, 0);
  std::vector<int64_t> fill(m.v2e_ptr.begin(), m.v2e_ptr.end() - 1);
  for (int64_t e = 0; e < m.ne; ++e)
    for (int k = 0; k < nvert; ++k) {
      int32_t v = m.cells[e * nvert + k];
      m.v2e[fill[v]] = (int32_t)e;
      m.v2e_k[fill[v]] = (int8_t)k;
      fill[v]++;
    }
  m.max_patch = 0;
  for (int64_t v = 0; v < m.nv; ++v)
    m.max_patch = std::max<int>(m.max_patch, (int)(m.v2e_ptr[v + 1] - m.v2e_ptr[v]));

  // vertex adjacency (sorted, unique)
  m.adj_ptr.assign(m.nv + 1, 0);
  m.adj.clear();
  std::vector<int32_t> nb;
  for (int64_t v = 0; v < m.nv; ++v) {
    nb.clear();
    for (int64_t i = m.v2e_ptr[v]; i < m.v2e_ptr[v + 1]; ++i) {
      int32_t e = m.v2e[i];
      for (int k = 0; k < nvert; ++k) {
        int32_t w = m.cells[e * nvert + k];
        if (w != v) nb.push_back(w);
      }
    }
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    m.adj.insert(m.adj.end(), nb.begin(), nb.end());
    m.adj_ptr[v + 1] = (int64_t)m.adj.size();
  }
}

}  // namespace mtp
