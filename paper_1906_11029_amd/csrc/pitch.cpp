// Tent pitching on the host (section 2: one vertex moves at a time, limited by causality;
// vertices at graph distance >= 2 move independently and form a layer).
//
// Rule: per element k_T = slope*sqrt(eps mu) / min_i sum_{j != i} |grad lambda_j|, per
// edge k_vw = min over the edge's elements.  The vertex with the smallest (time, id) moves
// to min(t_end, Q floor((min_w tau_w + k_vw)/Q - 1e-3)), Q = 2^-24.  Every edge then keeps
// |tau_v - tau_w| <= k_vw, so on every element
//   |grad phi| = |sum_{j != i} (tau_j - tau_i) grad lambda_j| <= slope*sqrt(eps mu),
// and the minimum vertex always advances (no stalls).  Times are multiples of Q.  On a curved
// (quadratic) triangle grad lambda_j varies; its k_T takes the largest value of
// min_i sum_{j != i} |grad lambda_j(x)| over the barycentric lattice (i/12, j/12).
#include <algorithm>
#include <cmath>
#include <functional>
#include <queue>

#include "internal.h"

namespace mtp {

void pitch(const Mesh& m, double t_end, double slope, Tents& out) {
  const int d = m.d, nvert = d + 1;
  const double Q = std::ldexp(1.0, -24);
  const double SAFETY = 1e-3;
  // element step k_T
  std::vector<double> kT(m.ne);
  for (int64_t e = 0; e < m.ne; ++e) {
    double nrm[4], tot = 0.0;
    for (int j = 0; j < nvert; ++j) {
      const double* g = &m.grad_lam[(e * nvert + j) * d];
      double s = 0.0;
      for (int i = 0; i < d; ++i) s += g[i] * g[i];
      nrm[j] = std::sqrt(s);
      tot += nrm[j];
    }
    double best = 1e300;
    for (int i = 0; i < nvert; ++i) best = std::min(best, tot - nrm[i]);
    kT[e] = slope * std::sqrt(m.eps[e] * m.mu[e]) / best;
    // a curved element: the same bound taken pointwise, at its worst point of the lattice
    if (m.n_curved > 0 && m.curved[e]) kT[e] = curved_step(m, e, slope);
  }
  // edge steps aligned with the adjacency CSR
  std::vector<double> kvw(m.adj.size(), 1e300);
  for (int64_t v = 0; v < m.nv; ++v) {
    const int32_t* nb0 = &m.adj[m.adj_ptr[v]];
    const int32_t* nb1 = m.adj.data() + m.adj_ptr[v + 1];
    for (int64_t i = m.v2e_ptr[v]; i < m.v2e_ptr[v + 1]; ++i) {
      int32_t e = m.v2e[i];
      for (int k = 0; k < nvert; ++k) {
        int32_t w = m.cells[e * nvert + k];
        if (w == v) continue;
        int64_t pos = std::lower_bound(nb0, nb1, w) - m.adj.data();
        kvw[pos] = std::min(kvw[pos], kT[e]);
      }
    }
  }

  std::vector<double> tau(m.nv, 0.0);
  std::vector<int32_t> last(m.nv, -1);
  using Item = std::pair<double, int32_t>;
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
  for (int64_t v = 0; v < m.nv; ++v) heap.push({0.0, (int32_t)v});
  std::vector<int32_t> V, L;
  std::vector<double> TB, TT;
  while (!heap.empty()) {
    auto [tv, v] = heap.top();
    heap.pop();
    if (tv >= t_end) continue;
    double t_plus = 1e300;
    int32_t lay = last[v];
    for (int64_t i = m.adj_ptr[v]; i < m.adj_ptr[v + 1]; ++i) {
      int32_t w = m.adj[i];
      t_plus = std::min(t_plus, tau[w] + kvw[i]);
      lay = std::max(lay, last[w]);
    }
    lay += 1;
    double t_new = std::min(t_end, Q * std::floor(t_plus / Q - SAFETY));
    if (!(t_new > tv)) throw Error(MTP_ERR_PITCH, "vertex " + std::to_string(v) + " cannot advance");
    last[v] = lay;
    V.push_back(v);
    TB.push_back(tv);
    TT.push_back(t_new);
    L.push_back(lay);
    tau[v] = t_new;
    if (t_new < t_end) heap.push({t_new, v});
  }

  // sort by layer, stable in pitching order
  const size_t nt = V.size();
  std::vector<size_t> idx(nt);
  for (size_t i = 0; i < nt; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return L[a] < L[b]; });
  out.t_end = t_end;
  out.slope = slope;
  out.vertex.resize(nt);
  out.t_bot.resize(nt);
  out.t_top.resize(nt);
  out.layer.resize(nt);
  for (size_t i = 0; i < nt; ++i) {
    out.vertex[i] = V[idx[i]];
    out.t_bot[i] = TB[idx[i]];
    out.t_top[i] = TT[idx[i]];
    out.layer[i] = L[idx[i]];
  }
  int32_t nl = nt ? out.layer.back() + 1 : 0;
  out.layer_ptr.assign(nl + 1, 0);
  for (size_t i = 0; i < nt; ++i) out.layer_ptr[out.layer[i] + 1]++;
  for (int32_t l = 0; l < nl; ++l) out.layer_ptr[l + 1] += out.layer_ptr[l];
}

}  // namespace mtp
