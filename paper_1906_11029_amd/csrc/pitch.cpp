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
//
// The colour rule moves the vertices in another order: the vertex graph is coloured greedily
// (vertex ids ascending, smallest colour no neighbour holds), and the colours take turns; at
// its turn every vertex of the colour below t_end moves to the same target, capped at
// tau_v + 1.5 min_w k_vw, if that lies above its time.  A colour is an independent set, so
// its moves read only fronts of other colours and commute.  A vertex that waited while its
// neighbours rose would otherwise make a pole up to twice its smallest edge step; the
// pseudo-time operator scales with the pole height, and such tents next to a material jump
// made the SAT recursion grow without bound.  The cap keeps every pole at most 1.5 edge
// steps.  The global minimum vertex moves at its colour's turn by at least min_w k_vw, so
// every C turns something moves (no stalls).  Both rules put a tent in layer 1 + the largest
// layer of itself and its neighbours.
#include <algorithm>
#include <cmath>
#include <functional>
#include <queue>

#include "internal.h"

namespace mtp {

namespace {

// greedy colouring of the vertex graph: vertex ids ascending, smallest colour unused by
// the already coloured neighbours
int32_t colour_vertices(const Mesh& m, std::vector<int32_t>& col) {
  col.assign(m.nv, -1);
  int32_t n_col = 0;
  std::vector<int64_t> seen;   // seen[c] == v: colour c is taken around v
  for (int64_t v = 0; v < m.nv; ++v) {
    for (int64_t i = m.adj_ptr[v]; i < m.adj_ptr[v + 1]; ++i) {
      int32_t c = col[m.adj[i]];
      if (c >= 0) {
        if ((size_t)c >= seen.size()) seen.resize(c + 1, -1);
        seen[c] = v;
      }
    }
    int32_t c = 0;
    while ((size_t)c < seen.size() && seen[c] == v) ++c;
    col[v] = c;
    n_col = std::max(n_col, c + 1);
  }
  return n_col;
}

}  // namespace

// The automatic rule: both tables, and the one with less work, the sum over its tents of
// the patch sizes (a tent's cost grows with its patch); the minimum-vertex table on a tie.
// The colour pitch stops as soon as its work reaches the minimum-vertex table's, since it
// can no longer win (work only grows): the same choice, without finishing a table that can
// be far larger (the jittered Delaunay cube: 48 times the tents).
void pitch(const Mesh& m, double t_end, double slope, int rule, Tents& out) {
  if (rule == MTP_PITCH_AUTO) {
    Tents a, b;
    pitch_rule(m, t_end, slope, MTP_PITCH_MIN_VERTEX, a);
    int64_t wa = 0;
    for (int32_t v : a.vertex) wa += m.v2e_ptr[v + 1] - m.v2e_ptr[v];
    const bool done = pitch_rule(m, t_end, slope, MTP_PITCH_COLOUR, b, wa);
    out = done ? std::move(b) : std::move(a);
    return;
  }
  pitch_rule(m, t_end, slope, rule, out);
}

bool pitch_rule(const Mesh& m, double t_end, double slope, int rule, Tents& out, int64_t work_limit) {
  const int d = m.d, nvert = d + 1;
  const double Q = std::ldexp(1.0, -24);
  const double SAFETY = 1e-3;
  const double POLE_CAP = 1.5;   // colour rule: pole height <= 1.5 min_w k_vw
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
  std::vector<int32_t> V, L;
  std::vector<double> TB, TT;
  // target of vertex v and its layer; emits the tent if the target lies above tau_v
  auto target = [&](int32_t v, int32_t& lay) {
    double t_plus = 1e300;
    lay = last[v];
    for (int64_t i = m.adj_ptr[v]; i < m.adj_ptr[v + 1]; ++i) {
      int32_t w = m.adj[i];
      t_plus = std::min(t_plus, tau[w] + kvw[i]);
      lay = std::max(lay, last[w]);
    }
    lay += 1;
    return std::min(t_end, Q * std::floor(t_plus / Q - SAFETY));
  };
  int64_t work = 0;   // sum of the emitted tents' patch sizes
  auto emit = [&](int32_t v, double t_new, int32_t lay) {
    work += m.v2e_ptr[v + 1] - m.v2e_ptr[v];
    last[v] = lay;
    V.push_back(v);
    TB.push_back(tau[v]);
    TT.push_back(t_new);
    L.push_back(lay);
    tau[v] = t_new;
  };
  if (rule == MTP_PITCH_MIN_VERTEX) {
    using Item = std::pair<double, int32_t>;
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
    for (int64_t v = 0; v < m.nv; ++v) heap.push({0.0, (int32_t)v});
    while (!heap.empty()) {
      auto [tv, v] = heap.top();
      heap.pop();
      if (tv >= t_end) continue;
      int32_t lay;
      double t_new = target(v, lay);
      if (!(t_new > tv)) throw Error(MTP_ERR_PITCH, "vertex " + std::to_string(v) + " cannot advance");
      emit(v, t_new, lay);
      if (t_new < t_end) heap.push({t_new, v});
    }
  } else if (rule == MTP_PITCH_COLOUR) {
    std::vector<int32_t> col;
    const int32_t n_col = colour_vertices(m, col);
    std::vector<int64_t> cls_ptr(n_col + 1, 0);
    std::vector<int32_t> cls(m.nv);
    for (int64_t v = 0; v < m.nv; ++v) cls_ptr[col[v] + 1]++;
    for (int32_t c = 0; c < n_col; ++c) cls_ptr[c + 1] += cls_ptr[c];
    {
      std::vector<int64_t> fill(cls_ptr.begin(), cls_ptr.end() - 1);
      for (int64_t v = 0; v < m.nv; ++v) cls[fill[col[v]]++] = (int32_t)v;   // ids ascending per colour
    }
    // pole cap per vertex, tau_v + 1.5 min_w k_vw, each operation rounded on its own (no
    // contraction into a fused multiply-add)
    std::vector<double> kcap(m.nv, 1e300);
    for (int64_t v = 0; v < m.nv; ++v) {
      double k = 1e300;
      for (int64_t i = m.adj_ptr[v]; i < m.adj_ptr[v + 1]; ++i) k = std::min(k, kvw[i]);
      kcap[v] = POLE_CAP * k;
    }
    auto capped = [&](int32_t v, double t_new) {
#pragma clang fp contract(off)
      const double cap = tau[v] + kcap[v];
      return std::min(t_new, std::min(t_end, Q * std::floor(cap / Q - SAFETY)));
    };
    int64_t below = m.nv;   // vertices still below t_end
    int32_t idle = 0;       // consecutive turns without a move
    for (int32_t c = 0; below > 0; c = (c + 1) % n_col) {
      bool moved = false;
      for (int64_t i = cls_ptr[c]; i < cls_ptr[c + 1]; ++i) {
        int32_t v = cls[i], lay;
        if (tau[v] >= t_end) continue;
        const double t_new = capped(v, target(v, lay));
        if (!(t_new > tau[v])) continue;
        emit(v, t_new, lay);
        moved = true;
        if (t_new >= t_end) --below;
        if (work >= work_limit) return false;   // no less work than the limit: give up
      }
      idle = moved ? 0 : idle + 1;
      if (idle > n_col) throw Error(MTP_ERR_PITCH, "colour pitching made no progress");
    }
  } else {
    throw Error(MTP_ERR_ARG, "unknown pitching rule " + std::to_string(rule));
  }

  // sort by layer, stable in pitching order
  const size_t nt = V.size();
  std::vector<size_t> idx(nt);
  for (size_t i = 0; i < nt; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return L[a] < L[b]; });
  out.t_end = t_end;
  out.slope = slope;
  out.rule = rule;
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
  return true;
}

}  // namespace mtp
