// Tent dependency graph of one slab (section 2: a tent may be pitched, and evolved, once
// the tents it depends on are done).  Tent t at vertex V reads and writes the elements of
// the vertex patch of V and reads the front time of every vertex of those elements, i.e.
// of V and its neighbours.  Its predecessors are therefore the latest earlier tent at V
// and at each neighbour of V.  With the tents sorted by layer (a tent's layer exceeds the
// layers of those tents, and tents of one layer share no vertex or neighbour), a scan in
// table order that remembers the last tent per vertex finds exactly these predecessors.
#include <algorithm>

#include "internal.h"

namespace mtp {

void tent_dag(const Mesh& m, const Tents& t, std::vector<int32_t>& pred_count, std::vector<int32_t>& succ_ptr,
              std::vector<int32_t>& succ, int32_t& nready) {
  const int64_t n = (int64_t)t.vertex.size();
  std::vector<int32_t> last(m.nv, -1);
  std::vector<int32_t> pred_ptr(n + 1, 0), pred;
  pred.reserve(n * 8);
  pred_count.assign(n, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t V = t.vertex[i];
    auto add = [&](int32_t u) {
      if (last[u] >= 0) pred.push_back(last[u]);
    };
    add(V);
    for (int64_t k = m.adj_ptr[V]; k < m.adj_ptr[V + 1]; ++k) add(m.adj[k]);
    pred_ptr[i + 1] = (int32_t)pred.size();
    pred_count[i] = pred_ptr[i + 1] - pred_ptr[i];
    last[V] = (int32_t)i;
  }
  // successors: the transpose of the predecessor lists (CSR, successors in table order)
  succ_ptr.assign(n + 1, 0);
  for (int32_t p : pred) succ_ptr[p + 1]++;
  for (int64_t i = 0; i < n; ++i) succ_ptr[i + 1] += succ_ptr[i];
  succ.assign(pred.size(), 0);
  std::vector<int32_t> fill(succ_ptr.begin(), succ_ptr.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t k = pred_ptr[i]; k < pred_ptr[i + 1]; ++k) succ[fill[pred[k]]++] = (int32_t)i;
  // the tents without predecessor are exactly the first layer, i.e. a prefix of the table
  nready = 0;
  while (nready < n && pred_count[nready] == 0) ++nready;
  for (int64_t i = nready; i < n; ++i)
    if (pred_count[i] == 0) throw Error(MTP_ERR_PITCH, "tent without predecessor outside the first layer");
}

int64_t tent_dag_edges(const Mesh& m, const Tents& t) {
  std::vector<char> seen(m.nv, 0);
  int64_t e = 0;
  for (int32_t V : t.vertex) {
    if (seen[V]) ++e;
    for (int64_t k = m.adj_ptr[V]; k < m.adj_ptr[V + 1]; ++k) e += seen[m.adj[k]];
    seen[V] = 1;
  }
  return e;
}

}  // namespace mtp
