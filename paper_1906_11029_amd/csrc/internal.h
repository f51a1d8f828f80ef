// Internal host-side structures of the MTP library (not part of the C interface).
#pragma once
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/mtp.h"

namespace mtp {

struct Error : std::runtime_error {
  mtp_status code;
  Error(mtp_status c, const std::string& msg) : std::runtime_error(msg), code(c) {}
};

// Conforming simplicial mesh with the topology the tents need.
struct Mesh {
  int d = 0;
  int64_t nv = 0, ne = 0;
  std::vector<double> coords;    // nv*d
  std::vector<int32_t> cells;    // ne*(d+1)
  std::vector<double> eps, mu;   // ne (acoustics: kappa, rho)
  int system = 0;                // MTP_SYSTEM_MAXWELL or MTP_SYSTEM_ACOUSTIC
  std::vector<int32_t> face_bc;  // ne*(d+1)
  std::vector<int32_t> nbr;      // ne*(d+1): neighbour across local face j, -1 on boundary
  std::vector<int8_t> nbr_face;  // ne*(d+1): local face index of this face in the neighbour
  std::vector<double> grad_lam;  // ne*(d+1)*d: gradients of the barycentric coordinates
  std::vector<double> volume;    // ne
  std::vector<int64_t> v2e_ptr;  // nv+1 : vertex patch (elements containing the vertex)
  std::vector<int32_t> v2e;      //        element ids
  std::vector<int8_t> v2e_k;     //        local index of the vertex in that element
  std::vector<int64_t> adj_ptr;  // nv+1 : vertex neighbours
  std::vector<int32_t> adj;
  int max_patch = 0;
};

// Tents sorted by layer (stable in pitching order).
struct Tents {
  double t_start = 0.0;             // front time the table starts from (times below are relative to it)
  double t_end = 0.0;               // slab height: the table runs from relative time 0 to t_end
  double slope = 0.5;
  std::vector<int32_t> vertex;
  std::vector<double> t_bot, t_top;
  std::vector<int32_t> layer;
  std::vector<int64_t> layer_ptr;   // n_layers + 1
};

// Reference-element tables for nodal DG of degree p on the d-simplex, with the tent
// vertex renumbered to local vertex 0.
struct RefElem {
  int d = 0, p = 0, np = 0, nf = 0;
  std::vector<int> mi;        // np*(d+1): barycentric multi-index of every node
  std::vector<double> S;      // d*np*np : S_l = Mhat^{-1} D_l, stored [l][a][b] (b = test)
  std::vector<double> L;      // d*nf*np : L_j = Mhat^{-1} E_j, stored [j][s][b]
  std::vector<int> fnode;     // d*2*nf  : volume node of face node s, [j][o][s]
  std::vector<int> fswap;     // nf: face node with the two non-V face vertices exchanged
  std::vector<int> perm;      // (d+1)*np: node of the original numbering for each node
                              //           of the numbering with vertex k moved to 0
  std::vector<double> Mhat;   // np*np reference mass (for tests / diagnostics)
};

RefElem build_refelem(int d, int p);
// order of the original local vertices after moving vertex k to position 0
void vertex_order(int d, int k, int* order);

void build_topology(Mesh& m);
void pitch(const Mesh& m, double t_end, double slope, Tents& out);
// dependency graph of the tents (table order): predecessor counts, successors (CSR) and the
// number of leading tents without predecessor
void tent_dag(const Mesh& m, const Tents& t, std::vector<int32_t>& pred_count, std::vector<int32_t>& succ_ptr,
              std::vector<int32_t>& succ, int32_t& nready);
int64_t tent_dag_edges(const Mesh& m, const Tents& t);

// allocation-free advance (capi.cpp): the thread's error message, the solver's device, and
// mtp_advance_to on the persistent schedule with its scratch at a given device address
void set_last_error(const char* msg);
int solver_device(mtp_solver s);
void advance_to_dag_scratch(mtp_solver s, double T, char* d_scratch, size_t cap);

// tuning table (tune.cpp): launch choices by configuration key
struct TuneEntry {
  int schedule = 0, tile_order = 0;
  double grid_frac = 1.0;
  double ms_best = 0.0, ms_default = 0.0;
  int candidates = 0;
};
bool tune_find(const std::string& key, TuneEntry* out);
void tune_put(const std::string& key, const TuneEntry& e);
void tune_clear_all();
int tune_count();
void tune_save_file(const char* path);   // throws Error
void tune_load_file(const char* path);   // throws Error; merges

}  // namespace mtp
