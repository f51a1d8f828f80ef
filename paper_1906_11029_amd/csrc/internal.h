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
  // quadratic (curved) triangles, 2D only: geo = ne*6*2 geometry nodes (vertices in cell
  // order, then the midpoints of edges (0,1), (1,2), (0,2)); curved[e] != 0 where a
  // midpoint node is not the straight midpoint.  Empty for an all-affine mesh.
  std::vector<double> geo;
  std::vector<uint8_t> curved;
  int64_t n_curved = 0;
};

// Tents sorted by layer (stable in pitching order).
struct Tents {
  double t_start = 0.0;             // front time the table starts from (times below are relative to it)
  double t_end = 0.0;               // slab height: the table runs from relative time 0 to t_end
  double slope = 0.5;
  int rule = 0;                     // MTP_PITCH_*
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
void pitch(const Mesh& m, double t_end, double slope, int rule, Tents& out);
// one ordering; the colour rule gives up (returns false, out untouched) once the sum of its
// tents' patch sizes reaches work_limit
bool pitch_rule(const Mesh& m, double t_end, double slope, int rule, Tents& out,
                int64_t work_limit = INT64_MAX);
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

// curved quadratic triangles (curved.cpp)
void set_curved_p2(Mesh& m, const double* nodes);            // validates; throws Error
double curved_step(const Mesh& m, int64_t e, double slope);  // pitcher step of a curved element
void curved_node(const Mesh& m, int64_t e, const double* xh, double* x);   // x = map_e(xh)

// The curved-element tent path of one solver: which tents run on it (those whose patch
// holds a curved element), the zone of elements their patches cover, and the tables its
// kernel reads (quadrature rules, reference basis at the points, per zone element the
// geometry at the points and the weight-adjusted inverse mass).
struct CurvedPlan {
  int p = 0, np = 0, nq = 0, nfq = 0;      // nq = (p + 4)^2 volume points, nfq = p + 4 face points
  std::vector<uint8_t> tent_curved;        // per tent of the table
  std::vector<int32_t> zone;               // ne: zone index or -1
  std::vector<int32_t> zone_elem;          // nz: element of each zone index
  int max_patch = 0;                       // largest patch of a curved tent
  // table sizes (doubles / ints)
  size_t n_ref() const { return (size_t)nq * np * 3 + (size_t)nq * 3 + 3 * (size_t)nfq * (np + 3); }
  size_t n_geo() const { return zone_elem.size() * ((size_t)nq * 5 + (size_t)np * np + 3 * (size_t)nfq * 3); }
};
CurvedPlan curved_plan(const Mesh& m, const Tents& t, int p);
// ref: V[q][a], Gr[q][a][l], Lam[q][k], then per face f: Vf[f][q][a], Lamf[f][q][k];
// geo per zone element z: Q[z][q][5] (w |det J|, J^{-1}[l][r]), Minv[z][a][b], F[z][f][q][3]
// (w |dx/ds|, outward unit normal); nbr per zone element and face: neighbour element or
// -1 - boundary kind, and (neighbour face | reversed << 2)
void curved_tables(const Mesh& m, const CurvedPlan& cp, const std::vector<int32_t>& mi, std::vector<double>& ref,
                   std::vector<double>& geo, std::vector<int32_t>& nbr);

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
