// C interface (include/mtp.h): mesh, pitching, solver set-up, layer sweep, read-out.
// Every entry point converts exceptions into an mtp_status and a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"

struct mtp_mesh_s { mtp::Mesh m; };
struct mtp_tents_s { mtp::Tents t; };

namespace mtp {

static thread_local std::string g_last_error;

static void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(MTP_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Device workspace layout: every array 256-byte aligned.
struct Layout {
  size_t off = 0;
  size_t add(size_t bytes) {
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  }
};

struct Offsets {
  size_t W, tau, stage, grad_lam, cells, eps, mu, coords, pptr, pelem, pinfo, fptr, face, tv, tt, S, L,
      fnode, fswap, perm, mi, err, slab, dag_indeg, dag_indeg0, dag_sptr, dag_succ, dag_queue, dag_ctl,
      cref, cgeo, cnbr, czone, opg, frg, total;
};

// opg_bytes: the matrix-core kernel's operator block when it stays in device memory (0 if not);
// frg_bytes: the F/R slots of the extra-large patch class (0 if not)
static Offsets plan(const Mesh& m, const Tents& t, const RefElem& R, int nc, size_t opg_bytes, size_t frg_bytes) {
  Layout L;
  Offsets o;
  const int d = m.d;
  const size_t ptot = m.v2e.size();
  o.W = L.add(sizeof(double) * m.ne * nc * R.np);
  o.tau = L.add(sizeof(double) * m.nv);
  o.stage = L.add(sizeof(double) * m.ne * nc * R.np);
  o.grad_lam = L.add(sizeof(double) * m.ne * (d + 1) * d);
  o.cells = L.add(sizeof(int32_t) * m.ne * (d + 1));
  o.eps = L.add(sizeof(double) * m.ne);
  o.mu = L.add(sizeof(double) * m.ne);
  o.coords = L.add(sizeof(double) * m.nv * d);
  o.pptr = L.add(sizeof(int32_t) * (m.nv + 1));
  o.pelem = L.add(sizeof(int32_t) * ptot);
  o.pinfo = L.add(sizeof(int32_t) * ptot * (1 + d));
  o.fptr = L.add(sizeof(int32_t) * (m.nv + 1));
  o.face = L.add(sizeof(int32_t) * ptot * d);
  o.tv = L.add(sizeof(int32_t) * std::max<size_t>(1, t.vertex.size()));
  o.tt = L.add(sizeof(double) * std::max<size_t>(1, t.vertex.size()));
  o.S = L.add(sizeof(double) * R.S.size());
  o.L = L.add(sizeof(double) * R.L.size());
  o.fnode = L.add(sizeof(int32_t) * R.fnode.size());
  o.fswap = L.add(sizeof(int32_t) * R.fswap.size());
  o.perm = L.add(sizeof(int32_t) * R.perm.size());
  o.mi = L.add(sizeof(int32_t) * R.mi.size());
  o.err = L.add(sizeof(int32_t) * 4);
  o.slab = L.add(sizeof(double) * 4);
  const size_t nt = std::max<size_t>(1, t.vertex.size());
  o.dag_indeg = L.add(sizeof(int32_t) * nt);
  o.dag_indeg0 = L.add(sizeof(int32_t) * nt);
  o.dag_sptr = L.add(sizeof(int32_t) * (nt + 1));
  o.dag_succ = L.add(sizeof(int32_t) * std::max<int64_t>(1, tent_dag_edges(m, t)));
  o.dag_queue = L.add(sizeof(int32_t) * nt);
  o.dag_ctl = L.add(sizeof(int32_t) * 4);
  // curved-element tent path (empty for an all-affine mesh)
  const CurvedPlan cp = curved_plan(m, t, R.p);
  const bool cur = !cp.zone_elem.empty();
  o.cref = L.add(cur ? sizeof(double) * cp.n_ref() : 0);
  o.cgeo = L.add(cur ? sizeof(double) * cp.n_geo() : 0);
  o.cnbr = L.add(cur ? sizeof(int32_t) * cp.zone_elem.size() * 6 : 0);
  o.czone = L.add(cur ? sizeof(int32_t) * m.ne : 0);
  o.opg = L.add(opg_bytes);
  o.frg = L.add(frg_bytes);
  o.total = L.off;
  return o;
}

// Static per-vertex patch tables: for every element of the patch of V, the local index
// k of V and, for each face j (1..d) of the element renumbered with V first, the
// patch-local neighbour, its face index in its own renumbering and the relative
// orientation of the two faces' vertex orders (3D), or -1 - boundary kind.
static void patch_tables(const Mesh& m, std::vector<int32_t>& ptr, std::vector<int32_t>& elem,
                         std::vector<int32_t>& info) {
  const int d = m.d, nv = d + 1;
  ptr.assign(m.nv + 1, 0);
  elem.assign(m.v2e.size(), 0);
  info.assign(m.v2e.size() * (1 + d), 0);
  for (int64_t v = 0; v <= m.nv; ++v) ptr[v] = (int32_t)m.v2e_ptr[v];
  for (int64_t V = 0; V < m.nv; ++V) {
    const int64_t b0 = m.v2e_ptr[V], b1 = m.v2e_ptr[V + 1];
    for (int64_t i = b0; i < b1; ++i) {
      const int32_t e = m.v2e[i];
      const int k = m.v2e_k[i];
      elem[i] = e;
      int32_t* inf = &info[i * (1 + d)];
      inf[0] = k;
      int order[4];
      vertex_order(d, k, order);
      for (int jn = 1; jn <= d; ++jn) {
        const int f = order[jn];  // original local face index
        const int32_t e2 = m.nbr[e * nv + f];
        if (e2 < 0) {
          inf[jn] = -1 - m.face_bc[e * nv + f];
          continue;
        }
        int64_t pos = -1;
        for (int64_t q = b0; q < b1; ++q)
          if (m.v2e[q] == e2) { pos = q - b0; break; }
        if (pos < 0) throw Error(MTP_ERR_MESH, "face neighbour outside the vertex patch");
        const int k2 = m.v2e_k[b0 + pos];
        int order2[4];
        vertex_order(d, k2, order2);
        const int f2 = m.nbr_face[e * nv + f];
        int j2 = -1;
        for (int q = 1; q <= d; ++q)
          if (order2[q] == f2) j2 = q;
        if (j2 < 1) throw Error(MTP_ERR_MESH, "inconsistent face neighbour");
        int o = 0;
        if (d == 3) {
          // the face's two vertices other than V, in e's renumbered order
          int fv[2], c = 0;
          for (int q = 1; q <= 3; ++q)
            if (q != jn) fv[c++] = m.cells[e * nv + order[q]];
          // their positions in e2's renumbered order
          int p0 = -1, p1 = -1;
          for (int q = 1; q <= 3; ++q) {
            int g = m.cells[e2 * nv + order2[q]];
            if (g == fv[0]) p0 = q;
            if (g == fv[1]) p1 = q;
          }
          if (p0 < 0 || p1 < 0) throw Error(MTP_ERR_MESH, "face vertices do not match");
          o = (p0 < p1) ? 0 : 1;
        }
        inf[jn] = (int32_t)((pos << 4) | (j2 << 1) | o);
      }
    }
  }
}

// Owned faces per vertex patch, from the patch info codes: each interior face once (by
// the lower patch index of its two elements), each boundary face by its element.
static void patch_faces(const Mesh& m, const std::vector<int32_t>& info, std::vector<int32_t>& ptr,
                        std::vector<int32_t>& faces) {
  const int d = m.d;
  ptr.assign(m.nv + 1, 0);
  faces.clear();
  for (int64_t V = 0; V < m.nv; ++V) {
    const int64_t b0 = m.v2e_ptr[V], b1 = m.v2e_ptr[V + 1];
    for (int64_t i = b0; i < b1; ++i) {
      const int e = (int)(i - b0);
      for (int j = 1; j <= d; ++j) {
        const int32_t code = info[i * (1 + d) + j];
        if (code < 0 || (code >> 4) > e) faces.push_back((e << 2) | (j - 1));
      }
    }
    ptr[V + 1] = (int32_t)faces.size();
  }
}

}  // namespace mtp

struct mtp_solver_s {
  mtp::Mesh mesh;
  mtp::Tents tents;
  mtp::RefElem ref;
  mtp::Offsets off;
  mtp::KernelParams kp;
  int p = 0, q = 0, m = 0, nc = 0;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int64_t slab = 0;          // completed slabs
  int64_t layers_done = 0;   // layers done in the current slab
  double t_base = 0.0;       // front time at the start of slab 0
  bool has_data_faces = false;
  int kernel = 0;            // 0 vector-ALU FP64, 1 matrix-core FP64, 2 matrix-core FP32
  int schedule = MTP_SCHEDULE_LAYERS;
  int method = MTP_METHOD_SAT;
  int device = 0;            // HIP device current at creation (the workspace's)
  // tuned launch choices (results do not depend on them): persistent grid as a fraction of
  // the resident maximum dag_grid_max, tile assignment in kp.tile_order, schedule above
  int dag_grid_max = 0;
  double grid_frac = 1.0;
  bool tuned_from_table = false;
  // curved-element path: within each layer the affine tents come first (layer_na of them),
  // then the tents whose patch holds a curved element
  bool curved = false;
  std::vector<int64_t> layer_na;
  mtp::CurvedParams cparams{};
  // a layer's curved tents run on a side stream beside its affine tents (disjoint patches),
  // forked from and joined back into the layer's stream by two events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // one slab (slab begin, every layer or the persistent DAG launch, slab end) captured once
  // and replayed per slab
  bool use_graph = true;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
};

struct mtp_batch_s {
  // Solvers of one degree run together: the batch keeps its kernel parameters sorted by
  // degree (internal index j holds solver order[j]), so each degree group is a contiguous
  // range [s0, s1) served by the single-degree kernels.
  struct Group {
    int p = 0, max_patch = 0, s0 = 0, s1 = 0;
    int grid_max = 0;             // resident maximum of the group's persistent kernel
    mtp::BatchDag bd{};           // persistent schedule over the group's tent DAGs
    double* opg = nullptr;        // the group's operator block in device memory (classes that
                                  // keep it there), staged by the batch; null otherwise
  };
  struct Launch {                 // one layer of one degree group
    int64_t seg0 = 0, blocks = 0;
    int nseg = 0, group = 0;
  };
  std::vector<mtp_solver> solvers;   // in the caller's order
  std::vector<int> order;
  std::vector<Group> groups;
  std::vector<Launch> launches;
  int kernel = 0, d = 0, system = 0, method = 0;
  double* frg = nullptr;          // F/R slots of the 48-tet class (kFrgSlots of them), or null
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  mtp::KernelParams* d_kps = nullptr;
  mtp::BatchSeg* d_segs = nullptr;
  std::vector<mtp::KernelParams> h_kps;
  int schedule = MTP_SCHEDULE_LAYERS;
  int tile_order = 0;             // tuned tile assignment of every solver's tents in the batch
  double grid_frac = 1.0;         // tuned persistent grid, fraction of each group's maximum
  bool tuned_from_table = false;
  bool dag_ok = true;             // every group's persistent kernel can be resident
  bool use_graph = true;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
};

using namespace mtp;

#define MTP_TRY try {
#define MTP_CATCH                                        \
  }                                                      \
  catch (const mtp::Error& e) {                          \
    g_last_error = e.what();                             \
    return e.code;                                       \
  }                                                      \
  catch (const std::bad_alloc& e) {                      \
    g_last_error = "host memory exhausted";              \
    return MTP_ERR_NOMEM;                                \
  }                                                      \
  catch (const std::exception& e) {                      \
    g_last_error = e.what();                             \
    return MTP_ERR_ARG;                                  \
  }                                                      \
  return MTP_OK;

static void check_status(mtp_status st) {
  if (st != MTP_OK) throw Error(st, g_last_error);
}

static void require(bool c, mtp_status code, const char* msg) {
  if (!c) throw Error(code, msg);
}

extern "C" {

const char* mtp_last_error(void) { return g_last_error.c_str(); }

mtp_status mtp_mesh_create(int32_t dim, int64_t nv, const double* coords, int64_t ne, const int32_t* cells,
                           const double* eps, const double* mu, const int32_t* face_bc, mtp_mesh* out) {
  MTP_TRY
  require(out && coords && cells, MTP_ERR_ARG, "null pointer");
  require(dim == 2 || dim == 3, MTP_ERR_ARG, "dim must be 2 or 3");
  require(nv > 0 && ne > 0 && nv < (1LL << 31) && ne < (1LL << 31), MTP_ERR_ARG, "bad sizes");
  auto* h = new mtp_mesh_s();
  try {
    Mesh& m = h->m;
    m.d = dim;
    m.nv = nv;
    m.ne = ne;
    m.coords.assign(coords, coords + nv * dim);
    m.cells.assign(cells, cells + ne * (dim + 1));
    m.eps = eps ? std::vector<double>(eps, eps + ne) : std::vector<double>(ne, 1.0);
    m.mu = mu ? std::vector<double>(mu, mu + ne) : std::vector<double>(ne, 1.0);
    m.face_bc = face_bc ? std::vector<int32_t>(face_bc, face_bc + ne * (dim + 1))
                        : std::vector<int32_t>(ne * (dim + 1), MTP_BC_PEC);
    for (double c : m.coords) require(std::isfinite(c), MTP_ERR_MESH, "non-finite coordinate");
    build_topology(m);
  } catch (...) {
    delete h;
    throw;
  }
  *out = h;
  MTP_CATCH
}

mtp_status mtp_mesh_set_curved_p2(mtp_mesh mesh, const double* nodes) {
  MTP_TRY
  require(mesh && nodes, MTP_ERR_ARG, "null pointer");
  set_curved_p2(mesh->m, nodes);
  MTP_CATCH
}

mtp_status mtp_mesh_set_system(mtp_mesh mesh, int32_t system) {
  MTP_TRY
  require(mesh, MTP_ERR_ARG, "null mesh");
  require(system == MTP_SYSTEM_MAXWELL || system == MTP_SYSTEM_ACOUSTIC, MTP_ERR_ARG, "unknown system");
  mesh->m.system = system;
  MTP_CATCH
}

mtp_status mtp_mesh_info(mtp_mesh mesh, int32_t* dim, int64_t* nv, int64_t* ne, int32_t* max_patch) {
  MTP_TRY
  require(mesh, MTP_ERR_ARG, "null mesh");
  if (dim) *dim = mesh->m.d;
  if (nv) *nv = mesh->m.nv;
  if (ne) *ne = mesh->m.ne;
  if (max_patch) *max_patch = mesh->m.max_patch;
  MTP_CATCH
}

void mtp_mesh_destroy(mtp_mesh mesh) { delete mesh; }

mtp_status mtp_pitch_layers(mtp_mesh mesh, double t_start, double t_end, double slope_fraction, mtp_tents* out) {
  return mtp_pitch_layers_rule(mesh, t_start, t_end, slope_fraction, MTP_PITCH_MIN_VERTEX, out);
}

mtp_status mtp_pitch_layers_rule(mtp_mesh mesh, double t_start, double t_end, double slope_fraction, int32_t rule,
                                 mtp_tents* out) {
  MTP_TRY
  require(mesh && out, MTP_ERR_ARG, "null pointer");
  require(std::isfinite(t_start) && std::isfinite(t_end) && t_end > t_start, MTP_ERR_ARG,
          "need finite t_start < t_end");
  require(slope_fraction > 0 && slope_fraction < 1, MTP_ERR_CAUSALITY, "slope fraction must be in (0,1)");
  require(rule == MTP_PITCH_MIN_VERTEX || rule == MTP_PITCH_COLOUR || rule == MTP_PITCH_AUTO, MTP_ERR_ARG,
          "unknown pitching rule");
  auto* h = new mtp_tents_s();
  try {
    // times relative to t_start: the table is a slab pattern that solvers apply from their
    // current flat front, and one table serves every slab bit for bit
    pitch(mesh->m, t_end - t_start, slope_fraction, rule, h->t);
    h->t.t_start = t_start;
  } catch (...) {
    delete h;
    throw;
  }
  *out = h;
  MTP_CATCH
}

mtp_status mtp_tents_rule(mtp_tents tents, int32_t* rule) {
  MTP_TRY
  require(tents && rule, MTP_ERR_ARG, "null pointer");
  *rule = tents->t.rule;
  MTP_CATCH
}

mtp_status mtp_tents_query(mtp_tents tents, int64_t* n_tents, int64_t* n_layers, int64_t* layer_ptr) {
  MTP_TRY
  require(tents, MTP_ERR_ARG, "null tents");
  const Tents& t = tents->t;
  if (n_tents) *n_tents = (int64_t)t.vertex.size();
  if (n_layers) *n_layers = (int64_t)t.layer_ptr.size() - 1;
  if (layer_ptr) std::copy(t.layer_ptr.begin(), t.layer_ptr.end(), layer_ptr);
  MTP_CATCH
}

mtp_status mtp_tents_export(mtp_tents tents, int32_t* vertex, double* t_bot, double* t_top, int32_t* layer) {
  MTP_TRY
  require(tents, MTP_ERR_ARG, "null tents");
  const Tents& t = tents->t;
  if (vertex) std::copy(t.vertex.begin(), t.vertex.end(), vertex);
  if (t_bot) for (size_t i = 0; i < t.t_bot.size(); ++i) t_bot[i] = t.t_start + t.t_bot[i];
  if (t_top) for (size_t i = 0; i < t.t_top.size(); ++i) t_top[i] = t.t_start + t.t_top[i];
  if (layer) std::copy(t.layer.begin(), t.layer.end(), layer);
  MTP_CATCH
}

void mtp_tents_destroy(mtp_tents tents) { delete tents; }

// field components of the mesh's system
static int ncomp(const Mesh& m) { return m.system == MTP_SYSTEM_ACOUSTIC ? m.d + 1 : (m.d == 3 ? 6 : 3); }

// Kernel choice: 0 = vector-ALU FP64, 1 = matrix-core FP64, 2 = matrix-core FP32 (mixed).
static int check_config(const Mesh& m, int p, int q, int mm, int precision) {
  require(precision != MTP_BF16X3, MTP_ERR_UNSUPPORTED, "split-BF16 contractions are not built");
  require(precision == MTP_FP64 || precision == MTP_MIXED_FP32 || precision == MTP_FP64_VALU,
          MTP_ERR_UNSUPPORTED, "unknown precision");
  require(q >= 1 && q <= 32 && mm >= 1 && mm <= 1024, MTP_ERR_ARG, "q must be in 1..32 and m in 1..1024");
  // P5 in 3D runs on the matrix-core kernels only
  const bool mfma_only = m.d == 3 && p == 5;
  require(tent_kernel_supported(m.d, p) || mfma_only, MTP_ERR_UNSUPPORTED, "degree p not covered for this dimension");
  require(!(mfma_only && precision == MTP_FP64_VALU), MTP_ERR_UNSUPPORTED,
          "the vector-ALU kernel covers p <= 4 in 3D");
  const size_t lim = 160 * 1024;
  if (m.n_curved > 0) {
    require(m.d == 2 && m.system == MTP_SYSTEM_MAXWELL, MTP_ERR_UNSUPPORTED, "curved elements: 2D Maxwell only");
    require(p >= 1 && p <= 4, MTP_ERR_UNSUPPORTED, "curved elements: degrees 1..4");
    // the curved tents run in FP64 (their own kernel); the layer's other tents in the precision asked
    require(precision == MTP_FP64 || precision == MTP_FP64_VALU || precision == MTP_MIXED_FP32,
            MTP_ERR_UNSUPPORTED, "curved elements: FP64 or mixed (split-BF16 is not built)");
    require(tent_curved_lds_bytes(p, m.max_patch, false) <= lim, MTP_ERR_UNSUPPORTED,
            "largest vertex patch does not fit the curved-element kernel's LDS");
    for (int64_t e = 0; e < m.ne; ++e)
      for (int f = 0; f < 3; ++f) {
        bool near = false;   // a data face of an element that shares a vertex with a curved one
        for (int v = 0; v < 3 && !near; ++v) {
          const int32_t V = m.cells[e * 3 + v];
          for (int64_t k = m.v2e_ptr[V]; k < m.v2e_ptr[V + 1]; ++k) near = near || m.curved[m.v2e[k]];
        }
        require(!(near && m.nbr[e * 3 + f] < 0 && m.face_bc[e * 3 + f] == MTP_BC_DATA), MTP_ERR_UNSUPPORTED,
                "curved elements: walls only (no data faces next to a curved element)");
      }
  }
  const size_t lds_valu = tent_kernel_lds_bytes(m.d, p, m.max_patch);
  const int np = (m.d == 2) ? (p + 1) * (p + 2) / 2 : (p + 1) * (p + 2) * (p + 3) / 6;
  const int block = (m.d == 2) ? 128 : 256;
  const bool valu_ok = lds_valu <= lim && m.max_patch * np <= block * 8;
  if (m.system == MTP_SYSTEM_ACOUSTIC) {
    require(precision != MTP_FP64_VALU, MTP_ERR_UNSUPPORTED, "acoustics runs on the matrix-core kernels");
    require(tent_mfma_lds_bytes(m.d, p, m.max_patch, precision == MTP_MIXED_FP32, 1) <= lim, MTP_ERR_UNSUPPORTED,
            "largest vertex patch does not fit the matrix-core kernel's LDS");
    return precision == MTP_MIXED_FP32 ? 2 : 1;
  }
  if (precision == MTP_MIXED_FP32) {
    require(tent_mfma_lds_bytes(m.d, p, m.max_patch, 1) <= lim, MTP_ERR_UNSUPPORTED,
            "largest vertex patch does not fit the matrix-core kernel's LDS");
    return 2;
  }
  if (precision == MTP_FP64 && tent_mfma_lds_bytes(m.d, p, m.max_patch, 0) <= lim) return 1;
  require(valu_ok && !mfma_only, MTP_ERR_UNSUPPORTED, "largest vertex patch does not fit the 160 KiB of LDS");
  return 0;
}

// Bytes of the operator block that the solver's matrix-core kernel keeps in device memory
// (P4 patches of more than 24 tets), 0 when the kernel stages it in LDS.
static size_t opg_bytes(const Mesh& m, int p, int kernel) {
  return kernel == 0 ? 0 : tent_mfma_opg_bytes(m.d, p, m.max_patch, kernel == 2, m.system);
}

// P4 patches of 37-48 tets in 3D keep the tent's F/R in device memory, one slot per
// workgroup: kFrgSlots slots (four per compute unit of the largest device; the launches cap
// their grid at it), about 104 KB each.
static constexpr int kFrgSlots = 1024;
static size_t frg_bytes(const Mesh& m, int p, int kernel) {
  return kernel == 0 ? 0 : tent_mfma_frg_bytes(m.d, p, m.max_patch, kernel == 2, m.system) * kFrgSlots;
}

mtp_status mtp_solver_workspace_size(mtp_mesh mesh, mtp_tents tents, int32_t p, int32_t q, int32_t m,
                                     int32_t precision, size_t* bytes) {
  MTP_TRY
  require(mesh && tents && bytes, MTP_ERR_ARG, "null pointer");
  const int kernel = check_config(mesh->m, p, q, m, precision);
  RefElem R = build_refelem(mesh->m.d, p);
  *bytes = plan(mesh->m, tents->t, R, ncomp(mesh->m), opg_bytes(mesh->m, p, kernel), frg_bytes(mesh->m, p, kernel)).total;
  MTP_CATCH
}

// ------------------------------------------------------------------ tuning keys and choices
// "<arch>x<compute units>" of a device, e.g. gfx950x256
static std::string device_tag(int dev) {
  hipDeviceProp_t pr;
  check_hip(hipGetDeviceProperties(&pr, dev), "device properties");
  std::string arch = pr.gcnArchName;
  const size_t c = arch.find(':');
  if (c != std::string::npos) arch.resize(c);
  return arch + "x" + std::to_string(pr.multiProcessorCount);
}
static int patch_class(int d, int p, int max_patch) {
  return max_patch <= 8 ? 8 : max_patch <= 24 ? 24 : (d == 3 && p == 4 && max_patch <= 36) ? 36 : 48;
}
static int log2_class(int64_t n) {
  int c = 0;
  while (c < 62 && ((int64_t)1 << (c + 1)) <= n) ++c;
  return c;
}
// tents per slab in factors of 4 (a slab's tent count moves with the materials and the
// mesh grading; the launch choice does not change within such a band)
static int tents_class(int64_t n) { return log2_class(n) / 2; }
static std::string solver_key(mtp_solver s) {
  return "solver|" + device_tag(s->device) + "|d" + std::to_string(s->mesh.d) + "|sys" +
         std::to_string(s->mesh.system) + "|p" + std::to_string(s->p) + "|k" + std::to_string(s->kernel) + "|m" +
         std::to_string(s->method) + "|nt" + std::to_string(patch_class(s->mesh.d, s->p, s->mesh.max_patch)) + "|t" +
         std::to_string(tents_class((int64_t)s->tents.vertex.size()));
}
static void drop_graph(mtp_solver s);
static void release_side(mtp_solver s);
static void validate_choice(int schedule, int tile_order, double grid_frac) {
  require(schedule == MTP_SCHEDULE_LAYERS || schedule == MTP_SCHEDULE_DAG, MTP_ERR_ARG, "unknown schedule");
  require(tile_order >= MTP_TILES_DEFAULT && tile_order <= MTP_TILES_COLUMN_MAJOR, MTP_ERR_ARG,
          "unknown tile order");
  require(grid_frac > 0.0 && grid_frac <= 1.0, MTP_ERR_ARG, "grid_frac must lie in (0, 1]");
}
// the solver's stream must be idle (or the solver new); drops the captured slab graph
static void solver_apply(mtp_solver s, int schedule, int tile_order, double grid_frac) {
  drop_graph(s);
  s->schedule = schedule;
  s->kp.tile_order = tile_order;
  s->grid_frac = grid_frac;
  s->kp.dag_grid = s->dag_grid_max > 0 ? std::max(1, (int)std::lround(grid_frac * s->dag_grid_max)) : 0;
}

mtp_status mtp_solver_create(mtp_mesh mesh, mtp_tents tents, int32_t p, int32_t q, int32_t m, int32_t precision,
                             double alpha, void* d_workspace, size_t bytes, void* hip_stream, mtp_solver* out) {
  MTP_TRY
  require(mesh && tents && out && d_workspace, MTP_ERR_ARG, "null pointer");
  require(alpha >= 0 && std::isfinite(alpha), MTP_ERR_ARG, "alpha must be >= 0");
  const int kernel = check_config(mesh->m, p, q, m, precision);
  auto* s = new mtp_solver_s();
  s->kernel = kernel;
  try {
    s->mesh = mesh->m;
    s->tents = tents->t;
    CurvedPlan cplan = curved_plan(mesh->m, s->tents, p);
    s->curved = !cplan.zone_elem.empty();
    if (s->curved) {   // affine tents first within each layer, then the curved ones
      Tents& T = s->tents;
      const int64_t nl = (int64_t)T.layer_ptr.size() - 1;
      std::vector<size_t> ord;
      std::vector<uint8_t> flag;
      for (int64_t l = 0; l < nl; ++l) {
        int64_t na = 0;
        for (int pass = 0; pass < 2; ++pass)
          for (int64_t i = T.layer_ptr[l]; i < T.layer_ptr[l + 1]; ++i)
            if (cplan.tent_curved[i] == pass) {
              ord.push_back((size_t)i);
              flag.push_back((uint8_t)pass);
              na += pass == 0;
            }
        s->layer_na.push_back(na);
      }
      auto perm = [&](auto& v) {
        auto o = v;
        for (size_t i = 0; i < ord.size(); ++i) o[i] = v[ord[i]];
        v.swap(o);
      };
      perm(T.vertex);
      perm(T.t_bot);
      perm(T.t_top);
      perm(T.layer);
      cplan = curved_plan(mesh->m, T, p);   // zone numbering of the reordered table
    }
    s->ref = build_refelem(mesh->m.d, p);
    s->p = p;
    s->q = q;
    s->m = m;
    s->nc = ncomp(mesh->m);
    s->off = plan(s->mesh, s->tents, s->ref, s->nc, opg_bytes(s->mesh, p, kernel), frg_bytes(s->mesh, p, kernel));
    require(bytes >= s->off.total, MTP_ERR_ARG, "workspace too small");
    s->ws = static_cast<char*>(d_workspace);
    s->stream = static_cast<hipStream_t>(hip_stream);
    const Mesh& M = s->mesh;
    for (int64_t i = 0; i < M.ne * (M.d + 1); ++i)
      if (M.nbr[i] < 0 && M.face_bc[i] == MTP_BC_DATA) s->has_data_faces = true;

    std::vector<int32_t> pptr, pelem, pinfo, fptr, faces;
    patch_tables(M, pptr, pelem, pinfo);
    patch_faces(M, pinfo, fptr, faces);
    auto up = [&](size_t off, const void* src, size_t n) {
      if (n) check_hip(hipMemcpyAsync(s->ws + off, src, n, hipMemcpyHostToDevice, s->stream), "upload");
    };
    up(s->off.grad_lam, M.grad_lam.data(), M.grad_lam.size() * 8);
    up(s->off.cells, M.cells.data(), M.cells.size() * 4);
    up(s->off.eps, M.eps.data(), M.eps.size() * 8);
    up(s->off.mu, M.mu.data(), M.mu.size() * 8);
    up(s->off.coords, M.coords.data(), M.coords.size() * 8);
    up(s->off.pptr, pptr.data(), pptr.size() * 4);
    up(s->off.pelem, pelem.data(), pelem.size() * 4);
    up(s->off.pinfo, pinfo.data(), pinfo.size() * 4);
    up(s->off.fptr, fptr.data(), fptr.size() * 4);
    up(s->off.face, faces.data(), faces.size() * 4);
    up(s->off.tv, s->tents.vertex.data(), s->tents.vertex.size() * 4);
    up(s->off.tt, s->tents.t_top.data(), s->tents.t_top.size() * 8);
    up(s->off.S, s->ref.S.data(), s->ref.S.size() * 8);
    up(s->off.L, s->ref.L.data(), s->ref.L.size() * 8);
    up(s->off.fnode, s->ref.fnode.data(), s->ref.fnode.size() * 4);
    up(s->off.fswap, s->ref.fswap.data(), s->ref.fswap.size() * 4);
    up(s->off.perm, s->ref.perm.data(), s->ref.perm.size() * 4);
    up(s->off.mi, s->ref.mi.data(), s->ref.mi.size() * 4);
    check_hip(hipMemsetAsync(s->ws + s->off.W, 0, sizeof(double) * M.ne * s->nc * s->ref.np, s->stream), "memset");
    check_hip(hipMemsetAsync(s->ws + s->off.tau, 0, sizeof(double) * M.nv, s->stream), "memset");
    check_hip(hipMemsetAsync(s->ws + s->off.err, 0, 16, s->stream), "memset");

    KernelParams& kp = s->kp;
    std::memset(&kp, 0, sizeof(kp));
    kp.d = M.d;
    kp.p = p;
    kp.q = q;
    kp.m = m;
    kp.nc = s->nc;
    kp.system = M.system;
    kp.np = s->ref.np;
    kp.nf = s->ref.nf;
    kp.alpha = alpha;
    kp.grad_lam = reinterpret_cast<const double*>(s->ws + s->off.grad_lam);
    kp.cells = reinterpret_cast<const int32_t*>(s->ws + s->off.cells);
    kp.eps = reinterpret_cast<const double*>(s->ws + s->off.eps);
    kp.mu = reinterpret_cast<const double*>(s->ws + s->off.mu);
    kp.coords = reinterpret_cast<const double*>(s->ws + s->off.coords);
    kp.patch_ptr = reinterpret_cast<const int32_t*>(s->ws + s->off.pptr);
    kp.patch_elem = reinterpret_cast<const int32_t*>(s->ws + s->off.pelem);
    kp.patch_info = reinterpret_cast<const int32_t*>(s->ws + s->off.pinfo);
    kp.pface_ptr = reinterpret_cast<const int32_t*>(s->ws + s->off.fptr);
    kp.pface = reinterpret_cast<const int32_t*>(s->ws + s->off.face);
    kp.fswap = reinterpret_cast<const int32_t*>(s->ws + s->off.fswap);
    kp.S = reinterpret_cast<const double*>(s->ws + s->off.S);
    kp.L = reinterpret_cast<const double*>(s->ws + s->off.L);
    kp.fnode = reinterpret_cast<const int32_t*>(s->ws + s->off.fnode);
    kp.perm = reinterpret_cast<const int32_t*>(s->ws + s->off.perm);
    kp.mi = reinterpret_cast<const int32_t*>(s->ws + s->off.mi);
    kp.W = reinterpret_cast<double*>(s->ws + s->off.W);
    kp.tau = reinterpret_cast<double*>(s->ws + s->off.tau);
    kp.err = reinterpret_cast<int32_t*>(s->ws + s->off.err);
    kp.tent_vertex = reinterpret_cast<const int32_t*>(s->ws + s->off.tv);
    kp.tent_top = reinterpret_cast<const double*>(s->ws + s->off.tt);
    kp.slab = reinterpret_cast<double*>(s->ws + s->off.slab);
    kp.max_patch = M.max_patch;
    // tent DAG for the persistent schedule
    {
      std::vector<int32_t> indeg, sptr, succ;
      int32_t nready = 0;
      tent_dag(M, s->tents, indeg, sptr, succ, nready);
      up(s->off.dag_indeg0, indeg.data(), indeg.size() * 4);
      up(s->off.dag_sptr, sptr.data(), sptr.size() * 4);
      up(s->off.dag_succ, succ.data(), succ.size() * 4);
      kp.dag_indeg = reinterpret_cast<int32_t*>(s->ws + s->off.dag_indeg);
      kp.dag_indeg0 = reinterpret_cast<const int32_t*>(s->ws + s->off.dag_indeg0);
      kp.dag_succ_ptr = reinterpret_cast<const int32_t*>(s->ws + s->off.dag_sptr);
      kp.dag_succ = reinterpret_cast<const int32_t*>(s->ws + s->off.dag_succ);
      kp.dag_queue = reinterpret_cast<int32_t*>(s->ws + s->off.dag_queue);
      kp.dag_ctl = reinterpret_cast<int32_t*>(s->ws + s->off.dag_ctl);
      kp.dag_n = (int32_t)s->tents.vertex.size();
      kp.dag_nready = nready;
      int dev = 0, khz = 0;
      check_hip(hipGetDevice(&dev), "device");
      s->device = dev;
      check_hip(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev), "wall clock rate");
      kp.dag_wait_ticks = (int64_t)khz * 1000 * 10;   // 10 s
      if (frg_bytes(M, p, kernel) > 0) {   // F/R slots of the extra-large patch class
        kp.frg = reinterpret_cast<double*>(s->ws + s->off.frg);
        kp.frg_slots = kFrgSlots;
      }
      kp.dag_grid = s->kernel == 0 ? 0 : tent_dag_grid(kp, s->kernel == 2);
      if (kp.frg) kp.dag_grid = std::min(kp.dag_grid, kp.frg_slots);
    }
    check_hip(prepare_tent_kernel(kp, s->kernel), "tent kernel attributes");
    if (opg_bytes(s->mesh, p, kernel) > 0) {   // the operator block, written once
      kp.opg = reinterpret_cast<double*>(s->ws + s->off.opg);
      check_hip(stage_tent_operator_mfma(kp, s->kernel == 2, s->stream), "operator staging");
    }
    if (s->curved) {
      // tables of the curved-element path; the persistent schedule does not cover it
      std::vector<double> cref, cgeo;
      std::vector<int32_t> cnbr;
      curved_tables(M, cplan, s->ref.mi, cref, cgeo, cnbr);
      up(s->off.cref, cref.data(), cref.size() * 8);
      up(s->off.cgeo, cgeo.data(), cgeo.size() * 8);
      up(s->off.cnbr, cnbr.data(), cnbr.size() * 4);
      up(s->off.czone, cplan.zone.data(), cplan.zone.size() * 4);
      CurvedParams& c = s->cparams;
      c.ref = reinterpret_cast<const double*>(s->ws + s->off.cref);
      c.geo = reinterpret_cast<const double*>(s->ws + s->off.cgeo);
      c.nbr = reinterpret_cast<const int32_t*>(s->ws + s->off.cnbr);
      c.zone = reinterpret_cast<const int32_t*>(s->ws + s->off.czone);
      c.p = p;
      c.max_patch = cplan.max_patch;
      c.geo_lds = tent_curved_lds_bytes(p, cplan.max_patch, true) <= 160 * 1024 ? 1 : 0;
      c.lds = tent_curved_lds_bytes(p, cplan.max_patch, c.geo_lds != 0);
      check_hip(launch_tent_curved(kp, c, 0, -1, nullptr), "curved kernel attributes");
      check_hip(hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking), "side stream");
      check_hip(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming), "fork event");
      check_hip(hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming), "join event");
      kp.dag_grid = 0;
    }
    check_hip(launch_slab_reset(kp, 0.0, s->tents.t_end, s->stream), "slab state");
    check_hip(hipStreamSynchronize(s->stream), "upload sync");
    s->dag_grid_max = kp.dag_grid;
    TuneEntry te;
    if (s->kernel != 0 && tune_find(solver_key(s), &te)) {
      if (te.schedule == MTP_SCHEDULE_DAG && s->dag_grid_max <= 0) te.schedule = MTP_SCHEDULE_LAYERS;
      solver_apply(s, te.schedule, te.tile_order, te.grid_frac);
      s->tuned_from_table = true;
    }
  } catch (...) {
    release_side(s);
    delete s;
    throw;
  }
  *out = s;
  MTP_CATCH
}

static void release_side(mtp_solver s) {
  if (s->side) (void)hipStreamSynchronize(s->side);
  if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
  if (s->ev_join) (void)hipEventDestroy(s->ev_join);
  if (s->side) (void)hipStreamDestroy(s->side);
  s->ev_fork = s->ev_join = nullptr;
  s->side = nullptr;
}

static void drop_graph(mtp_solver s) {
  if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  if (s->cap) (void)hipStreamDestroy(s->cap);
  s->gexec = nullptr;
  s->graph = nullptr;
  s->cap = nullptr;
}

void mtp_solver_destroy(mtp_solver solver) {
  if (!solver) return;
  (void)hipStreamSynchronize(solver->stream);
  drop_graph(solver);
  release_side(solver);
  delete solver;
}

mtp_status mtp_node_coords(mtp_solver s, double* xyz) {
  MTP_TRY
  require(s && xyz, MTP_ERR_ARG, "null pointer");
  const Mesh& M = s->mesh;
  const int d = M.d, np = s->ref.np, p = s->p;
  for (int64_t e = 0; e < M.ne; ++e) {
    if (M.n_curved > 0 && M.curved[e]) {   // the quadratic map of the reference node
      for (int a = 0; a < np; ++a) {
        const double xh[2] = {(double)s->ref.mi[a * 3 + 1] / p, (double)s->ref.mi[a * 3 + 2] / p};
        curved_node(M, e, xh, &xyz[(e * np + a) * 2]);
      }
      continue;
    }
    for (int a = 0; a < np; ++a)
      for (int i = 0; i < d; ++i) {
        double x = 0.0;
        for (int v = 0; v <= d; ++v)
          x += (double)s->ref.mi[a * (d + 1) + v] / p * M.coords[M.cells[e * (d + 1) + v] * d + i];
        xyz[(e * np + a) * d + i] = x;
      }
  }
  MTP_CATCH
}

mtp_status mtp_set_fields(mtp_solver s, const double* nodal, int32_t on_device, double t0) {
  MTP_TRY
  require(s && nodal, MTP_ERR_ARG, "null pointer");
  require(std::isfinite(t0), MTP_ERR_ARG, "t0 must be finite");
  const Mesh& M = s->mesh;
  const size_t n = (size_t)M.ne * s->ref.np * s->nc;
  const double* src = nodal;
  if (!on_device) {
    for (size_t i = 0; i < n; ++i) require(std::isfinite(nodal[i]), MTP_ERR_NONFINITE, "non-finite field value");
    check_hip(hipMemcpyAsync(s->ws + s->off.stage, nodal, n * 8, hipMemcpyHostToDevice, s->stream), "copy");
    src = reinterpret_cast<const double*>(s->ws + s->off.stage);
  }
  check_hip(launch_set_fields(s->kp, M.ne, src, t0, M.nv, s->stream), "set_fields");
  check_hip(launch_slab_reset(s->kp, t0, s->tents.t_end, s->stream), "slab state");
  if (!on_device) check_hip(hipStreamSynchronize(s->stream), "sync");
  s->t_base = t0;
  s->slab = 0;
  s->layers_done = 0;
  MTP_CATCH
}

mtp_status mtp_set_planewave_bc(mtp_solver s, const double* amp, const double* kvec, double omega, double phase) {
  MTP_TRY
  require(s && amp && kvec, MTP_ERR_ARG, "null pointer");
  for (int c = 0; c < s->nc; ++c) require(std::isfinite(amp[c]), MTP_ERR_ARG, "non-finite amplitude");
  for (int i = 0; i < s->mesh.d; ++i) require(std::isfinite(kvec[i]), MTP_ERR_ARG, "non-finite wave vector");
  require(std::isfinite(omega) && std::isfinite(phase), MTP_ERR_ARG, "non-finite omega or phase");
  // the captured slab graph holds the kernel parameter block by value: drop it so that the
  // next advance_to captures the new boundary data (work already enqueued keeps the old)
  check_hip(hipStreamSynchronize(s->stream), "sync");
  drop_graph(s);
  for (int c = 0; c < s->nc; ++c) s->kp.pw_amp[c] = amp[c];
  for (int i = 0; i < s->mesh.d; ++i) s->kp.pw_k[i] = kvec[i];
  s->kp.pw_omega = omega;
  s->kp.pw_phase = phase;
  s->kp.has_data = 1;
  MTP_CATCH
}

static void run_layer(mtp_solver s, int64_t layer, hipStream_t st) {
  const Tents& T = s->tents;
  const int64_t first = T.layer_ptr[layer];
  int64_t count = T.layer_ptr[layer + 1] - first;
  if (s->curved) {   // the layer's tents with a curved element in their patch, after the others
    const int64_t na = s->layer_na[layer];
    if (count > na && na > 0) {   // both kinds: the curved tents on the side stream, beside the others
      check_hip(hipEventRecord(s->ev_fork, st), "fork");
      check_hip(hipStreamWaitEvent(s->side, s->ev_fork, 0), "fork wait");
      check_hip(launch_tent_curved(s->kp, s->cparams, first + na, count - na, s->side), "curved tent kernel");
      check_hip(hipEventRecord(s->ev_join, s->side), "join");
    } else if (count > na) {
      check_hip(launch_tent_curved(s->kp, s->cparams, first + na, count - na, st), "curved tent kernel");
    }
    if (na > 0) {
      if (s->kernel == 0)
        check_hip(launch_tent_layer(s->kp, first, na, st), "tent kernel");
      else
        check_hip(launch_tent_layer_mfma(s->kp, first, na, s->kernel == 2, st), "tent kernel");
    }
    if (count > na && na > 0) check_hip(hipStreamWaitEvent(st, s->ev_join, 0), "join wait");
    return;
  }
  if (s->kernel == 0)
    check_hip(launch_tent_layer(s->kp, first, count, st), "tent kernel");
  else
    check_hip(launch_tent_layer_mfma(s->kp, first, count, s->kernel == 2, st), "tent kernel");
}

static void run_slab(mtp_solver s, hipStream_t st) {
  const int64_t nl = (int64_t)s->tents.layer_ptr.size() - 1;
  check_hip(launch_slab_begin(s->kp, st), "slab begin");
  if (s->schedule == MTP_SCHEDULE_DAG) {
    check_hip(launch_dag_reset(s->kp, st), "dag reset");
    check_hip(launch_tent_dag_mfma(s->kp, s->kernel == 2, st), "persistent tent kernel");
  } else {
    for (int64_t l = 0; l < nl; ++l) run_layer(s, l, st);
  }
  check_hip(launch_slab_end(s->kp, st), "slab end");
}

// Capture one slab on a private stream (default priority) and instantiate it.
static void build_graph(mtp_solver s) {
  check_hip(hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking), "capture stream");
  check_hip(hipStreamBeginCapture(s->cap, hipStreamCaptureModeRelaxed), "begin capture");
  try {
    run_slab(s, s->cap);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(s->cap, &g);
    if (g) (void)hipGraphDestroy(g);
    drop_graph(s);
    throw;
  }
  check_hip(hipStreamEndCapture(s->cap, &s->graph), "end capture");
  check_hip(hipGraphInstantiate(&s->gexec, s->graph, nullptr, nullptr, 0), "graph instantiate");
}

// n whole slabs from a flat front: replays of the captured slab graph, or eager launches
static void solver_slabs(mtp_solver s, int64_t n) {
  if (n > 0 && s->use_graph && !s->gexec) build_graph(s);
  for (int64_t j = 0; j < n; ++j) {
    if (s->use_graph)
      check_hip(hipGraphLaunch(s->gexec, s->stream), "graph launch");
    else
      run_slab(s, s->stream);
    s->slab++;
  }
}

mtp_status mtp_layer_advance(mtp_solver s, int64_t layer) {
  MTP_TRY
  require(s, MTP_ERR_ARG, "null solver");
  require(!s->has_data_faces || s->kp.has_data, MTP_ERR_STATE, "data boundary faces need mtp_set_planewave_bc");
  const int64_t nl = (int64_t)s->tents.layer_ptr.size() - 1;
  require(layer == s->layers_done && layer < nl, MTP_ERR_STATE, "layers must run in order");
  if (layer == 0) check_hip(launch_slab_begin(s->kp, s->stream), "slab begin");
  run_layer(s, layer, s->stream);
  s->layers_done++;
  if (s->layers_done == nl) {
    check_hip(launch_slab_end(s->kp, s->stream), "slab end");
    s->layers_done = 0;
    s->slab++;
  }
  MTP_CATCH
}

mtp_status mtp_advance_to(mtp_solver s, double T) {
  MTP_TRY
  require(s, MTP_ERR_ARG, "null solver");
  require(s->layers_done == 0, MTP_ERR_STATE, "front is not flat (a slab is half done)");
  require(!s->has_data_faces || s->kp.has_data, MTP_ERR_STATE, "data boundary faces need mtp_set_planewave_bc");
  const double h = s->tents.t_end;
  const double now = s->t_base + s->slab * h;
  const double k = (T - now) / h;
  const int64_t nslab = (int64_t)std::llround(k);
  require(std::fabs(k - (double)nslab) < 1e-9 && nslab >= 0, MTP_ERR_STATE,
          "T must be the front time plus a whole number of slabs");
  solver_slabs(s, nslab);
  MTP_CATCH
}

mtp_status mtp_front(mtp_solver s, double* t_front, int64_t* layers_done) {
  MTP_TRY
  require(s, MTP_ERR_ARG, "null solver");
  if (t_front) *t_front = s->t_base + s->slab * s->tents.t_end;
  if (layers_done) *layers_done = s->layers_done;
  MTP_CATCH
}

static mtp_status read_out(mtp_solver s, double* nodal, int32_t on_device, int raw) {
  MTP_TRY
  require(s && nodal, MTP_ERR_ARG, "null pointer");
  const Mesh& M = s->mesh;
  const size_t n = (size_t)M.ne * s->ref.np * s->nc;
  double* dst = on_device ? nodal : reinterpret_cast<double*>(s->ws + s->off.stage);
  check_hip(launch_get_fields(s->kp, M.ne, dst, raw, s->stream), "get_fields");
  int32_t err[4] = {0, 0, 0, 0};
  check_hip(hipMemcpyAsync(err, s->ws + s->off.err, 16, hipMemcpyDeviceToHost, s->stream), "copy");
  if (!on_device) check_hip(hipMemcpyAsync(nodal, dst, n * 8, hipMemcpyDeviceToHost, s->stream), "copy");
  check_hip(hipStreamSynchronize(s->stream), "sync");
  if (err[0] & ERRF_CAUSALITY) throw Error(MTP_ERR_DEVICE, "a tent met eps*mu - |grad phi|^2 <= 0");
  if (err[1] & ERRF_NONFINITE) throw Error(MTP_ERR_NONFINITE, "non-finite field values");
  if (err[2] & ERRF_DAG_WAIT)
    throw Error(MTP_ERR_DEVICE, "persistent schedule: a wait for a ready tent exceeded its bound (slab aborted)");
  MTP_CATCH
}

mtp_status mtp_get_fields(mtp_solver s, double* nodal, int32_t on_device) { return read_out(s, nodal, on_device, 0); }
mtp_status mtp_get_state(mtp_solver s, double* nodal, int32_t on_device) { return read_out(s, nodal, on_device, 1); }

mtp_status mtp_slab_dof_updates(mtp_solver s, double* dof_updates, int64_t* n_tents) {
  MTP_TRY
  require(s, MTP_ERR_ARG, "null solver");
  const Mesh& M = s->mesh;
  double tot = 0.0;
  for (int32_t v : s->tents.vertex) tot += (double)(M.v2e_ptr[v + 1] - M.v2e_ptr[v]);
  const int stages = s->method == MTP_METHOD_RK4 ? 4 : s->q;
  if (dof_updates) *dof_updates = tot * s->nc * s->ref.np * s->m * stages;
  if (n_tents) *n_tents = (int64_t)s->tents.vertex.size();
  MTP_CATCH
}

// ------------------------------------------------------------------ batches of solves
static void batch_check(const mtp_solver* solvers, int32_t n) {
  require(solvers && n >= 1, MTP_ERR_ARG, "empty batch");
  for (int i = 0; i < n; ++i) {
    const mtp_solver s = solvers[i];
    require(s != nullptr, MTP_ERR_ARG, "null solver in batch");
    require(s->kernel == 1 || s->kernel == 2, MTP_ERR_UNSUPPORTED, "batches need the matrix-core kernels");
    require(s->kernel == solvers[0]->kernel && s->mesh.d == solvers[0]->mesh.d, MTP_ERR_UNSUPPORTED,
            "a batch needs one dimension and precision");
    require(s->method == solvers[0]->method, MTP_ERR_UNSUPPORTED, "a batch needs one method (SAT or RK4)");
    require(s->mesh.system == solvers[0]->mesh.system, MTP_ERR_UNSUPPORTED, "a batch needs one system");
    require(!s->curved, MTP_ERR_UNSUPPORTED, "batches do not run curved elements");
    for (int j = 0; j < i; ++j) require(solvers[j] != s, MTP_ERR_ARG, "solver listed twice");
  }
}

static size_t batch_segments(const mtp_solver* solvers, int32_t n) {
  size_t tot = 0;
  for (int i = 0; i < n; ++i) tot += solvers[i]->tents.layer_ptr.size() - 1;
  return tot;
}

static int64_t batch_tents(const mtp_solver* solvers, int32_t n) {
  int64_t tot = 0;
  for (int i = 0; i < n; ++i) tot += (int64_t)solvers[i]->tents.vertex.size();
  return tot;
}

// At most one group per degree.
constexpr int kMaxBatchGroups = 8;

struct BatchLayout {
  size_t kps, segs, queue, ctl, off, roff, frg, opg, total;
  size_t frg_bytes = 0;   // F/R slots of a degree group in the 48-tet class (shared by the groups)
  size_t opg_bytes = 0;   // operator blocks of the degree groups whose class keeps it in device memory
};
// largest vertex patch of the batch's solvers of degree p
static int group_max_patch(const mtp_solver* solvers, int32_t n, int p) {
  int g = 0;
  for (int j = 0; j < n; ++j)
    if (solvers[j]->p == p) g = std::max(g, solvers[j]->mesh.max_patch);
  return g;
}
static BatchLayout batch_layout(const mtp_solver* solvers, int32_t n) {
  Layout L;
  BatchLayout o;
  o.kps = L.add(sizeof(KernelParams) * n);
  o.segs = L.add(sizeof(BatchSeg) * batch_segments(solvers, n));
  o.queue = L.add(sizeof(int32_t) * std::max<int64_t>(1, batch_tents(solvers, n)));
  o.ctl = L.add(sizeof(int32_t) * 4);
  o.off = L.add(sizeof(int32_t) * (n + kMaxBatchGroups));    // per group: n_g + 1 entries
  o.roff = L.add(sizeof(int32_t) * (n + kMaxBatchGroups));
  // a degree group whose largest patch falls in the 48-tet P4 class keeps its tents' F/R in
  // kFrgSlots slots; the groups run one after another on the batch's stream and share them
  size_t slot = 0;
  for (int i = 0; i < n; ++i) {
    const mtp_solver s = solvers[i];
    slot = std::max(slot, tent_mfma_frg_bytes(s->mesh.d, s->p, group_max_patch(solvers, n, s->p), s->kernel == 2,
                                              s->mesh.system));
  }
  o.frg_bytes = slot * kFrgSlots;
  o.frg = L.add(o.frg_bytes);
  // a degree group whose class keeps the operator block in device memory runs on the batch's
  // own copy: a member whose own patches fit a smaller class has none
  std::vector<int> degs;
  for (int i = 0; i < n; ++i)
    if (std::find(degs.begin(), degs.end(), solvers[i]->p) == degs.end()) degs.push_back(solvers[i]->p);
  for (int p : degs) {
    const mtp_solver s = solvers[0];
    o.opg_bytes += (tent_mfma_opg_bytes(s->mesh.d, p, group_max_patch(solvers, n, p), s->kernel == 2, s->mesh.system) +
                    255) / 256 * 256;
  }
  o.opg = L.add(o.opg_bytes);
  o.total = L.off;
  return o;
}

mtp_status mtp_batch_workspace_size(const mtp_solver* solvers, int32_t n, size_t* bytes) {
  MTP_TRY
  require(bytes, MTP_ERR_ARG, "null pointer");
  batch_check(solvers, n);
  *bytes = batch_layout(solvers, n).total;
  MTP_CATCH
}

static std::string batch_key(mtp_batch b) {
  std::string degs;
  int64_t tents = 0;
  int cls = 0;
  for (const auto& g : b->groups) {
    degs += std::to_string(g.p);
    cls = std::max(cls, patch_class(b->d, g.p, g.max_patch));
  }
  for (mtp_solver s : b->solvers) tents += (int64_t)s->tents.vertex.size();
  return "batch|" + device_tag(b->solvers[0]->device) + "|d" + std::to_string(b->d) + "|sys" + std::to_string(b->system) +
         "|m" + std::to_string(b->method) + "|p" + degs + "|k" +
         std::to_string(b->kernel) + "|nt" + std::to_string(cls) + "|t" + std::to_string(tents_class(tents)) +
         "|n" + std::to_string(log2_class((int64_t)b->solvers.size()));
}
static void drop_batch_graph(mtp_batch b);
// the batch's stream must be idle (or the batch new); drops the captured slab graph
static void batch_apply(mtp_batch b, int schedule, int tile_order, double grid_frac) {
  drop_batch_graph(b);
  b->schedule = schedule;
  b->tile_order = tile_order;
  b->grid_frac = grid_frac;
  for (auto& g : b->groups) g.bd.grid = g.grid_max > 0 ? std::max(1, (int)std::lround(grid_frac * g.grid_max)) : 0;
}

mtp_status mtp_batch_create(const mtp_solver* solvers, int32_t n, void* d_workspace, size_t bytes, void* hip_stream,
                            mtp_batch* out) {
  MTP_TRY
  require(out && d_workspace, MTP_ERR_ARG, "null pointer");
  batch_check(solvers, n);
  auto* b = new mtp_batch_s();
  try {
    b->solvers.assign(solvers, solvers + n);
    b->kernel = solvers[0]->kernel;
    b->d = solvers[0]->mesh.d;
    b->system = solvers[0]->mesh.system;
    b->method = solvers[0]->method;
    // degree groups: stable sort by degree
    b->order.resize(n);
    for (int i = 0; i < n; ++i) b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](int x, int y) { return solvers[x]->p < solvers[y]->p; });
    for (int j = 0; j < n; ++j) {
      const mtp_solver s = solvers[b->order[j]];
      if (b->groups.empty() || b->groups.back().p != s->p) {
        mtp_batch_s::Group g;
        g.p = s->p;
        g.s0 = j;
        b->groups.push_back(g);
      }
      auto& g = b->groups.back();
      g.s1 = j + 1;
      g.max_patch = std::max(g.max_patch, s->mesh.max_patch);
    }
    for (const auto& g : b->groups)
      require(tent_mfma_lds_bytes(b->d, g.p, g.max_patch, b->kernel == 2, b->system) <= 160 * 1024, MTP_ERR_UNSUPPORTED,
              "largest vertex patch of the batch does not fit the matrix-core kernel's LDS");
    const BatchLayout lo = batch_layout(solvers, n);
    require(bytes >= lo.total, MTP_ERR_ARG, "workspace too small");
    require(batch_tents(solvers, n) < (int64_t)1 << 31, MTP_ERR_UNSUPPORTED, "more than 2^31 - 1 tents per batch slab");
    b->ws = static_cast<char*>(d_workspace);
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->d_kps = reinterpret_cast<KernelParams*>(b->ws + lo.kps);
    b->d_segs = reinterpret_cast<BatchSeg*>(b->ws + lo.segs);
    if (lo.frg_bytes > 0) b->frg = reinterpret_cast<double*>(b->ws + lo.frg);
    // the operator blocks of the groups that keep it in device memory, staged once here
    {
      size_t off = 0;
      for (auto& g : b->groups) {
        const size_t nb = tent_mfma_opg_bytes(b->d, g.p, g.max_patch, b->kernel == 2, b->system);
        if (nb == 0) continue;
        require(off + nb <= lo.opg_bytes, MTP_ERR_STATE, "batch operator blocks exceed their region");
        KernelParams kp = solvers[b->order[g.s0]]->kp;   // the degree's reference tables
        kp.max_patch = g.max_patch;
        kp.opg = reinterpret_cast<double*>(b->ws + lo.opg + off);
        check_hip(stage_tent_operator_mfma(kp, b->kernel == 2, b->stream), "batch operator staging");
        g.opg = kp.opg;
        off += (nb + 255) / 256 * 256;
      }
    }
    // persistent schedule, per group: tent ids solver by solver, first-layer tents first in the queue
    {
      std::vector<int32_t> off(n + kMaxBatchGroups, 0), roff(n + kMaxBatchGroups, 0);
      for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        auto& g = b->groups[gi];
        const int base = g.s0 + (int)gi;   // the group's arrays start here
        int64_t ticks = 0;
        for (int j = g.s0; j < g.s1; ++j) {
          const mtp_solver s = solvers[b->order[j]];
          off[base + j - g.s0 + 1] = off[base + j - g.s0] + (int32_t)s->tents.vertex.size();
          roff[base + j - g.s0 + 1] = roff[base + j - g.s0] + s->kp.dag_nready;
          ticks = std::max(ticks, s->kp.dag_wait_ticks);
        }
        g.bd.queue = reinterpret_cast<int32_t*>(b->ws + lo.queue);   // shared: the groups run one after another
        g.bd.ctl = reinterpret_cast<int32_t*>(b->ws + lo.ctl);
        g.bd.off = reinterpret_cast<const int32_t*>(b->ws + lo.off) + base;
        g.bd.roff = reinterpret_cast<const int32_t*>(b->ws + lo.roff) + base;
        g.bd.nsolv = g.s1 - g.s0;
        g.bd.n = off[base + g.s1 - g.s0];
        g.bd.wait_ticks = ticks;
        g.bd.system = b->system;
        g.bd.method = b->method;
        g.grid_max = tent_batch_dag_grid(b->d, g.p, g.max_patch, b->kernel == 2, b->system, b->method);
        if (b->frg) g.grid_max = std::min(g.grid_max, kFrgSlots);   // one F/R slot per workgroup
        g.bd.grid = g.grid_max;
        if (g.grid_max <= 0) b->dag_ok = false;
      }
      check_hip(hipMemcpyAsync(b->ws + lo.off, off.data(), off.size() * 4, hipMemcpyHostToDevice, b->stream),
                "upload");
      check_hip(hipMemcpyAsync(b->ws + lo.roff, roff.data(), roff.size() * 4, hipMemcpyHostToDevice, b->stream),
                "upload");
    }
    // layer schedule: global layer l runs layer l of every solver that has it, one launch per group
    int64_t nl = 0;
    for (int i = 0; i < n; ++i) nl = std::max<int64_t>(nl, (int64_t)solvers[i]->tents.layer_ptr.size() - 1);
    std::vector<BatchSeg> segs;
    for (int64_t l = 0; l < nl; ++l) {
      for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        const auto& g = b->groups[gi];
        mtp_batch_s::Launch la;
        la.seg0 = (int64_t)segs.size();
        la.group = (int)gi;
        for (int j = g.s0; j < g.s1; ++j) {
          const Tents& T = solvers[b->order[j]]->tents;
          if (l + 1 >= (int64_t)T.layer_ptr.size()) continue;
          BatchSeg sg;
          sg.block0 = la.blocks;
          sg.first = T.layer_ptr[l];
          sg.count = T.layer_ptr[l + 1] - T.layer_ptr[l];
          sg.solver = j;
          sg.pad = 0;
          segs.push_back(sg);
          la.blocks += sg.count;
        }
        la.nseg = (int)((int64_t)segs.size() - la.seg0);
        if (la.nseg > 0) b->launches.push_back(la);
      }
    }
    check_hip(hipMemcpyAsync(b->d_segs, segs.data(), segs.size() * sizeof(BatchSeg), hipMemcpyHostToDevice,
                             b->stream), "upload");
    for (const auto& g : b->groups) {
      BatchLaunch bl{b->d_kps, b->d_segs, 0, -1, b->d, g.p, g.max_patch, b->system, b->method,
                     b->frg ? kFrgSlots : 0};
      check_hip(launch_tent_batch_mfma(bl, b->kernel == 2, nullptr), "batch kernel attributes");
    }
    check_hip(hipStreamSynchronize(b->stream), "sync");
    TuneEntry te;
    if (tune_find(batch_key(b), &te)) {
      if (te.schedule == MTP_SCHEDULE_DAG && !b->dag_ok) te.schedule = MTP_SCHEDULE_LAYERS;
      batch_apply(b, te.schedule, te.tile_order, te.grid_frac);
      b->tuned_from_table = true;
    }
  } catch (...) {
    delete b;
    throw;
  }
  *out = b;
  MTP_CATCH
}

static void batch_slab(mtp_batch b, hipStream_t st) {
  const int n = (int)b->solvers.size();
  check_hip(launch_batch_slab(b->d_kps, n, 0, st), "batch slab begin");
  if (b->schedule == MTP_SCHEDULE_DAG) {
    for (const auto& g : b->groups) {
      check_hip(launch_batch_dag_reset(b->d_kps + g.s0, g.bd, st), "batch dag reset");
      check_hip(launch_tent_batch_dag_mfma(b->d_kps + g.s0, g.bd, b->d, g.p, g.max_patch, b->kernel == 2, st),
                "persistent batched tent kernel");
    }
  } else {
    for (const auto& la : b->launches) {
      const auto& g = b->groups[la.group];
      BatchLaunch bl{b->d_kps, b->d_segs + la.seg0, la.nseg, la.blocks, b->d, g.p, g.max_patch, b->system,
                     b->method, b->frg ? kFrgSlots : 0};
      check_hip(launch_tent_batch_mfma(bl, b->kernel == 2, st), "batched tent kernel");
    }
  }
  check_hip(launch_batch_slab(b->d_kps, n, 1, st), "batch slab end");
}

static void drop_batch_graph(mtp_batch b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->cap = nullptr;
}

mtp_status mtp_batch_advance(mtp_batch b, int64_t n_slabs) {
  MTP_TRY
  require(b, MTP_ERR_ARG, "null batch");
  require(n_slabs >= 0, MTP_ERR_ARG, "negative slab count");
  const int n = (int)b->solvers.size();
  b->h_kps.resize(n);
  for (int j = 0; j < n; ++j) {
    mtp_solver s = b->solvers[b->order[j]];
    require(s->layers_done == 0, MTP_ERR_STATE, "a solver of the batch is in the middle of a slab");
    require(!s->has_data_faces || s->kp.has_data, MTP_ERR_STATE, "data boundary faces need mtp_set_planewave_bc");
    require(s->method == b->method, MTP_ERR_STATE, "a solver's method changed after the batch was created");
    b->h_kps[j] = s->kp;
    b->h_kps[j].tile_order = b->tile_order;
    // the 48-tet class: every launch takes its F/R slots from the batch's own; a group whose
    // class keeps the operator block in device memory reads the batch's copy
    b->h_kps[j].frg = b->frg;
    b->h_kps[j].frg_slots = b->frg ? kFrgSlots : 0;
    for (const auto& g : b->groups)
      if (j >= g.s0 && j < g.s1 && g.opg) b->h_kps[j].opg = g.opg;
    // work the solvers enqueued on their own streams comes first
    if (s->stream != b->stream) check_hip(hipStreamSynchronize(s->stream), "sync solver stream");
  }
  if (n_slabs == 0) return MTP_OK;
  check_hip(hipMemcpyAsync(b->d_kps, b->h_kps.data(), n * sizeof(KernelParams), hipMemcpyHostToDevice, b->stream),
            "upload");
  if (b->use_graph && !b->gexec) {
    check_hip(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "capture stream");
    check_hip(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed), "begin capture");
    try {
      batch_slab(b, b->cap);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(b->cap, &g);
      if (g) (void)hipGraphDestroy(g);
      drop_batch_graph(b);
      throw;
    }
    check_hip(hipStreamEndCapture(b->cap, &b->graph), "end capture");
    check_hip(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0), "graph instantiate");
  }
  for (int64_t k = 0; k < n_slabs; ++k) {
    if (b->use_graph)
      check_hip(hipGraphLaunch(b->gexec, b->stream), "graph launch");
    else
      batch_slab(b, b->stream);
  }
  for (int i = 0; i < n; ++i) {
    b->solvers[i]->slab += n_slabs;
    // later work on a solver's own stream waits for the batch
    if (b->solvers[i]->stream != b->stream) check_hip(hipStreamSynchronize(b->stream), "sync batch stream");
  }
  MTP_CATCH
}

mtp_status mtp_batch_set_schedule(mtp_batch b, int32_t schedule) {
  MTP_TRY
  require(b, MTP_ERR_ARG, "null batch");
  require(schedule == MTP_SCHEDULE_LAYERS || schedule == MTP_SCHEDULE_DAG, MTP_ERR_ARG, "unknown schedule");
  if (schedule == MTP_SCHEDULE_DAG)
    require(b->dag_ok, MTP_ERR_UNSUPPORTED, "the persistent batched kernel cannot be resident");
  if (schedule != b->schedule) {
    check_hip(hipStreamSynchronize(b->stream), "sync");
    drop_batch_graph(b);
    b->schedule = schedule;
  }
  MTP_CATCH
}

mtp_status mtp_batch_set_graph(mtp_batch b, int32_t on) {
  MTP_TRY
  require(b, MTP_ERR_ARG, "null batch");
  b->use_graph = on != 0;
  MTP_CATCH
}

void mtp_batch_destroy(mtp_batch b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  drop_batch_graph(b);
  delete b;
}

mtp_status mtp_solver_set_graph(mtp_solver s, int32_t on) {
  MTP_TRY
  require(s, MTP_ERR_ARG, "null solver");
  s->use_graph = on != 0;
  MTP_CATCH
}

mtp_status mtp_solver_set_schedule(mtp_solver s, int32_t schedule) {
  MTP_TRY
  require(s, MTP_ERR_ARG, "null solver");
  require(schedule == MTP_SCHEDULE_LAYERS || schedule == MTP_SCHEDULE_DAG, MTP_ERR_ARG, "unknown schedule");
  require(s->layers_done == 0, MTP_ERR_STATE, "front is not flat (a slab is half done)");
  if (schedule == MTP_SCHEDULE_DAG)
    require(s->kernel != 0 && s->dag_grid_max > 0, MTP_ERR_UNSUPPORTED,
            "the persistent schedule needs the matrix-core kernel resident on the device");
  if (schedule != s->schedule) {
    check_hip(hipStreamSynchronize(s->stream), "sync");
    drop_graph(s);
    s->schedule = schedule;
  }
  MTP_CATCH
}

mtp_status mtp_solver_set_method(mtp_solver s, int32_t method) {
  MTP_TRY
  require(s, MTP_ERR_ARG, "null solver");
  require(method == MTP_METHOD_SAT || method == MTP_METHOD_RK4, MTP_ERR_ARG, "unknown method");
  require(s->layers_done == 0, MTP_ERR_STATE, "front is not flat (a slab is half done)");
  require(method == MTP_METHOD_SAT || !s->curved, MTP_ERR_UNSUPPORTED, "curved elements run SAT only");
  if (method == MTP_METHOD_RK4)
    require(s->kernel == 1, MTP_ERR_UNSUPPORTED, "the RK4 variant runs on the FP64 matrix-core kernel");
  if (method != s->method) {
    check_hip(hipStreamSynchronize(s->stream), "sync");
    drop_graph(s);   // the captured launches hold the old parameter block
    s->method = method;
    s->kp.method = method;
  }
  MTP_CATCH
}

mtp_status mtp_solver_set_flux(mtp_solver s, int32_t flux) {
  MTP_TRY
  require(s, MTP_ERR_ARG, "null solver");
  require(flux == MTP_FLUX_PENALTY || flux == MTP_FLUX_IMPEDANCE, MTP_ERR_ARG, "unknown flux");
  require(s->layers_done == 0, MTP_ERR_STATE, "front is not flat (a slab is half done)");
  require(flux == MTP_FLUX_PENALTY || !s->curved, MTP_ERR_UNSUPPORTED, "curved elements use the penalty flux");
  if (flux == MTP_FLUX_IMPEDANCE)
    require(s->kernel != 0, MTP_ERR_UNSUPPORTED, "the impedance-matched flux runs on the matrix-core kernels");
  if (flux != s->kp.flux_kind) {
    check_hip(hipStreamSynchronize(s->stream), "sync");
    drop_graph(s);   // the captured launches hold the old parameter block
    s->kp.flux_kind = flux;
  }
  MTP_CATCH
}

mtp_status mtp_solver_set_dag_wait(mtp_solver s, double seconds) {
  MTP_TRY
  require(s, MTP_ERR_ARG, "null solver");
  require(seconds >= 0.0 && seconds <= 3600.0, MTP_ERR_ARG, "wait bound must be in [0, 3600] s");
  int dev = 0, khz = 0;
  check_hip(hipGetDevice(&dev), "device");
  check_hip(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev), "wall clock rate");
  check_hip(hipStreamSynchronize(s->stream), "sync");
  s->kp.dag_wait_ticks = (int64_t)(seconds * khz * 1000.0);
  drop_graph(s);   // the captured launch holds the old parameter block
  MTP_CATCH
}

mtp_status mtp_tents_dag_size(mtp_mesh mesh, mtp_tents tents, int64_t* n_edges) {
  MTP_TRY
  require(mesh && tents && n_edges, MTP_ERR_ARG, "null pointer");
  *n_edges = tent_dag_edges(mesh->m, tents->t);
  MTP_CATCH
}

mtp_status mtp_tents_dag(mtp_mesh mesh, mtp_tents tents, int32_t* pred_count, int32_t* succ_ptr, int32_t* succ,
                         int32_t* n_ready) {
  MTP_TRY
  require(mesh && tents, MTP_ERR_ARG, "null pointer");
  std::vector<int32_t> pc, sp, sc;
  int32_t nr = 0;
  tent_dag(mesh->m, tents->t, pc, sp, sc, nr);
  if (pred_count) std::copy(pc.begin(), pc.end(), pred_count);
  if (succ_ptr) std::copy(sp.begin(), sp.end(), succ_ptr);
  if (succ) std::copy(sc.begin(), sc.end(), succ);
  if (n_ready) *n_ready = nr;
  MTP_CATCH
}

// ------------------------------------------------------------------ checkpoint, stats
namespace {
struct CkptHeader {
  char magic[8];
  int32_t version, dim, system, p, q, m, nc, np;
  int64_t ne, nv, n_tents;
  double t_base, height;
  int64_t slab, layers_done;
  uint64_t checksum;
};
uint64_t fnv1a(const void* data, size_t n, uint64_t h) {
  const unsigned char* b = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}
const char kMagic[8] = {'M', 'T', 'P', 'C', 'K', 'P', 'T', '1'};
}  // namespace

mtp_status mtp_checkpoint_write(mtp_solver s, const char* path) {
  MTP_TRY
  require(s && path, MTP_ERR_ARG, "null pointer");
  const Mesh& M = s->mesh;
  const size_t nw = (size_t)M.ne * s->nc * s->ref.np;
  std::vector<double> W(nw), tau(M.nv);
  check_hip(hipStreamSynchronize(s->stream), "sync");
  check_hip(hipMemcpy(W.data(), s->ws + s->off.W, nw * 8, hipMemcpyDeviceToHost), "copy");
  check_hip(hipMemcpy(tau.data(), s->ws + s->off.tau, M.nv * 8, hipMemcpyDeviceToHost), "copy");
  CkptHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kMagic, 8);
  h.version = 1;
  h.dim = M.d;
  h.system = M.system;
  h.p = s->p;
  h.q = s->q;
  h.m = s->m;
  h.nc = s->nc;
  h.np = s->ref.np;
  h.ne = M.ne;
  h.nv = M.nv;
  h.n_tents = (int64_t)s->tents.vertex.size();
  h.t_base = s->t_base;
  h.height = s->tents.t_end;
  h.slab = s->slab;
  h.layers_done = s->layers_done;
  h.checksum = fnv1a(tau.data(), tau.size() * 8, fnv1a(W.data(), nw * 8, 1469598103934665603ull));
  FILE* f = std::fopen(path, "wb");
  require(f != nullptr, MTP_ERR_ARG, "cannot open the checkpoint file for writing");
  const bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 && std::fwrite(W.data(), 8, nw, f) == nw &&
                  std::fwrite(tau.data(), 8, tau.size(), f) == tau.size();
  const bool closed = std::fclose(f) == 0;
  require(ok && closed, MTP_ERR_ARG, "checkpoint write failed");
  MTP_CATCH
}

mtp_status mtp_checkpoint_read(mtp_solver s, const char* path) {
  MTP_TRY
  require(s && path, MTP_ERR_ARG, "null pointer");
  const Mesh& M = s->mesh;
  FILE* f = std::fopen(path, "rb");
  require(f != nullptr, MTP_ERR_ARG, "cannot open the checkpoint file");
  CkptHeader h;
  const size_t nw = (size_t)M.ne * s->nc * s->ref.np;
  std::vector<double> W, tau;
  bool ok = std::fread(&h, sizeof(h), 1, f) == 1 && std::memcmp(h.magic, kMagic, 8) == 0 && h.version == 1;
  const bool same = ok && h.dim == M.d && h.system == M.system && h.p == s->p && h.q == s->q && h.m == s->m &&
                    h.nc == s->nc && h.np == s->ref.np && h.ne == M.ne && h.nv == M.nv &&
                    h.n_tents == (int64_t)s->tents.vertex.size() && h.height == s->tents.t_end &&
                    h.layers_done >= 0 && h.layers_done < (int64_t)s->tents.layer_ptr.size() - 1 && h.slab >= 0;
  if (ok && same) {
    W.resize(nw);
    tau.resize(M.nv);
    ok = std::fread(W.data(), 8, nw, f) == nw && std::fread(tau.data(), 8, tau.size(), f) == tau.size();
  }
  std::fclose(f);
  require(ok, MTP_ERR_ARG, "not a checkpoint of this library, or truncated");
  require(same, MTP_ERR_STATE, "checkpoint of a different mesh, tent table or discretisation");
  require(fnv1a(tau.data(), tau.size() * 8, fnv1a(W.data(), nw * 8, 1469598103934665603ull)) == h.checksum,
          MTP_ERR_ARG, "checkpoint checksum mismatch");
  check_hip(hipStreamSynchronize(s->stream), "sync");
  check_hip(hipMemcpy(s->ws + s->off.W, W.data(), nw * 8, hipMemcpyHostToDevice), "upload");
  check_hip(hipMemcpy(s->ws + s->off.tau, tau.data(), M.nv * 8, hipMemcpyHostToDevice), "upload");
  // device slab state: [0] bottom of the current slab, [1] height, [2] front at slab 0, [3] slabs done
  const double slab[4] = {h.t_base + h.slab * h.height, h.height, h.t_base, (double)h.slab};
  check_hip(hipMemcpy(s->ws + s->off.slab, slab, sizeof(slab), hipMemcpyHostToDevice), "upload");
  check_hip(hipMemset(s->ws + s->off.err, 0, 16), "clear error flags");
  s->t_base = h.t_base;
  s->slab = h.slab;
  s->layers_done = h.layers_done;
  MTP_CATCH
}

mtp_status mtp_stats(mtp_solver s, mtp_stats_t* out) {
  MTP_TRY
  require(s && out, MTP_ERR_ARG, "null pointer");
  std::memset(out, 0, sizeof(*out));
  out->slabs_done = s->slab;
  out->layers_done = s->layers_done;
  out->n_tents = (int64_t)s->tents.vertex.size();
  out->n_layers = (int64_t)s->tents.layer_ptr.size() - 1;
  out->front_time = s->t_base + s->slab * s->tents.t_end;
  check_status(mtp_slab_dof_updates(s, &out->dof_updates_per_slab, nullptr));
  check_status(mtp_slab_flops(s, &out->flops_per_slab));
  out->kernel = s->kernel;
  out->schedule = s->schedule;
  out->method = s->method;
  out->flux = s->kp.flux_kind;
  out->system = s->mesh.system;
  out->persistent_workgroups = s->kp.dag_grid;
  MTP_CATCH
}

mtp_status mtp_solver_kernel(mtp_solver s, int32_t* kernel) {
  MTP_TRY
  require(s && kernel, MTP_ERR_ARG, "null pointer");
  *kernel = s->kernel;
  MTP_CATCH
}

mtp_status mtp_slab_flops(mtp_solver s, double* flops) {
  MTP_TRY
  require(s && flops, MTP_ERR_ARG, "null pointer");
  const Mesh& M = s->mesh;
  const int d = M.d, np = s->ref.np, nf = s->ref.nf, nc = s->nc;
  // algorithmic work per element and stage: volume contraction 2 np (d np) nc, face lift
  // 2 np nf nc d, face flux about 30 d nf (3D) / 12 d nf (2D), reference-direction flux
  // formation about 54 np (3D) / 12 np (2D), pointwise M' correction and inverse about
  // 100 np (3D) / 30 np (2D), Taylor sum 2 nc np (3D P4: 70,160 flop, 334 per spacetime DOF)
  const double vol = 2.0 * np * (d * np) * nc;
  const double lift = 2.0 * np * nf * nc * d;
  const double flx = (d == 3 ? 30.0 : 12.0) * d * nf;
  const double adir = (d == 3 ? 54.0 : 12.0) * np;
  const double kin = (d == 3 ? 100.0 : 30.0) * np;
  const double tay = 2.0 * nc * np;
  double elem_tents = 0.0;
  for (int32_t v : s->tents.vertex) elem_tents += (double)(M.v2e_ptr[v + 1] - M.v2e_ptr[v]);
  const int stages = s->method == MTP_METHOD_RK4 ? 4 : s->q;
  *flops = elem_tents * s->m * stages * (vol + lift + flx + adir + kin + tay);
  MTP_CATCH
}

// ------------------------------------------------------------------ tuning
mtp_status mtp_solver_set_tuning(mtp_solver s, const mtp_tuning* c) {
  MTP_TRY
  require(s && c, MTP_ERR_ARG, "null pointer");
  validate_choice(c->schedule, c->tile_order, c->grid_frac);
  require(s->layers_done == 0, MTP_ERR_STATE, "front is not flat (a slab is half done)");
  if (c->schedule == MTP_SCHEDULE_DAG)
    require(s->kernel != 0 && s->dag_grid_max > 0, MTP_ERR_UNSUPPORTED,
            "the persistent schedule needs the matrix-core kernel resident on the device");
  require(s->kernel != 0 || (c->tile_order == MTP_TILES_DEFAULT && c->grid_frac == 1.0), MTP_ERR_UNSUPPORTED,
          "the vector-ALU kernel has no tiles and no persistent grid");
  check_hip(hipStreamSynchronize(s->stream), "sync");
  solver_apply(s, c->schedule, c->tile_order, c->grid_frac);
  s->tuned_from_table = false;
  MTP_CATCH
}

mtp_status mtp_solver_get_tuning(mtp_solver s, mtp_tuning* c, int32_t* from_table) {
  MTP_TRY
  require(s && c, MTP_ERR_ARG, "null pointer");
  c->schedule = s->schedule;
  c->tile_order = s->kp.tile_order;
  c->grid_frac = s->grid_frac;
  if (from_table) *from_table = s->tuned_from_table ? 1 : 0;
  MTP_CATCH
}

mtp_status mtp_batch_set_tuning(mtp_batch b, const mtp_tuning* c) {
  MTP_TRY
  require(b && c, MTP_ERR_ARG, "null pointer");
  validate_choice(c->schedule, c->tile_order, c->grid_frac);
  if (c->schedule == MTP_SCHEDULE_DAG)
    require(b->dag_ok, MTP_ERR_UNSUPPORTED, "the persistent batched kernel cannot be resident");
  check_hip(hipStreamSynchronize(b->stream), "sync");
  batch_apply(b, c->schedule, c->tile_order, c->grid_frac);
  b->tuned_from_table = false;
  MTP_CATCH
}

mtp_status mtp_batch_get_tuning(mtp_batch b, mtp_tuning* c, int32_t* from_table) {
  MTP_TRY
  require(b && c, MTP_ERR_ARG, "null pointer");
  c->schedule = b->schedule;
  c->tile_order = b->tile_order;
  c->grid_frac = b->grid_frac;
  if (from_table) *from_table = b->tuned_from_table ? 1 : 0;
  MTP_CATCH
}

}  // extern "C"

namespace {

// Device copy of the mutable state of a set of solvers (W, front, slab state, error flags)
// and their host slab counters, for running trial slabs and putting everything back.
class StateSnapshot {
 public:
  StateSnapshot(const std::vector<mtp_solver>& ss, hipStream_t st) : ss_(ss), st_(st) {
    size_t tot = 0;
    for (mtp_solver s : ss_) {
      Part p;
      p.nw = (size_t)s->mesh.ne * s->nc * s->ref.np;
      p.nv = (size_t)s->mesh.nv;
      p.off = tot;
      p.slab = s->slab;
      p.t_base = s->t_base;
      tot += (p.nw + p.nv + 4) * 8 + 16;
      parts_.push_back(p);
    }
    if (hipMalloc(&buf_, std::max<size_t>(tot, 8)) != hipSuccess) {
      (void)hipGetLastError();
      buf_ = nullptr;
      throw Error(MTP_ERR_NOMEM, "device memory for the tuning snapshot");
    }
    copy(true);
  }
  ~StateSnapshot() {
    (void)hipStreamSynchronize(st_);
    if (buf_) (void)hipFree(buf_);
  }
  void restore() {
    copy(false);
    for (size_t i = 0; i < ss_.size(); ++i) {
      ss_[i]->slab = parts_[i].slab;
      ss_[i]->t_base = parts_[i].t_base;
      ss_[i]->layers_done = 0;
    }
  }

 private:
  struct Part {
    size_t nw = 0, nv = 0, off = 0;
    int64_t slab = 0;
    double t_base = 0.0;
  };
  void copy(bool save) {
    for (size_t i = 0; i < ss_.size(); ++i) {
      mtp_solver s = ss_[i];
      const Part& p = parts_[i];
      char* b = buf_ + p.off;
      const std::pair<char*, size_t> regs[4] = {{s->ws + s->off.W, p.nw * 8},
                                                {s->ws + s->off.tau, p.nv * 8},
                                                {s->ws + s->off.slab, 32},
                                                {s->ws + s->off.err, 16}};
      size_t o = 0;
      for (const auto& r : regs) {
        if (save)
          check_hip(hipMemcpyAsync(b + o, r.first, r.second, hipMemcpyDeviceToDevice, st_), "snapshot");
        else
          check_hip(hipMemcpyAsync(r.first, b + o, r.second, hipMemcpyDeviceToDevice, st_), "restore");
        o += r.second;
      }
    }
    check_hip(hipStreamSynchronize(st_), "sync");
  }
  std::vector<mtp_solver> ss_;
  hipStream_t st_;
  std::vector<Part> parts_;
  char* buf_ = nullptr;
};

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() {
    check_hip(hipEventCreate(&a), "event");
    check_hip(hipEventCreate(&b), "event");
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// the solvers' states (W, then the error words) in one host vector
void read_states(const std::vector<mtp_solver>& ss, std::vector<double>& w, int32_t* err_or) {
  size_t tot = 0;
  for (mtp_solver s : ss) tot += (size_t)s->mesh.ne * s->nc * s->ref.np;
  w.resize(tot);
  size_t o = 0;
  *err_or = 0;
  for (mtp_solver s : ss) {
    const size_t nw = (size_t)s->mesh.ne * s->nc * s->ref.np;
    int32_t err[4] = {0, 0, 0, 0};
    check_hip(hipStreamSynchronize(s->stream), "sync");
    check_hip(hipMemcpy(w.data() + o, s->ws + s->off.W, nw * 8, hipMemcpyDeviceToHost), "copy");
    check_hip(hipMemcpy(err, s->ws + s->off.err, 16, hipMemcpyDeviceToHost), "copy");
    *err_or |= err[0] | err[1] | err[2] | err[3];
    o += nw;
  }
}

struct Choice {
  int schedule = MTP_SCHEDULE_LAYERS, order = MTP_TILES_DEFAULT;
  double frac = 1.0, ms = 0.0;
};

// The search shared by solvers and batches: tile orders on the layer schedule, then the
// persistent schedule with the best order, then smaller persistent grids if it wins.
// run(c, n) applies c and runs n slabs on the stream; trial() wraps it with the state
// restore, the bit-for-bit check of the first slab and the event timing.
template <class Apply, class Run>
Choice search(const std::vector<mtp_solver>& ss, hipStream_t st, bool has_tiles, bool dag_ok, int slabs,
              Apply apply, Run run, int* ncand, double* ms_default) {
  StateSnapshot snap(ss, st);
  EventPair ev;
  std::vector<double> ref, cur;
  auto trial = [&](Choice c) -> Choice {
    snap.restore();
    apply(c);
    run(1);
    int32_t err = 0;
    read_states(ss, cur, &err);
    if (err != 0) throw Error(MTP_ERR_DEVICE, "a tuning candidate set the device error flags");
    if (ref.empty())
      ref.swap(cur);
    else if (std::memcmp(ref.data(), cur.data(), ref.size() * 8) != 0)
      throw Error(MTP_ERR_DEVICE, "a tuning candidate changed the results");
    check_hip(hipEventRecord(ev.a, st), "event");
    run(slabs);
    check_hip(hipEventRecord(ev.b, st), "event");
    check_hip(hipEventSynchronize(ev.b), "event sync");
    float ms = 0.0f;
    check_hip(hipEventElapsedTime(&ms, ev.a, ev.b), "event time");
    read_states(ss, cur, &err);
    if (err != 0) throw Error(MTP_ERR_DEVICE, "a tuning candidate set the device error flags");
    c.ms = ms / slabs;
    ++*ncand;
    return c;
  };
  Choice dflt;
  Choice best;
  try {
    dflt = trial(Choice{});
    best = dflt;
    if (has_tiles) {
      for (int o = MTP_TILES_ROUND_ROBIN; o <= MTP_TILES_COLUMN_MAJOR; ++o) {
        Choice c;
        c.order = o;
        c = trial(c);
        if (c.ms < best.ms) best = c;
      }
      if (dag_ok) {
        Choice c;
        c.schedule = MTP_SCHEDULE_DAG;
        c.order = best.order;
        c = trial(c);
        if (c.ms < best.ms) {
          best = c;
          for (double f : {0.75, 0.5}) {
            Choice g = best;
            g.frac = f;
            g = trial(g);
            if (g.ms < best.ms) best = g;
          }
        }
      }
    }
  } catch (...) {
    snap.restore();
    throw;
  }
  snap.restore();
  if (best.ms > 0.98 * dflt.ms) best = dflt;
  *ms_default = dflt.ms;
  return best;
}

}  // namespace

extern "C" {

mtp_status mtp_solver_tune(mtp_solver s, int32_t slabs, mtp_tune_result* out) {
  MTP_TRY
  require(s && out, MTP_ERR_ARG, "null pointer");
  require(slabs >= 1, MTP_ERR_ARG, "slabs_per_trial must be >= 1");
  require(s->layers_done == 0, MTP_ERR_STATE, "front is not flat (a slab is half done)");
  require(!s->has_data_faces || s->kp.has_data, MTP_ERR_STATE, "data boundary faces need mtp_set_planewave_bc");
  check_hip(hipStreamSynchronize(s->stream), "sync");
  int32_t err[4] = {0, 0, 0, 0};
  check_hip(hipMemcpy(err, s->ws + s->off.err, 16, hipMemcpyDeviceToHost), "copy");
  require((err[0] | err[1] | err[2] | err[3]) == 0, MTP_ERR_STATE,
          "the solver has pending device errors (read them with mtp_get_fields first)");
  const Choice orig{s->schedule, s->kp.tile_order, s->grid_frac, 0.0};
  const bool orig_table = s->tuned_from_table;
  int ncand = 0;
  double ms_default = 0.0;
  Choice best;
  try {
    best = search(
        {s}, s->stream, s->kernel != 0, s->kernel != 0 && s->dag_grid_max > 0, slabs,
        [&](const Choice& c) { solver_apply(s, c.schedule, c.order, c.frac); },
        [&](int64_t n) { solver_slabs(s, n); }, &ncand, &ms_default);
  } catch (...) {
    solver_apply(s, orig.schedule, orig.order, orig.frac);
    s->tuned_from_table = orig_table;
    throw;
  }
  solver_apply(s, best.schedule, best.order, best.frac);
  s->tuned_from_table = false;
  TuneEntry te;
  te.schedule = best.schedule;
  te.tile_order = best.order;
  te.grid_frac = best.frac;
  te.ms_best = best.ms;
  te.ms_default = ms_default;
  te.candidates = ncand;
  if (s->kernel != 0) tune_put(solver_key(s), te);
  out->best.schedule = best.schedule;
  out->best.tile_order = best.order;
  out->best.grid_frac = best.frac;
  out->ms_best = best.ms;
  out->ms_default = ms_default;
  out->candidates = ncand;
  MTP_CATCH
}

mtp_status mtp_batch_tune(mtp_batch b, int32_t slabs, mtp_tune_result* out) {
  MTP_TRY
  require(b && out, MTP_ERR_ARG, "null pointer");
  require(slabs >= 1, MTP_ERR_ARG, "slabs_per_trial must be >= 1");
  for (mtp_solver s : b->solvers) {
    require(s->layers_done == 0, MTP_ERR_STATE, "a solver of the batch is in the middle of a slab");
    require(!s->has_data_faces || s->kp.has_data, MTP_ERR_STATE, "data boundary faces need mtp_set_planewave_bc");
    check_hip(hipStreamSynchronize(s->stream), "sync");
    int32_t err[4] = {0, 0, 0, 0};
    check_hip(hipMemcpy(err, s->ws + s->off.err, 16, hipMemcpyDeviceToHost), "copy");
    require((err[0] | err[1] | err[2] | err[3]) == 0, MTP_ERR_STATE,
            "a solver of the batch has pending device errors (read them with mtp_get_fields first)");
  }
  check_hip(hipStreamSynchronize(b->stream), "sync");
  const Choice orig{b->schedule, b->tile_order, b->grid_frac, 0.0};
  const bool orig_table = b->tuned_from_table;
  int ncand = 0;
  double ms_default = 0.0;
  Choice best;
  try {
    best = search(
        b->solvers, b->stream, true, b->dag_ok, slabs,
        [&](const Choice& c) { batch_apply(b, c.schedule, c.order, c.frac); },
        [&](int64_t n) { check_status(mtp_batch_advance(b, n)); }, &ncand, &ms_default);
  } catch (...) {
    batch_apply(b, orig.schedule, orig.order, orig.frac);
    b->tuned_from_table = orig_table;
    throw;
  }
  batch_apply(b, best.schedule, best.order, best.frac);
  b->tuned_from_table = false;
  TuneEntry te;
  te.schedule = best.schedule;
  te.tile_order = best.order;
  te.grid_frac = best.frac;
  te.ms_best = best.ms;
  te.ms_default = ms_default;
  te.candidates = ncand;
  tune_put(batch_key(b), te);
  out->best.schedule = best.schedule;
  out->best.tile_order = best.order;
  out->best.grid_frac = best.frac;
  out->ms_best = best.ms;
  out->ms_default = ms_default;
  out->candidates = ncand;
  MTP_CATCH
}

mtp_status mtp_tune_save(const char* path) {
  MTP_TRY
  require(path != nullptr, MTP_ERR_ARG, "null path");
  tune_save_file(path);
  MTP_CATCH
}

mtp_status mtp_tune_load(const char* path) {
  MTP_TRY
  require(path != nullptr, MTP_ERR_ARG, "null path");
  tune_load_file(path);
  MTP_CATCH
}

mtp_status mtp_tune_clear(void) {
  MTP_TRY
  tune_clear_all();
  MTP_CATCH
}

mtp_status mtp_tune_size(int32_t* n) {
  MTP_TRY
  require(n != nullptr, MTP_ERR_ARG, "null pointer");
  *n = tune_count();
  MTP_CATCH
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free advance
namespace mtp {

void set_last_error(const char* msg) { g_last_error = msg; }

int solver_device(mtp_solver s) { return s->device; }

// mtp_advance_to on the persistent schedule with its per-slab scratch (working predecessor
// counts, ready queue, control words) at d_scratch (cap bytes) instead of the solver's
// workspace; eager launches on the solver's stream, no graph, nothing allocated.
void advance_to_dag_scratch(mtp_solver s, double T, char* d_scratch, size_t cap) {
  require(s != nullptr, MTP_ERR_ARG, "null solver");
  require(s->kernel != 0 && s->kp.dag_grid > 0, MTP_ERR_UNSUPPORTED,
          "the persistent schedule needs the matrix-core kernel resident on the device");
  require(s->layers_done == 0, MTP_ERR_STATE, "front is not flat (a slab is half done)");
  require(!s->has_data_faces || s->kp.has_data, MTP_ERR_STATE, "data boundary faces need mtp_set_planewave_bc");
  const double h = s->tents.t_end;
  const double now = s->t_base + s->slab * h;
  const double k = (T - now) / h;
  const int64_t nslab = (int64_t)std::llround(k);
  require(std::fabs(k - (double)nslab) < 1e-9 && nslab >= 0, MTP_ERR_STATE,
          "T must be the front time plus a whole number of slabs");
  const size_t n = (size_t)std::max(1, s->kp.dag_n);
  Layout L;
  const size_t o_indeg = L.add(4 * n), o_queue = L.add(4 * n), o_ctl = L.add(16);
  if (L.off > cap) {
    char msg[160];
    std::snprintf(msg, sizeof msg, "a slab of %d tents needs %zu bytes of scratch; the static array holds %zu",
                  s->kp.dag_n, L.off, cap);
    throw Error(MTP_ERR_UNSUPPORTED, msg);
  }
  KernelParams kp = s->kp;
  kp.dag_indeg = reinterpret_cast<int32_t*>(d_scratch + o_indeg);
  kp.dag_queue = reinterpret_cast<int32_t*>(d_scratch + o_queue);
  kp.dag_ctl = reinterpret_cast<int32_t*>(d_scratch + o_ctl);
  for (int64_t j = 0; j < nslab; ++j) {
    check_hip(launch_slab_begin(kp, s->stream), "slab begin");
    check_hip(launch_dag_reset(kp, s->stream), "dag reset");   // clears every scratch word the slab reads
    check_hip(launch_tent_dag_mfma(kp, s->kernel == 2, s->stream), "persistent tent kernel");
    check_hip(launch_slab_end(kp, s->stream), "slab end");
    s->slab++;
  }
}

}  // namespace mtp
