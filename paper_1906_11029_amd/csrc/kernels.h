// Device-side parameter blocks shared by the host solver and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mtp {

struct KernelParams {
  int d, p, q, m, nc, np, nf;
  double alpha;
  // mesh
  const double* grad_lam;  // ne*(d+1)*d
  const int32_t* cells;    // ne*(d+1)
  const double* eps;       // ne
  const double* mu;        // ne
  const double* coords;    // nv*d
  // vertex patches (static): per entry element id and info = [k, fcode_1..fcode_d]
  //   fcode >= 0: (patch-local neighbour << 4) | (neighbour face (1..d) << 1) | orientation
  //   fcode <  0: -1 - boundary kind
  const int32_t* patch_ptr;
  const int32_t* patch_elem;
  const int32_t* patch_info;
  // faces of the patch computed once each: (patch element << 2) | face j (0-based), the
  // face owned by the lower patch index of its two elements, boundary faces by their element
  const int32_t* pface_ptr;   // nv+1
  const int32_t* pface;
  // reference tables
  const double* S;         // d*np*np [l][a][b]
  const double* L;         // d*nf*np [j][s][b]
  const int32_t* fnode;    // d*2*nf
  const int32_t* perm;     // (d+1)*np
  const int32_t* mi;       // np*(d+1)
  const int32_t* fswap;    // nf
  // state
  double* W;               // ne*nc*np  [e][c][node]
  // matrix-core kernels whose operator block does not fit the LDS beside the tent region:
  // the block in device memory (null otherwise)
  double* opg;
  // the extra-large patch class (F/R of the tent in device memory): frg_slots slots of one
  // workgroup's F/R each; the launches keep their grid within frg_slots (null / 0 otherwise)
  double* frg;
  int32_t frg_slots;
  double* tau;             // nv
  int32_t* err;            // device error flags
  // tents of the launch
  const int32_t* tent_vertex;
  const double* tent_top;
  // slab state in device memory: [0] time of the current slab's bottom (tent times are
  // relative to it), [1] slab height, [2] front time at slab 0, [3] completed slabs
  double* slab;
  // tent DAG of the persistent schedule: in-degree (working copy, refreshed from dag_indeg0
  // before every slab), successors (CSR), ready queue (-1 = slot not yet filled) and control
  // words [0] next slot to claim, [1] next slot to fill, [2] abort.  The dag_nready tents
  // without predecessor are the first ones of the tent table (layer 0).
  int32_t* dag_indeg;
  const int32_t* dag_indeg0;
  const int32_t* dag_succ_ptr;
  const int32_t* dag_succ;
  int32_t* dag_queue;
  int32_t* dag_ctl;
  int32_t dag_n, dag_nready, dag_grid;
  int64_t dag_wait_ticks;  // bound of any wait for a ready tent, in wall-clock ticks
  // time stepping inside a tent: 0 = SAT (q stages), 1 = classical RK4 on W (the naive
  // variant; FP64 matrix-core kernel only)
  int method;
  // face flux: 0 = the alpha-weighted upwind flux as printed, 1 = impedance-matched
  int flux_kind;
  // equations: 0 = Maxwell (E, H), 1 = linear acoustics (p, v)
  int system;
  // plane-wave boundary data
  int has_data;
  double pw_amp[6], pw_k[3], pw_omega, pw_phase;
  int max_patch;
  // assignment of the product's tiles to waves (tuned; results do not depend on it)
  int tile_order;
};

// One segment of a batched launch: layer slice (first, count) of solver `solver`, run by
// workgroups block0 .. block0 + count - 1.
struct BatchSeg {
  int64_t block0;
  int64_t first;
  int64_t count;
  int32_t solver;
  int32_t pad;
};

// Persistent schedule of a batch: one queue of global tent ids (solver offset + tent) over
// the tent DAGs of every solver (each solver's in-degrees and successors in its own
// parameter block).
struct BatchDag {
  int32_t* queue;        // n slots
  int32_t* ctl;          // [0] next slot to claim, [1] next slot to fill, [2] abort
  const int32_t* off;    // nsolv + 1: first global id of each solver
  const int32_t* roff;   // nsolv + 1: first queue slot of each solver's first-layer tents
  int32_t nsolv, n, grid;
  int64_t wait_ticks;
  int32_t system;        // MTP_SYSTEM_* of every solver of the batch
  int32_t method;        // MTP_METHOD_* of every solver of the batch (RK4: FP64 only)
};

struct BatchLaunch {
  const KernelParams* kps;   // device array, one entry per solver
  const BatchSeg* segs;      // device array, nseg entries sorted by block0
  int nseg;
  int64_t blocks;            // total workgroups (-1: only set the LDS attribute)
  int d, p, max_patch;
  int system;                // MTP_SYSTEM_* of every solver of the batch
  int method;                // MTP_METHOD_* of every solver of the batch (RK4: FP64 only)
  int frg_slots;             // the batch's F/R slots (classes with F/R in device memory; 0: none)
};

// The curved-element tent path: reference tables, per zone element tables and neighbours,
// the zone map (see CurvedPlan), and the launch shape.
struct CurvedParams {
  const double* ref;
  const double* geo;
  const int32_t* nbr;
  const int32_t* zone;
  int p, max_patch;
  int geo_lds;   // 1: the patch elements' geometry blocks are staged in LDS
  size_t lds;
};

// error flag bits
enum { ERRF_CAUSALITY = 1, ERRF_NONFINITE = 2, ERRF_DAG_WAIT = 4 };

size_t tent_kernel_lds_bytes(int d, int p, int max_patch);
bool tent_kernel_supported(int d, int p);
hipError_t launch_tent_layer(const KernelParams& kp, int64_t first, int64_t count, hipStream_t s);
// matrix-core variant: fp32 = 0 contracts in FP64, fp32 = 1 in FP32 (mixed path)
size_t tent_mfma_lds_bytes(int d, int p, int max_patch, int fp32, int system = 0);
// bytes of the operator block a matrix-core solver keeps in device memory (0: in LDS), and
// the launch that writes it to kp.opg once
size_t tent_mfma_opg_bytes(int d, int p, int max_patch, int fp32, int system);
hipError_t stage_tent_operator_mfma(const KernelParams& kp, int fp32, hipStream_t s);
// bytes of one workgroup's F/R slot in device memory (0: F/R in LDS)
size_t tent_mfma_frg_bytes(int d, int p, int max_patch, int fp32, int system);
hipError_t launch_tent_layer_mfma(const KernelParams& kp, int64_t first, int64_t count, int fp32, hipStream_t s);
// persistent schedule: reset the DAG state for one slab, then run every tent of the slab in
// one launch of kp.dag_grid workgroups (grid < 0: only set the kernel attributes)
hipError_t launch_dag_reset(const KernelParams& kp, hipStream_t s);
hipError_t launch_tent_dag_mfma(const KernelParams& kp, int fp32, hipStream_t s);
// workgroups of the persistent kernel that fit the device at once (0 if it cannot run)
int tent_dag_grid(const KernelParams& kp, int fp32);
// the same for a batch (kps: device array of the solvers' parameter blocks)
hipError_t launch_batch_dag_reset(const KernelParams* kps, const BatchDag& bd, hipStream_t s);
hipError_t launch_tent_batch_dag_mfma(const KernelParams* kps, const BatchDag& bd, int d, int p, int max_patch,
                                      int fp32, hipStream_t s);
int tent_batch_dag_grid(int d, int p, int max_patch, int fp32, int system = 0, int method = 0);
hipError_t launch_set_fields(const KernelParams& kp, int64_t ne, const double* u_nodal, double t0,
                             int64_t nv, hipStream_t s);
hipError_t launch_get_fields(const KernelParams& kp, int64_t ne, double* out, int raw, hipStream_t s);
hipError_t launch_tent_batch_mfma(const BatchLaunch& bl, int fp32, hipStream_t s);
hipError_t launch_batch_slab(const KernelParams* kps, int n, int end, hipStream_t s);
// tents [first, first + count) of the table on the curved-element path (2D TE, P1..P4);
// count < 0: only set the kernel attributes
hipError_t launch_tent_curved(const KernelParams& kp, const CurvedParams& cp, int64_t first, int64_t count,
                              hipStream_t s);
// geo: with the patch elements' geometry blocks staged in LDS
size_t tent_curved_lds_bytes(int p, int max_patch, bool geo);
// slab bookkeeping on the device (graph-safe: kernels, no memsets)
hipError_t launch_slab_reset(const KernelParams& kp, double t0, double height, hipStream_t s);
hipError_t launch_slab_begin(const KernelParams& kp, hipStream_t s);
hipError_t launch_slab_end(const KernelParams& kp, hipStream_t s);
// set the dynamic-LDS attribute of the tent kernel a solver uses (outside graph capture)
hipError_t prepare_tent_kernel(const KernelParams& kp, int kernel);

}  // namespace mtp
