/*
 * mtp.h -- C interface of the MI355X (gfx950) library for explicit mapped tent pitching
 * (MTP) with structure-aware Taylor (SAT) time stepping for DG Maxwell.
 *
 * Method (Gopalakrishnan, Hochsteger, Schoeberl, Wintersteiger, "An Explicit Mapped Tent
 * Pitching Scheme for Maxwell Equations"):
 *   - section 2: the front is a P1 function (one time per vertex); a tent moves one
 *     vertex up; its spatial projection is the vertex patch; tents at vertices of graph
 *     distance >= 2 are independent and form a layer;
 *   - section 3: each tent is mapped to the cylinder patch x (0,1) by
 *     phi = (1-t) phi_b + t phi_t; the pulled-back system
 *     d_t (g(u) - f(u) grad phi) + div(delta f(u)) = 0, delta = phi_t - phi_b, is
 *     discretised by upwind DG of degree p, giving d/dt (M U) = A U;
 *   - section 4: q-stage SAT on m sub-intervals (eqs. coeff_rec, recursion-init) with
 *     the closed-form pointwise inverse of the mass form; Y = M U passes unchanged
 *     from one tent to the next.
 *
 * Conventions
 *   - Every call returns an mtp_status (0 = MTP_OK, < 0 error) and never aborts;
 *     mtp_last_error() returns a thread-local message for the last failure.
 *   - Arrays passed in are copied; the caller keeps ownership.  Handles are owned by
 *     the caller and released with the matching *_destroy.
 *   - Device memory comes from the caller: mtp_solver_workspace_size() reports the
 *     bytes, the caller allocates them (e.g. a torch uint8 tensor) and passes the
 *     device pointer to mtp_solver_create(); the library allocates no device memory.
 *     All device work is enqueued on the hip stream given at creation.
 *   - Field arrays in the interchange format are (ne, Np, nc) doubles: for each element
 *     its Np nodal values, each node holding the nc components (3D: Ex Ey Ez Hx Hy Hz;
 *     2D TE: Ex Ey Hz).  Nodes: reference coordinates (i/p, j/p[, k/p]), i fastest, then
 *     j, then k, with i+j(+k) <= p, mapped by x = v0 + sum_l xhat_l (v_l - v0) with the
 *     element's vertices in the order given to mtp_mesh_create.
 *   - Cells: (ne, dim+1) vertex ids; local face j is the face opposite local vertex j.
 */
#ifndef MTP_H
#define MTP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mtp_status;
typedef struct mtp_mesh_s* mtp_mesh;
typedef struct mtp_tents_s* mtp_tents;
typedef struct mtp_solver_s* mtp_solver;
typedef struct mtp_batch_s* mtp_batch;

enum {
  MTP_OK = 0,
  MTP_ERR_ARG = -1,         /* invalid argument (null pointer, size, range)            */
  MTP_ERR_MESH = -2,        /* non-conforming mesh, degenerate element, bad face kind  */
  MTP_ERR_CAUSALITY = -3,   /* slope fraction outside (0,1): tents would not be causal */
  MTP_ERR_PITCH = -4,       /* pitching made no progress (also: a tent table that is   */
                            /* not one mtp_pitch_layers made)                          */
  MTP_ERR_NONFINITE = -5,   /* non-finite field values                                 */
  MTP_ERR_DEVICE = -6,      /* HIP runtime error or a device-side check failed         */
  MTP_ERR_STATE = -7,       /* call out of order (e.g. advancing past the tent table)  */
  MTP_ERR_NOMEM = -8,       /* host memory exhausted                                   */
  MTP_ERR_UNSUPPORTED = -9  /* (dim, p) or patch size outside what the kernels cover   */
};
/* the name of the pitching status in the boundary sketch this interface follows */
enum { MTP_ERR_PITCH_STALL = MTP_ERR_PITCH };

/* boundary-condition kinds of boundary faces */
enum { MTP_BC_PEC = 0, MTP_BC_PMC = 1, MTP_BC_DATA = 2 };

/* equations (the method applies to linear hyperbolic systems in conservation form
 * d_t g(u) + div f(u) = 0; sections 1 and 3)
 *   MTP_SYSTEM_MAXWELL   u = (E, H) (3D) or (Ex, Ey, Hz) (2D TE), g(u) = (eps E, mu H)
 *   MTP_SYSTEM_ACOUSTIC  linear acoustics, u = (p, v), g(u) = (kappa p, rho v),
 *                        f(u) n = (v.n, p n); the mesh's eps / mu arrays hold kappa
 *                        (the inverse bulk modulus) and rho.  Boundary kinds: MTP_BC_PEC
 *                        is a pressure-release wall (p = 0), MTP_BC_PMC a rigid wall
 *                        (v.n = 0), MTP_BC_DATA a plane wave.  Matrix-core kernels, SAT,
 *                        single solves.                                             */
enum { MTP_SYSTEM_MAXWELL = 0, MTP_SYSTEM_ACOUSTIC = 1 };

/* arithmetic of the tent kernels (section 4's recursion Y_{i,n} = A U_{i,n-1}: the
 * contractions; the pointwise inverse and the Taylor sum of eq. taylor_pol)
 *   MTP_FP64       plain FP64; contractions on the FP64 matrix cores (falls back to the
 *                  vector-ALU kernel when a patch does not fit the matrix-core kernel)
 *   MTP_MIXED_FP32 the contractions of SAT stages n >= 2, which act on the small Taylor
 *                  coefficients U_{i,n-1}, n-1 >= 1, run on the FP32 matrix cores; the first
 *                  stage of every sub-interval (acting on U_{i,0}, the size of the fields),
 *                  the closed-form inversions, fluxes and the Taylor sum stay FP64
 *   MTP_FP64_VALU  plain FP64 on the vector ALUs (reference kernel)
 *   MTP_BF16X3     reserved for split-BF16 contractions of the stages n >= 2 (three BF16
 *                  products per FP32 product, FP32 accumulation); not built: solvers
 *                  asking for it get MTP_ERR_UNSUPPORTED                                */
enum { MTP_FP64 = 0, MTP_MIXED_FP32 = 1, MTP_FP64_VALU = 2, MTP_BF16X3 = 3 };

/* how a slab's tents are scheduled on the device
 *   MTP_SCHEDULE_LAYERS  one launch per layer (stream order is the layer barrier)
 *   MTP_SCHEDULE_DAG     one persistent launch per slab: workgroups take tents from a
 *                        device queue as soon as the tents they depend on are done
 *                        (see mtp_tents_dag), with no barrier between layers        */
enum { MTP_SCHEDULE_LAYERS = 0, MTP_SCHEDULE_DAG = 1 };

/* time stepping inside a tent (section 4)
 *   MTP_METHOD_SAT  the structure-aware Taylor recursion with q stages (default)
 *   MTP_METHOD_RK4  classical RK4 on dY/dth = A M(th)^{-1} Y + boundary data, m steps per
 *                   tent: the naive approach the paper contrasts with SAT, which loses
 *                   the order of the time stepping (for comparison studies)      */
enum { MTP_METHOD_SAT = 0, MTP_METHOD_RK4 = 1 };

/* numerical flux on the faces (section 3)
 *   MTP_FLUX_PENALTY    the printed upwind form 1/2 A(n)(u_in + u_out) + alpha P_t(u_in - u_out),
 *                       with no material parameters (default; alpha = 1/2 is the exact
 *                       upwind flux for unit impedance)
 *   MTP_FLUX_IMPEDANCE  the impedance-matched upwind flux A(n) u*, u* the interface state of
 *                       the Riemann problem between the two media (Z = sqrt(mu/eps)); equal
 *                       to the penalty form with alpha = 1/2 where Z = 1 on both sides   */
enum { MTP_FLUX_PENALTY = 0, MTP_FLUX_IMPEDANCE = 1 };

/* Equations the mesh's coefficients describe (MTP_SYSTEM_MAXWELL by default); set before
 * creating solvers (it fixes the field count nc: 6 / 3 for Maxwell, d + 1 for acoustics,
 * and the layout of every nodal array is [element][node][component]).  Pitching is the
 * same for both (wave speed 1/sqrt(eps mu)).  Errors: MTP_ERR_ARG. */
mtp_status mtp_mesh_set_system(mtp_mesh mesh, int32_t system);

/* Conforming simplicial mesh (section 2).  dim = 2 (triangles, TE fields) or 3 (tets).
 * coords (nv*dim), cells (ne*(dim+1), int32: meshes up to 2^31 - 1 vertices and elements),
 * eps/mu (ne) per-element material constants, face_bc (ne*(dim+1)) boundary kind per local
 * face, read only where the face lies on the domain boundary; NULL means PEC everywhere.
 * (The boundary is given per local face, not as a separate list of boundary faces: every
 * element's kinds sit beside its cell, and faces need not be matched on the host.)  All
 * arrays are copied.  Errors: MTP_ERR_ARG, MTP_ERR_MESH (zero-volume element, a face
 * shared by more than two elements, eps or mu <= 0). */
mtp_status mtp_mesh_create(int32_t dim, int64_t nv, const double* coords, int64_t ne,
                           const int32_t* cells, const double* eps, const double* mu,
                           const int32_t* face_bc, mtp_mesh* out);
mtp_status mtp_mesh_info(mtp_mesh mesh, int32_t* dim, int64_t* nv, int64_t* ne,
                         int32_t* max_patch);
void mtp_mesh_destroy(mtp_mesh mesh);

/* Curved elements (section 4: on the few curved elements the projection that follows the
 * pointwise closed-form inverse uses an approximation of the inverse mass matrix).  2D
 * only.  nodes (ne*6*2): six geometry nodes per triangle, the three vertices in cell order
 * (equal to the mesh's coordinates), then the midpoints of the edges (0,1), (1,2), (0,2);
 * the element map is the quadratic isoparametric one, x = sum_i nodes_i N_i(xhat).  An
 * element whose midpoint nodes are the straight midpoints stays affine; a shared edge must
 * carry one midpoint node.  The pitcher then bounds a curved element's hat-function
 * gradients over the element (the largest min_i sum_{j != i} |grad lambda_j| over the
 * barycentric lattice i/12, j/12), so call this before mtp_pitch_layers, and before
 * mtp_solver_create.  Solvers then run the tents whose patch holds a curved element on a
 * separate FP64 vector-ALU path, beside the layer's other tents (on a second stream, joined
 * before the next layer): every patch element by
 * quadrature (collapsed Gauss-Jacobi rule, p + 4 points per direction) with the element
 * map's Jacobian at the points, grad phi = J^{-T} sum_k tau_k gradhat lambdahat_k varying
 * inside the element, the closed-form inverse at the points, and the weight-adjusted
 * inverse mass Mhat^{-1} M_{1/J} Mhat^{-1} (M_{1/J} = int phi_a phi_b / |det J|, p + 8
 * points) for every projection.  Scope of such solvers: 2D Maxwell, p = 1..4, MTP_FP64,
 * MTP_FP64_VALU or MTP_MIXED_FP32 (the precision of the other tents; the curved ones always
 * run in FP64), SAT, the penalty flux, the layer schedule, walls
 * (PEC/PMC) next to curved elements; no batches.  mtp_node_coords maps a curved element's
 * nodes through its quadratic map.  Errors: MTP_ERR_ARG (null, dim != 2, the first three
 * nodes not the element's vertices, non-finite nodes), MTP_ERR_MESH (a shared edge with two
 * midpoint nodes, a curved element with a non-positive Jacobian on the lattice). */
mtp_status mtp_mesh_set_curved_p2(mtp_mesh mesh, const double* nodes);

/* Tent pitching on the host (section 2: the front is advanced one vertex at a time,
 * each step limited by causality; section 5 bounds the front slope by 1/(2c)), from the
 * flat front t = t_start to the flat front t = t_end.  Rule (the paper defers the
 * algorithm to earlier work; this is the library's documented choice): per element
 * k_T = slope_fraction*sqrt(eps mu) / min_i sum_{j!=i} |grad lambda_j|, per edge
 * k_vw = min over its elements; repeatedly the vertex with the smallest (time, id) moves
 * to min(H, Q floor((min over neighbours w of tau_w + k_vw)/Q - 1e-3)), Q = 2^-24,
 * H = t_end - t_start, times measured from t_start, in layer 1 + the largest layer of
 * itself and its neighbours.  Keeps |grad tau| <= slope_fraction*sqrt(eps mu) on every
 * element (the paper's experiments use 1/2).  The table is a slab of height H: a solver
 * applies it from its current flat front (mtp_set_fields' t0) and repeats it slab after
 * slab (mtp_advance_to), so one table serves every slab bit for bit.  Errors:
 * MTP_ERR_ARG (t_end <= t_start or not finite), MTP_ERR_CAUSALITY (slope_fraction not in
 * (0,1)), MTP_ERR_PITCH. */
mtp_status mtp_pitch_layers(mtp_mesh mesh, double t_start, double t_end, double slope_fraction,
                            mtp_tents* out);

/* Pitching rules (section 2 leaves the order in which vertices move open: any order that
 * keeps the causality bound yields a valid tent table). */
enum {
  MTP_PITCH_MIN_VERTEX = 0,   /* mtp_pitch_layers' rule: the (time, id)-smallest vertex moves   */
  MTP_PITCH_COLOUR = 1,       /* the vertex graph is coloured greedily (ids ascending, smallest */
                              /* colour no neighbour holds); the colours take turns, and at its */
                              /* turn every vertex of the colour below H moves (ids ascending)  */
                              /* to the target above, capped at tau_v + 1.5 min_w k_vw, if that */
                              /* lies above its time.                                           */
  MTP_PITCH_AUTO = 2          /* both tables; the one whose tents' patch sizes sum to less (the */
                              /* minimum-vertex table on a tie)                                 */
};
/* mtp_pitch_layers with a choice of rule.  Both rules keep the slope bound and put a tent
 * in layer 1 + the largest layer of itself and its neighbours, so both make tables that
 * solvers, batches and mtp_tents_dag take alike.  They differ in order: the minimum-vertex
 * rule advances the front in time order, which on irregular meshes serialises it (a disk of
 * triangles gets a few tents per layer); the colour rule advances a whole independent set
 * per turn and gives layers as wide as a colour class, at the price of more layers (and, on
 * graded 3D meshes with material jumps, more tents) where the minimum-vertex rule already
 * fills them.  The cap bounds the pole height, which the pseudo-time operator scales with:
 * a vertex that waited while its neighbours rose would otherwise make poles of two edge
 * steps.  The table is the same for the same mesh and arguments on every call.  Errors: as
 * mtp_pitch_layers, and MTP_ERR_ARG for an unknown rule. */
mtp_status mtp_pitch_layers_rule(mtp_mesh mesh, double t_start, double t_end, double slope_fraction,
                                 int32_t rule, mtp_tents* out);
/* The rule a tent table was pitched by (MTP_PITCH_MIN_VERTEX or MTP_PITCH_COLOUR; for
 * MTP_PITCH_AUTO, the one chosen).  Host only.  Errors: MTP_ERR_ARG. */
mtp_status mtp_tents_rule(mtp_tents tents, int32_t* rule);
/* Size of a tent table (section 2: tents whose vertices are at graph distance >= 2 are
 * independent; a layer is a set of such tents).  n_tents, n_layers; layer_ptr
 * (n_layers+1 entries, may be NULL) receives the start of each layer in the layer-sorted
 * tent order used by mtp_tents_export.  Host only.  Errors: MTP_ERR_ARG. */
mtp_status mtp_tents_query(mtp_tents tents, int64_t* n_tents, int64_t* n_layers, int64_t* layer_ptr);
/* The tent table itself (section 2: a tent is the vertex that moves, the front time at
 * that vertex below and above it; its spatial extent is the vertex patch), sorted by
 * layer (stable in pitching order): central vertex, bottom and top time (absolute:
 * t_start plus the relative time), layer.  Arrays of n_tents entries owned by the caller;
 * any pointer may be NULL.  Host only.  Errors: MTP_ERR_ARG. */
mtp_status mtp_tents_export(mtp_tents tents, int32_t* vertex, double* t_bot, double* t_top,
                            int32_t* layer);
void mtp_tents_destroy(mtp_tents tents);

/* Device workspace needed by a solver for (mesh, tents, p, q, m, precision). */
mtp_status mtp_solver_workspace_size(mtp_mesh mesh, mtp_tents tents, int32_t p, int32_t q,
                                     int32_t m, int32_t precision, size_t* bytes);
/* Create a solver: spatial degree p (1..5 in 2D, 1..5 in 3D; 3D P5 on the matrix-core
 * kernels only).  Vertex patches of up to 48 tets (section 2: a tent covers the vertex
 * patch).  P4 in 3D: up to 36 with the operator block in device memory, 37-48 with the
 * tent's face fluxes and stage residual in device memory as well (1024 workgroup slots of
 * about 104 KB that the workspace includes).  P5 in 3D: the operator block in device
 * memory, and for 25-48 tets the slots too (about 130 KB each).  A batch holding a degree
 * group with such slots has slots of its own in its workspace.  Taylor order q >= 1 and
 * m >= 1 sub-intervals per tent (section 4; the paper uses q = p+1, m = 2p), flux
 * penalty alpha (1/2 is the exact upwind flux for unit impedance, 1 the printed
 * coefficient).  d_workspace: device pointer of at least the reported bytes, owned by
 * the caller and kept alive until mtp_solver_destroy.  hip_stream: a hipStream_t (NULL =
 * default stream).  Uploads mesh, tents and reference operators; fields start at zero.
 * Errors: MTP_ERR_ARG, MTP_ERR_UNSUPPORTED, MTP_ERR_DEVICE. */
mtp_status mtp_solver_create(mtp_mesh mesh, mtp_tents tents, int32_t p, int32_t q, int32_t m,
                             int32_t precision, double alpha, void* d_workspace, size_t bytes,
                             void* hip_stream, mtp_solver* out);
void mtp_solver_destroy(mtp_solver solver);

/* Physical coordinates of the interchange nodes (the equispaced nodes of the degree-p
 * Lagrange basis described above; section 3 discretises each tent by DG of degree p):
 * host array of ne*Np*dim doubles owned by the caller.  Host only.  Errors: MTP_ERR_ARG. */
mtp_status mtp_node_coords(mtp_solver solver, double* xyz);

/* Set the fields u on the flat front t0 (normally the t_start of the tent table).
 * nodal: exactly ne*Np*nc doubles in the interchange layout (ne, Np, nc), a host pointer if
 * on_device == 0, else a device pointer on the solver's device; the library reads that many
 * values and no more (a shorter array is read past its end: the binding checks the shape).
 * Stores w = g(u) (section 4: Y = MU passes unchanged from one tent to the next).
 * Errors: MTP_ERR_ARG, MTP_ERR_NONFINITE (host input), MTP_ERR_DEVICE. */
mtp_status mtp_set_fields(mtp_solver solver, const double* nodal, int32_t on_device, double t0);

/* Boundary data for MTP_BC_DATA faces (section 5.1 prescribes initial and boundary values
 * from the exact solution): the plane wave u(x,t) = amp * cos(k.x - omega t + phase).
 * amp: nc doubles, the amplitude of every field component (Maxwell 3D: E then H; 2D TE:
 * Ex, Ey, Hz; acoustics: p then v), kvec: dim doubles, omega: angular frequency.  The
 * caller states the full field amplitude, so any medium and system is covered; for a
 * Maxwell wave in a uniform medium with direction d and wave number k (the boundary
 * sketch's (dir, k, amp_E, phase)) pass kvec = k d, omega = k/sqrt(eps mu) and
 * amp = (amp_E, sqrt(eps/mu) d x amp_E).  The ghost state on a data face of a tent is
 * u(x, phi(x,t)), entering the SAT recursion through its t-derivatives delta^n d_t^n u
 * (chain rule of the tent map), interpolated at the face nodes.  Takes effect for work
 * enqueued after the call (synchronises the solver's stream and drops the captured slab
 * graph, which holds the old data).  Errors: MTP_ERR_ARG (null or non-finite values). */
mtp_status mtp_set_planewave_bc(mtp_solver solver, const double* amp, const double* kvec,
                                double omega, double phase);

/* Enqueue the tents of one layer of the current slab (section 2: the tents of a layer are
 * causally independent and run concurrently; layers run in order).  Stream ordered,
 * asynchronous; layer must be the next one of the slab.  Errors: MTP_ERR_ARG,
 * MTP_ERR_STATE (out of order, or data faces without mtp_set_planewave_bc),
 * MTP_ERR_DEVICE. */
mtp_status mtp_layer_advance(mtp_solver solver, int64_t layer);
/* Enqueue whole slabs until the flat front reaches T (T must be the current front time
 * plus a whole number of slab heights).  Asynchronous.  By default the first call captures
 * one slab (every layer launch, section 2's layer order) into a HIP graph on a private
 * stream and every slab replays it on the solver's stream; the slab's time offset lives in
 * device memory, so one graph serves all slabs. */
mtp_status mtp_advance_to(mtp_solver solver, double T);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): mtp_advance_to on the persistent
 * schedule (MTP_SCHEDULE_DAG, whatever the solver's setting), launched eagerly on the
 * solver's stream with no graph or stream creation, its per-slab scratch (working
 * predecessor counts, ready queue, control words: 8 bytes per tent of the slab + 16,
 * rounded to 256-byte blocks) taken from a static device array of MTP_STATIC_SCRATCH_BYTES
 * that the library holds on each GPU it runs on until the process ends, instead of from
 * the solver's workspace.  It calls no allocating routine.  Every call on one GPU shares
 * that GPU's array and each slab re-initialises what it reads, so calls that run one after
 * the other are independent; calls whose work overlaps on one GPU (solvers advanced on
 * different streams at once) race on the array and must be serialised by the caller.
 * Results equal mtp_advance_to's bit for bit.  Errors: MTP_ERR_ARG, MTP_ERR_STATE (as
 * mtp_advance_to), MTP_ERR_UNSUPPORTED (a slab with more tents than the array holds,
 * about 1.05 million, or the vector-ALU kernel), MTP_ERR_DEVICE. */
#define MTP_STATIC_SCRATCH_BYTES (8u << 20)
mtp_status mtp_advance_to_static(mtp_solver solver, double T);
/* Current front time (flat) and number of layers done in the current slab.  Host only. */
mtp_status mtp_front(mtp_solver solver, double* t_front, int64_t* layers_done);

/* Read-out (section 4: on a flat front the mass form is diagonal in the materials, and
 * in general u = K(grad tau)^{-1} w node by node): writes ne*Np*nc doubles in the
 * interchange format to a host (on_device == 0) or device pointer owned by the caller.
 * Synchronises the solver's stream and surfaces device-side error flags (MTP_ERR_DEVICE:
 * a tent met eps*mu - |grad phi|^2 <= 0, or a persistent-schedule wait exceeded its
 * bound; MTP_ERR_NONFINITE). */
mtp_status mtp_get_fields(mtp_solver solver, double* nodal, int32_t on_device);
/* Raw state w = g(u) - f(u) grad tau (the variable tents pass on, section 4), same layout,
 * ownership and errors as mtp_get_fields. */
mtp_status mtp_get_state(mtp_solver solver, double* nodal, int32_t on_device);

/* Batches of independent solves (section 2: tents on different meshes are independent).
 * Every launch of a batch runs layer l of every solver in it, so small solves share the
 * GPU: solvers must use the matrix-core kernels with one dimension, system (Maxwell or
 * acoustics), precision and method (SAT, or the RK4 variant in FP64); degrees may differ (solvers of one degree
 * form a group, and each layer index is one launch per group, or each group one persistent
 * launch).  q, m, meshes, materials, fluxes and boundary data may differ too.  Errors:
 * MTP_ERR_UNSUPPORTED for mixed systems, dimensions, precisions or methods, and curved
 * solvers; mtp_batch_advance
 * returns MTP_ERR_STATE if a member's method changed after the batch was made.
 * mtp_batch_advance moves every
 * solver forward by n_slabs of its own slab height; the first call captures one batched
 * slab into a HIP graph that later calls replay.  Solvers keep their handles and state;
 * a solver must not be advanced on its own while a batch call is in flight.
 * d_workspace: caller-owned device memory of mtp_batch_workspace_size bytes: the parameter
 * blocks, layer segments and persistent-schedule queues, plus, for a degree group whose
 * largest patch puts it in a class that keeps the operator block or the face fluxes and
 * stage residual in device memory (3D P4 beyond 24 tets, 3D P5), the batch's own copy of
 * that block (staged at creation) and its own F/R slots. */
mtp_status mtp_batch_workspace_size(const mtp_solver* solvers, int32_t n, size_t* bytes);
mtp_status mtp_batch_create(const mtp_solver* solvers, int32_t n, void* d_workspace, size_t bytes,
                            void* hip_stream, mtp_batch* out);
mtp_status mtp_batch_advance(mtp_batch batch, int64_t n_slabs);
mtp_status mtp_batch_set_graph(mtp_batch batch, int32_t on);
/* Schedule of the batch's slabs: MTP_SCHEDULE_LAYERS (one launch per global layer index,
 * and degree group, the default) or MTP_SCHEDULE_DAG (per slab, one persistent launch per
 * degree group draining one queue of ready tents of the group's solvers; tents of different
 * solves and of uneven patch size share the workgroups; the wait bound is the largest of
 * the group's solvers').  Results are identical.
 * Errors: MTP_ERR_ARG, MTP_ERR_UNSUPPORTED (kernel cannot be resident). */
mtp_status mtp_batch_set_schedule(mtp_batch batch, int32_t schedule);
void mtp_batch_destroy(mtp_batch batch);

/* Spacetime DOF updates of one slab: sum over tents of nc*Np*n_T(tent)*m*q (the paper's
 * spacetime DOF count, section 5), and the tent count. */
mtp_status mtp_slab_dof_updates(mtp_solver solver, double* dof_updates, int64_t* n_tents);

/* on = 0: advance_to launches layer by layer instead of replaying the captured slab graph. */
mtp_status mtp_solver_set_graph(mtp_solver solver, int32_t on);

/* Tent dependency graph of a tent table (section 2: a tent may be pitched, and evolved,
 * once the tents it depends on are done).  Tent i (table order) at vertex V depends on
 * the latest earlier tent at V and at every neighbour of V: those are the tents whose
 * patch shares an element with its patch or whose vertex time it reads.  n_edges
 * receives the number of dependencies.  mtp_tents_dag fills pred_count (n_tents),
 * succ_ptr (n_tents + 1) and succ (n_edges; the dependants of tent i are
 * succ[succ_ptr[i] .. succ_ptr[i+1]), in table order) and n_ready, the number of leading
 * tents without dependency (the first layer).  Any output pointer may be NULL.  Host
 * only; the caller owns the arrays.  Errors: MTP_ERR_ARG, MTP_ERR_PITCH (a tent without
 * dependency outside the first layer: not a table made by mtp_pitch_layers). */
mtp_status mtp_tents_dag_size(mtp_mesh mesh, mtp_tents tents, int64_t* n_edges);
mtp_status mtp_tents_dag(mtp_mesh mesh, mtp_tents tents, int32_t* pred_count, int32_t* succ_ptr, int32_t* succ,
                         int32_t* n_ready);

/* Schedule of the solver's slabs (MTP_SCHEDULE_LAYERS by default).  MTP_SCHEDULE_DAG runs
 * every tent of a slab in one launch of as many workgroups as the device holds at once;
 * each takes the next released tent from a queue, runs it, and releases the tents that
 * depended on it (device-scope release/acquire, so W and the front are visible across the
 * chip's caches).  The result is identical to the layer schedule: every tent computes the
 * same values from the same inputs.  mtp_layer_advance always runs single layers.
 * Errors: MTP_ERR_ARG, MTP_ERR_STATE (half-done slab), MTP_ERR_UNSUPPORTED (vector-ALU
 * kernel, or the kernel cannot be resident). */
mtp_status mtp_solver_set_schedule(mtp_solver solver, int32_t schedule);

/* Time stepping of the solver's tents (MTP_METHOD_SAT by default).  MTP_METHOD_RK4 runs
 * four evaluations of the mapped right-hand side per sub-interval, each with the
 * closed-form pointwise inverse K(b(th))^{-1} at its own time th; q is then unused and
 * mtp_slab_dof_updates / mtp_slab_flops count 4 stages.  Errors: MTP_ERR_ARG,
 * MTP_ERR_STATE (half-done slab), MTP_ERR_UNSUPPORTED (RK4 needs the FP64 matrix-core
 * kernel, i.e. precision MTP_FP64 with the patch fitting it). */
mtp_status mtp_solver_set_method(mtp_solver solver, int32_t method);

/* Numerical flux of the solver's faces (MTP_FLUX_PENALTY by default).  Walls and
 * plane-wave data faces take the element's own medium on both sides.  Errors: MTP_ERR_ARG,
 * MTP_ERR_STATE (half-done slab), MTP_ERR_UNSUPPORTED (vector-ALU kernel). */
mtp_status mtp_solver_set_flux(mtp_solver solver, int32_t flux);

/* Bound (seconds, default 10) on any single wait of the persistent schedule for a tent to
 * be released.  A wait that exceeds it aborts the slab: every workgroup leaves, and the
 * next mtp_get_fields / mtp_get_state returns MTP_ERR_DEVICE; the fields are then
 * undefined.  No correct run waits anywhere near the default.  Errors: MTP_ERR_ARG. */
mtp_status mtp_solver_set_dag_wait(mtp_solver solver, double seconds);

/* Kernel the solver runs: 0 vector-ALU FP64, 1 matrix-core FP64, 2 matrix-core FP32. */
mtp_status mtp_solver_kernel(mtp_solver solver, int32_t* kernel);

/* Algorithmic flop count of one slab (section 5 counts the work in spacetime DOF,
 * sum over tents of N_dof m q; this counts the arithmetic behind them): per element of a
 * tent's patch and per stage, the volume contraction 2 Np (d Np) nc, the face lift
 * 2 Np Nf nc d, the face flux 30 d Nf (2D: 12 d Nf), the reference-direction flux formation
 * 54 Np (2D: 12 Np), the pointwise correction and inverse 100 Np (2D: 30 Np) and the Taylor
 * sum 2 nc Np, times m q (RK4: 4 m).  3D P4 Maxwell: 70,160 flop per element-stage, 334 per
 * spacetime DOF.  Host only.  Errors: MTP_ERR_ARG. */
mtp_status mtp_slab_flops(mtp_solver solver, double* flops);

/* Checkpoint of a solver's state (host file, binary): the nodal state W (the mapped
 * variable the tents pass on, section 4), the front tau and the position in the slab
 * sequence, with a header naming the discretisation and a checksum.  The state is
 * copied out after the solver's stream has drained.  mtp_checkpoint_read restores it
 * into a solver of the same mesh, tent table, p, q, m and system (errors: MTP_ERR_ARG for
 * an unreadable, foreign, truncated or corrupted file, MTP_ERR_STATE for a checkpoint of
 * another configuration); the device error flags are cleared and the captured slab graph
 * stays valid.  Continuing from a restored checkpoint gives the same values bit for bit
 * as not having stopped. */
mtp_status mtp_checkpoint_write(mtp_solver solver, const char* path);
mtp_status mtp_checkpoint_read(mtp_solver solver, const char* path);

/* Counters and configuration of a solver (host copy; no device work). */
typedef struct {
  int64_t slabs_done, layers_done;   /* position of the front */
  int64_t n_tents, n_layers;         /* per slab */
  double front_time;                 /* time of the last flat front */
  double dof_updates_per_slab;       /* as mtp_slab_dof_updates */
  double flops_per_slab;             /* as mtp_slab_flops */
  int32_t kernel, schedule, method, flux, system;
  int32_t persistent_workgroups;     /* grid of the persistent schedule (0: not available) */
} mtp_stats_t;
mtp_status mtp_stats(mtp_solver solver, mtp_stats_t* out);

/* Tuning of launch choices that leave the results unchanged bit for bit: the schedule
 * (MTP_SCHEDULE_LAYERS or MTP_SCHEDULE_DAG), the assignment of the matrix-core product's
 * tiles to the waves of a tent's workgroup, and the number of workgroups of the
 * persistent schedule as a fraction of the resident maximum.  Every tent computes the same
 * values under any choice, so tuning changes the time only.  (The paper fixes none of
 * these: they are choices of this implementation.) */
enum {
  MTP_TILES_DEFAULT = 0,        /* round robin; fixed balanced table for full 3D P4 patches */
  MTP_TILES_ROUND_ROBIN = 1,    /* round robin over the tiles numbered row block first */
  MTP_TILES_BLOCKED = 2,        /* each wave a run of consecutive tiles */
  MTP_TILES_COLUMN_MAJOR = 3    /* round robin over the tiles numbered column block first */
};
typedef struct {
  int32_t schedule;     /* MTP_SCHEDULE_* */
  int32_t tile_order;   /* MTP_TILES_* */
  double grid_frac;     /* persistent workgroups / resident maximum, in (0, 1] */
} mtp_tuning;
typedef struct {
  mtp_tuning best;           /* the choice applied */
  double ms_best;            /* its time per slab */
  double ms_default;         /* time per slab of {LAYERS, DEFAULT, 1} */
  int32_t candidates;        /* choices timed */
} mtp_tune_result;

/* Apply a choice to a solver or batch (drops the captured slab graph).  Errors:
 * MTP_ERR_ARG (unknown value, grid_frac outside (0, 1]), MTP_ERR_STATE (half-done slab),
 * MTP_ERR_UNSUPPORTED (persistent schedule not available, or a non-default choice on the
 * vector-ALU kernel). */
mtp_status mtp_solver_set_tuning(mtp_solver solver, const mtp_tuning* choice);
mtp_status mtp_solver_get_tuning(mtp_solver solver, mtp_tuning* choice, int32_t* from_table);
mtp_status mtp_batch_set_tuning(mtp_batch batch, const mtp_tuning* choice);
mtp_status mtp_batch_get_tuning(mtp_batch batch, mtp_tuning* choice, int32_t* from_table);

/* Time the candidate choices on the solver's (batch's) own slabs and apply the fastest:
 * the tile assignments on the layer schedule, then the persistent schedule with the best
 * of them, then (if that wins) smaller persistent grids.  Each candidate runs one untimed
 * slab and slabs_per_trial (>= 1) timed ones (HIP events on the solver's stream), starting
 * from the state at the call; the state is restored afterwards, so the solve continues as
 * if the call had not happened.  The first slab of every candidate is checked to give the
 * same state bit for bit as the default's (MTP_ERR_DEVICE otherwise).  A choice replaces
 * the default only if it is at least 2 % faster.  The result is also recorded in the
 * process-wide tuning table under the configuration's key (device, dimension, system,
 * degree(s), kernel, method, patch-size class and tents-per-slab class), from which later
 * mtp_solver_create / mtp_batch_create calls of the same key take their initial choice.
 * Allocates a temporary device copy of the state (hipMalloc; not for callers that cannot
 * allocate).  Synchronous.  Errors: MTP_ERR_ARG, MTP_ERR_STATE (half-done slab, or data
 * faces without boundary data), MTP_ERR_NOMEM, MTP_ERR_DEVICE. */
mtp_status mtp_solver_tune(mtp_solver solver, int32_t slabs_per_trial, mtp_tune_result* out);
mtp_status mtp_batch_tune(mtp_batch batch, int32_t slabs_per_trial, mtp_tune_result* out);

/* The process-wide tuning table as a JSON file (host): mtp_tune_save writes every entry,
 * mtp_tune_load merges a file's entries into the table (later entries replace earlier ones
 * of the same key), mtp_tune_clear empties it, mtp_tune_size counts its entries.
 * Thread-safe.  Errors: MTP_ERR_ARG (unreadable or malformed file, write failure). */
mtp_status mtp_tune_save(const char* path);
mtp_status mtp_tune_load(const char* path);
mtp_status mtp_tune_clear(void);
mtp_status mtp_tune_size(int32_t* n_entries);

const char* mtp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MTP_H */
