"""Thin Python binding of the MTP C interface (include/mtp.h).

Argument marshalling only: every function forwards to the C function of the same name
in libmtp.so; all tent arithmetic runs in the library's HIP kernels.  PyTorch supplies
device memory (the solver workspace) and the HIP stream.  Importing this module never
falls back to anything: if libmtp.so is missing, load() raises.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmtp.so")

MTP_OK = 0
MTP_BC_PEC, MTP_BC_PMC, MTP_BC_DATA = 0, 1, 2
MTP_FP64, MTP_MIXED_FP32, MTP_FP64_VALU, MTP_BF16X3 = 0, 1, 2, 3
MTP_SCHEDULE_LAYERS, MTP_SCHEDULE_DAG = 0, 1
MTP_METHOD_SAT, MTP_METHOD_RK4 = 0, 1
MTP_FLUX_PENALTY, MTP_FLUX_IMPEDANCE = 0, 1
MTP_SYSTEM_MAXWELL, MTP_SYSTEM_ACOUSTIC = 0, 1
MTP_TILES_DEFAULT, MTP_TILES_ROUND_ROBIN, MTP_TILES_BLOCKED, MTP_TILES_COLUMN_MAJOR = 0, 1, 2, 3
MTP_PITCH_MIN_VERTEX, MTP_PITCH_COLOUR, MTP_PITCH_AUTO = 0, 1, 2

# tuning table shipped with the package (measured on MI355X); MTP_TUNE_FILE names another
# file to load instead, or, set to the empty string, disables loading one
TUNE_FILE = os.path.join(_HERE, "tuning", "mi355x.json")

_lib = None


class MTPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mtp error {code}: {msg}")
        self.code = code


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not built: run python -m paper_1906_11029_amd.build")
    # torch first: the library then binds to the HIP runtime torch already loaded, so
    # workspace tensors and torch streams belong to the same runtime instance
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P, i32, i64, dbl, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    pp = C.POINTER(C.c_void_p)
    sig = {
        "mtp_mesh_create": [i32, i64, P, i64, P, P, P, P, pp],
        "mtp_mesh_info": [P, P, P, P, P],
        "mtp_mesh_set_system": [P, i32],
        "mtp_mesh_set_curved_p2": [P, P],
        "mtp_pitch_layers": [P, dbl, dbl, dbl, pp],
        "mtp_pitch_layers_rule": [P, dbl, dbl, dbl, i32, pp],
        "mtp_tents_rule": [P, P],
        "mtp_tents_query": [P, P, P, P],
        "mtp_tents_export": [P, P, P, P, P],
        "mtp_solver_workspace_size": [P, P, i32, i32, i32, i32, P],
        "mtp_solver_create": [P, P, i32, i32, i32, i32, dbl, P, sz, P, pp],
        "mtp_node_coords": [P, P],
        "mtp_set_fields": [P, P, i32, dbl],
        "mtp_set_planewave_bc": [P, P, P, dbl, dbl],
        "mtp_layer_advance": [P, i64],
        "mtp_advance_to": [P, dbl],
        "mtp_advance_to_static": [P, dbl],
        "mtp_front": [P, P, P],
        "mtp_get_fields": [P, P, i32],
        "mtp_get_state": [P, P, i32],
        "mtp_slab_dof_updates": [P, P, P],
        "mtp_slab_flops": [P, P],
        "mtp_solver_kernel": [P, P],
        "mtp_solver_set_graph": [P, i32],
        "mtp_solver_set_schedule": [P, i32],
        "mtp_solver_set_method": [P, i32],
        "mtp_solver_set_flux": [P, i32],
        "mtp_checkpoint_write": [P, C.c_char_p],
        "mtp_checkpoint_read": [P, C.c_char_p],
        "mtp_stats": [P, P],
        "mtp_solver_set_dag_wait": [P, dbl],
        "mtp_tents_dag_size": [P, P, P],
        "mtp_tents_dag": [P, P, P, P, P, P],
        "mtp_batch_workspace_size": [P, i32, P],
        "mtp_batch_create": [P, i32, P, sz, P, pp],
        "mtp_batch_advance": [P, i64],
        "mtp_batch_set_graph": [P, i32],
        "mtp_batch_set_schedule": [P, i32],
        "mtp_solver_set_tuning": [P, P],
        "mtp_solver_get_tuning": [P, P, P],
        "mtp_batch_set_tuning": [P, P],
        "mtp_batch_get_tuning": [P, P, P],
        "mtp_solver_tune": [P, i32, P],
        "mtp_batch_tune": [P, i32, P],
        "mtp_tune_save": [C.c_char_p],
        "mtp_tune_load": [C.c_char_p],
        "mtp_tune_clear": [],
        "mtp_tune_size": [P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int32
    for name in ("mtp_mesh_destroy", "mtp_tents_destroy", "mtp_solver_destroy", "mtp_batch_destroy"):
        f = getattr(L, name)
        f.argtypes = [P]
        f.restype = None
    L.mtp_last_error.argtypes = []
    L.mtp_last_error.restype = C.c_char_p
    _lib = L
    path = os.environ.get("MTP_TUNE_FILE", TUNE_FILE)
    if path and os.path.exists(path):
        _check(L.mtp_tune_load(os.fsencode(path)))
    return L


def _check(status):
    if status != MTP_OK:
        raise MTPError(status, load().mtp_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ----------------------------------------------------------------- C-named functions
def mtp_mesh_create(coords, cells, eps=None, mu=None, face_bc=None):
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    dim = coords.shape[1]
    eps = None if eps is None else np.ascontiguousarray(eps, dtype=np.float64)
    mu = None if mu is None else np.ascontiguousarray(mu, dtype=np.float64)
    face_bc = None if face_bc is None else np.ascontiguousarray(face_bc, dtype=np.int32)
    h = C.c_void_p()
    _check(load().mtp_mesh_create(dim, coords.shape[0], _ptr(coords), cells.shape[0], _ptr(cells),
                                  _ptr(eps), _ptr(mu), _ptr(face_bc), C.byref(h)))
    return h


def mtp_mesh_info(mesh):
    d, nv, ne, mp = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int32()
    _check(load().mtp_mesh_info(mesh, C.byref(d), C.byref(nv), C.byref(ne), C.byref(mp)))
    return {"dim": d.value, "nv": nv.value, "ne": ne.value, "max_patch": mp.value}


def mtp_mesh_destroy(mesh):
    load().mtp_mesh_destroy(mesh)


def _release(name, h):
    """Destroy handle h with the library call `name` from a finaliser. Skipped once the
    library is gone: at interpreter shutdown module globals are cleared, and the process
    releases its memory anyway."""
    lib = _lib
    if h and lib is not None:
        getattr(lib, name)(h)


def mtp_pitch_layers(mesh, t_start, t_end, slope_fraction=0.5):
    h = C.c_void_p()
    _check(load().mtp_pitch_layers(mesh, float(t_start), float(t_end), float(slope_fraction), C.byref(h)))
    return h


def mtp_pitch_layers_rule(mesh, t_start, t_end, slope_fraction=0.5, rule=0):
    h = C.c_void_p()
    _check(load().mtp_pitch_layers_rule(mesh, float(t_start), float(t_end), float(slope_fraction), int(rule),
                                        C.byref(h)))
    return h


def mtp_tents_query(tents):
    nt, nl = C.c_int64(), C.c_int64()
    _check(load().mtp_tents_query(tents, C.byref(nt), C.byref(nl), None))
    ptr = np.zeros(nl.value + 1, dtype=np.int64)
    _check(load().mtp_tents_query(tents, None, None, _ptr(ptr)))
    return nt.value, nl.value, ptr


def mtp_tents_export(tents):
    nt, _, _ = mtp_tents_query(tents)
    v = np.zeros(nt, dtype=np.int32)
    tb = np.zeros(nt)
    tt = np.zeros(nt)
    lay = np.zeros(nt, dtype=np.int32)
    _check(load().mtp_tents_export(tents, _ptr(v), _ptr(tb), _ptr(tt), _ptr(lay)))
    return {"vertex": v, "t_bot": tb, "t_top": tt, "layer": lay}


def mtp_tents_dag(mesh, tents):
    nt, _, _ = mtp_tents_query(tents)
    ne = C.c_int64()
    _check(load().mtp_tents_dag_size(mesh, tents, C.byref(ne)))
    pc = np.zeros(nt, dtype=np.int32)
    sp = np.zeros(nt + 1, dtype=np.int32)
    sc = np.zeros(max(ne.value, 1), dtype=np.int32)
    nr = C.c_int32()
    _check(load().mtp_tents_dag(mesh, tents, _ptr(pc), _ptr(sp), _ptr(sc), C.byref(nr)))
    return {"pred_count": pc, "succ_ptr": sp, "succ": sc[:ne.value], "n_ready": nr.value}


def mtp_tents_destroy(tents):
    load().mtp_tents_destroy(tents)


def mtp_solver_workspace_size(mesh, tents, p, q, m, precision=MTP_FP64):
    n = C.c_size_t()
    _check(load().mtp_solver_workspace_size(mesh, tents, p, q, m, precision, C.byref(n)))
    return n.value


def mtp_solver_create(mesh, tents, p, q, m, precision, alpha, workspace_ptr, nbytes, stream_ptr):
    h = C.c_void_p()
    _check(load().mtp_solver_create(mesh, tents, p, q, m, precision, float(alpha), C.c_void_p(workspace_ptr),
                                    nbytes, C.c_void_p(stream_ptr), C.byref(h)))
    return h


def mtp_solver_destroy(solver):
    load().mtp_solver_destroy(solver)


def mtp_node_coords(solver, ne, np_, dim):
    out = np.zeros((ne, np_, dim))
    _check(load().mtp_node_coords(solver, _ptr(out)))
    return out


def mtp_set_fields(solver, nodal, shape, t0=0.0):
    """nodal: numpy array (host) or torch CUDA tensor (device) of exactly `shape` =
    (ne, Np, nc) float64 values (the library reads that many)."""
    shape = tuple(int(x) for x in shape)
    if isinstance(nodal, np.ndarray):
        if tuple(nodal.shape) != shape:
            raise ValueError(f"nodal fields must have shape {shape}, got {tuple(nodal.shape)}")
        a = np.ascontiguousarray(nodal, dtype=np.float64)
        _check(load().mtp_set_fields(solver, _ptr(a), 0, float(t0)))
    else:
        if not (nodal.is_cuda and nodal.is_contiguous() and str(nodal.dtype) == "torch.float64"):
            raise ValueError("device fields must be a contiguous float64 CUDA tensor")
        if tuple(nodal.shape) != shape:
            raise ValueError(f"nodal fields must have shape {shape}, got {tuple(nodal.shape)}")
        _check(load().mtp_set_fields(solver, C.c_void_p(nodal.data_ptr()), 1, float(t0)))


def mtp_set_planewave_bc(solver, amp, kvec, omega, phase, nc, dim):
    """amp: nc field amplitudes, kvec: dim wave-vector components."""
    a = np.ascontiguousarray(amp, dtype=np.float64).ravel()
    k = np.ascontiguousarray(kvec, dtype=np.float64).ravel()
    if a.size != nc or k.size != dim:
        raise ValueError(f"need {nc} amplitudes and {dim} wave-vector components, got {a.size} and {k.size}")
    _check(load().mtp_set_planewave_bc(solver, _ptr(a), _ptr(k), float(omega), float(phase)))


def mtp_layer_advance(solver, layer):
    _check(load().mtp_layer_advance(solver, int(layer)))


def mtp_advance_to(solver, T):
    _check(load().mtp_advance_to(solver, float(T)))


def mtp_advance_to_static(solver, T):
    _check(load().mtp_advance_to_static(solver, float(T)))


def mtp_front(solver):
    t, l = C.c_double(), C.c_int64()
    _check(load().mtp_front(solver, C.byref(t), C.byref(l)))
    return t.value, l.value


def _read(fn, solver, shape, out):
    if out is None:
        host = np.zeros(shape)
        _check(fn(solver, _ptr(host), 0))
        return host
    assert out.is_cuda and out.is_contiguous() and tuple(out.shape) == tuple(shape)
    _check(fn(solver, C.c_void_p(out.data_ptr()), 1))
    return out


def mtp_get_fields(solver, shape, out=None):
    return _read(load().mtp_get_fields, solver, shape, out)


def mtp_get_state(solver, shape, out=None):
    return _read(load().mtp_get_state, solver, shape, out)


def mtp_slab_dof_updates(solver):
    d, n = C.c_double(), C.c_int64()
    _check(load().mtp_slab_dof_updates(solver, C.byref(d), C.byref(n)))
    return d.value, n.value


def mtp_slab_flops(solver):
    f = C.c_double()
    _check(load().mtp_slab_flops(solver, C.byref(f)))
    return f.value


def mtp_solver_set_graph(solver, on):
    _check(load().mtp_solver_set_graph(solver, int(on)))


def mtp_solver_set_schedule(solver, schedule):
    _check(load().mtp_solver_set_schedule(solver, int(schedule)))


def mtp_solver_set_method(solver, method):
    _check(load().mtp_solver_set_method(solver, int(method)))


def mtp_solver_set_flux(solver, flux):
    _check(load().mtp_solver_set_flux(solver, int(flux)))


class mtp_stats_t(C.Structure):
    _fields_ = [("slabs_done", C.c_int64), ("layers_done", C.c_int64), ("n_tents", C.c_int64),
                ("n_layers", C.c_int64), ("front_time", C.c_double), ("dof_updates_per_slab", C.c_double),
                ("flops_per_slab", C.c_double), ("kernel", C.c_int32), ("schedule", C.c_int32),
                ("method", C.c_int32), ("flux", C.c_int32), ("system", C.c_int32),
                ("persistent_workgroups", C.c_int32)]


def mtp_stats(solver):
    st = mtp_stats_t()
    _check(load().mtp_stats(solver, C.byref(st)))
    return {name: getattr(st, name) for name, _ in mtp_stats_t._fields_}


def mtp_checkpoint_write(solver, path):
    _check(load().mtp_checkpoint_write(solver, os.fsencode(path)))


def mtp_checkpoint_read(solver, path):
    _check(load().mtp_checkpoint_read(solver, os.fsencode(path)))


def mtp_solver_set_dag_wait(solver, seconds):
    _check(load().mtp_solver_set_dag_wait(solver, float(seconds)))


def mtp_solver_kernel(solver):
    k = C.c_int32()
    _check(load().mtp_solver_kernel(solver, C.byref(k)))
    return k.value


def _handles(solvers):
    arr = (C.c_void_p * len(solvers))(*[s.h.value for s in solvers])
    return arr


def mtp_batch_workspace_size(solvers):
    n = C.c_size_t()
    _check(load().mtp_batch_workspace_size(_handles(solvers), len(solvers), C.byref(n)))
    return n.value


def mtp_batch_create(solvers, workspace_ptr, nbytes, stream_ptr):
    h = C.c_void_p()
    _check(load().mtp_batch_create(_handles(solvers), len(solvers), C.c_void_p(workspace_ptr), nbytes,
                                   C.c_void_p(stream_ptr), C.byref(h)))
    return h


def mtp_batch_advance(batch, n_slabs):
    _check(load().mtp_batch_advance(batch, int(n_slabs)))


def mtp_batch_set_graph(batch, on):
    _check(load().mtp_batch_set_graph(batch, int(on)))


def mtp_batch_set_schedule(batch, schedule):
    _check(load().mtp_batch_set_schedule(batch, int(schedule)))


def mtp_batch_destroy(batch):
    load().mtp_batch_destroy(batch)


class mtp_tuning(C.Structure):
    _fields_ = [("schedule", C.c_int32), ("tile_order", C.c_int32), ("grid_frac", C.c_double)]


class mtp_tune_result(C.Structure):
    _fields_ = [("best", mtp_tuning), ("ms_best", C.c_double), ("ms_default", C.c_double),
                ("candidates", C.c_int32)]


def _tuning_dict(t):
    return {"schedule": t.schedule, "tile_order": t.tile_order, "grid_frac": t.grid_frac}


def _set_tuning(fn, h, schedule, tile_order, grid_frac):
    _check(fn(h, C.byref(mtp_tuning(int(schedule), int(tile_order), float(grid_frac)))))


def _get_tuning(fn, h):
    t, f = mtp_tuning(), C.c_int32()
    _check(fn(h, C.byref(t), C.byref(f)))
    out = _tuning_dict(t)
    out["from_table"] = bool(f.value)
    return out


def _tune(fn, h, slabs_per_trial):
    r = mtp_tune_result()
    _check(fn(h, int(slabs_per_trial), C.byref(r)))
    return {"best": _tuning_dict(r.best), "ms_best": r.ms_best, "ms_default": r.ms_default,
            "candidates": r.candidates}


def mtp_solver_set_tuning(solver, schedule, tile_order=MTP_TILES_DEFAULT, grid_frac=1.0):
    _set_tuning(load().mtp_solver_set_tuning, solver, schedule, tile_order, grid_frac)


def mtp_solver_get_tuning(solver):
    return _get_tuning(load().mtp_solver_get_tuning, solver)


def mtp_batch_set_tuning(batch, schedule, tile_order=MTP_TILES_DEFAULT, grid_frac=1.0):
    _set_tuning(load().mtp_batch_set_tuning, batch, schedule, tile_order, grid_frac)


def mtp_batch_get_tuning(batch):
    return _get_tuning(load().mtp_batch_get_tuning, batch)


def mtp_solver_tune(solver, slabs_per_trial=2):
    return _tune(load().mtp_solver_tune, solver, slabs_per_trial)


def mtp_batch_tune(batch, slabs_per_trial=2):
    return _tune(load().mtp_batch_tune, batch, slabs_per_trial)


def mtp_tune_save(path):
    _check(load().mtp_tune_save(os.fsencode(path)))


def mtp_tune_load(path):
    _check(load().mtp_tune_load(os.fsencode(path)))


def mtp_tune_clear():
    _check(load().mtp_tune_clear())


def mtp_tune_size():
    n = C.c_int32()
    _check(load().mtp_tune_size(C.byref(n)))
    return n.value


# ----------------------------------------------------------------- thin object wrappers
def mtp_mesh_set_system(mesh, system):
    _check(load().mtp_mesh_set_system(mesh, int(system)))


def mtp_mesh_set_curved_p2(mesh, nodes, ne):
    a = np.ascontiguousarray(nodes, dtype=np.float64)
    if a.shape != (ne, 6, 2):
        raise ValueError(f"curved nodes must have shape ({ne}, 6, 2), got {a.shape}")
    _check(load().mtp_mesh_set_curved_p2(mesh, _ptr(a)))


class Mesh:
    """system = MTP_SYSTEM_ACOUSTIC reads eps / mu as (kappa, rho) of linear acoustics."""

    def __init__(self, coords, cells, eps=None, mu=None, face_bc=None, system=MTP_SYSTEM_MAXWELL, curved=None):
        """curved: (ne, 6, 2) quadratic geometry nodes per triangle (mtp_mesh_set_curved_p2)."""
        self.h = mtp_mesh_create(coords, cells, eps, mu, face_bc)
        self.info = mtp_mesh_info(self.h)
        self.system = system
        if system != MTP_SYSTEM_MAXWELL:
            mtp_mesh_set_system(self.h, system)
        if curved is not None:
            mtp_mesh_set_curved_p2(self.h, curved, self.info["ne"])

    def __del__(self, _free=_release):   # bound at definition: safe at interpreter shutdown
        _free("mtp_mesh_destroy", getattr(self, "h", None))
        self.h = None


class Tents:
    def __init__(self, mesh, t_end, slope_fraction=0.5, t_start=0.0, rule=None):
        self.mesh = mesh
        if rule is None:
            self.h = mtp_pitch_layers(mesh.h, t_start, t_end, slope_fraction)
        else:
            self.h = mtp_pitch_layers_rule(mesh.h, t_start, t_end, slope_fraction, rule)
        r = C.c_int32()
        _check(load().mtp_tents_rule(self.h, C.byref(r)))
        self.rule = r.value   # the rule the table was pitched by (the chosen one for MTP_PITCH_AUTO)
        self.n_tents, self.n_layers, self.layer_ptr = mtp_tents_query(self.h)
        self.t_end = t_end

    def export(self):
        return mtp_tents_export(self.h)

    def dag(self):
        return mtp_tents_dag(self.mesh.h, self.h)

    def __del__(self, _free=_release):   # bound at definition: safe at interpreter shutdown
        _free("mtp_tents_destroy", getattr(self, "h", None))
        self.h = None


class Solver:
    """Device state of one solve.  The workspace is a torch uint8 tensor on `device`;
    work is enqueued on torch's current stream of that device (or `stream`)."""

    def __init__(self, mesh, tents, p, q, m, alpha=0.5, precision=MTP_FP64, device="cuda:0", stream=None):
        import torch
        self.mesh, self.tents, self.p, self.q, self.m = mesh, tents, p, q, m
        d = mesh.info["dim"]
        self.dim = d
        self.nc = d + 1 if mesh.system == MTP_SYSTEM_ACOUSTIC else (6 if d == 3 else 3)
        self.np = (p + 1) * (p + 2) // 2 if d == 2 else (p + 1) * (p + 2) * (p + 3) // 6
        self.shape = (mesh.info["ne"], self.np, self.nc)
        nbytes = mtp_solver_workspace_size(mesh.h, tents.h, p, q, m, precision)
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = mtp_solver_create(mesh.h, tents.h, p, q, m, precision, alpha, self.workspace.data_ptr(),
                                   nbytes, self.stream.cuda_stream)

    def node_coords(self):
        return mtp_node_coords(self.h, self.shape[0], self.np, self.dim)

    def set_fields(self, nodal, t0=0.0):
        mtp_set_fields(self.h, nodal, self.shape, t0)

    def set_planewave_bc(self, amp, kvec, omega, phase):
        mtp_set_planewave_bc(self.h, amp, kvec, omega, phase, self.nc, self.dim)

    def layer_advance(self, layer):
        mtp_layer_advance(self.h, layer)

    def advance_to(self, T):
        mtp_advance_to(self.h, T)

    def advance_to_static(self, T):
        mtp_advance_to_static(self.h, T)

    def front(self):
        return mtp_front(self.h)

    def get_fields(self, out=None):
        return mtp_get_fields(self.h, self.shape, out)

    def get_state(self, out=None):
        return mtp_get_state(self.h, self.shape, out)

    def slab_dof_updates(self):
        return mtp_slab_dof_updates(self.h)

    def slab_flops(self):
        return mtp_slab_flops(self.h)

    def kernel(self):
        return mtp_solver_kernel(self.h)

    def set_graph(self, on):
        mtp_solver_set_graph(self.h, int(bool(on)))

    def set_schedule(self, schedule):
        mtp_solver_set_schedule(self.h, schedule)

    def set_dag_wait(self, seconds):
        mtp_solver_set_dag_wait(self.h, seconds)

    def set_method(self, method):
        mtp_solver_set_method(self.h, method)

    def set_flux(self, flux):
        mtp_solver_set_flux(self.h, flux)

    def stats(self):
        return mtp_stats(self.h)

    def checkpoint_write(self, path):
        mtp_checkpoint_write(self.h, path)

    def checkpoint_read(self, path):
        mtp_checkpoint_read(self.h, path)

    def set_tuning(self, schedule, tile_order=MTP_TILES_DEFAULT, grid_frac=1.0):
        mtp_solver_set_tuning(self.h, schedule, tile_order, grid_frac)

    def tuning(self):
        return mtp_solver_get_tuning(self.h)

    def tune(self, slabs_per_trial=2):
        return mtp_solver_tune(self.h, slabs_per_trial)

    def __del__(self, _free=_release):   # bound at definition: safe at interpreter shutdown
        _free("mtp_solver_destroy", getattr(self, "h", None))
        self.h = None


class Batch:
    """Solvers advanced together, one launch per layer index across all of them."""

    def __init__(self, solvers, device="cuda:0", stream=None):
        import torch
        self.solvers = list(solvers)
        nbytes = mtp_batch_workspace_size(self.solvers)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=torch.device(device))
        self.stream = stream if stream is not None else torch.cuda.current_stream(torch.device(device))
        self.h = mtp_batch_create(self.solvers, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)

    def advance(self, n_slabs=1):
        mtp_batch_advance(self.h, n_slabs)

    def set_graph(self, on):
        mtp_batch_set_graph(self.h, int(bool(on)))

    def set_schedule(self, schedule):
        mtp_batch_set_schedule(self.h, schedule)

    def set_tuning(self, schedule, tile_order=MTP_TILES_DEFAULT, grid_frac=1.0):
        mtp_batch_set_tuning(self.h, schedule, tile_order, grid_frac)

    def tuning(self):
        return mtp_batch_get_tuning(self.h)

    def tune(self, slabs_per_trial=2):
        return mtp_batch_tune(self.h, slabs_per_trial)

    def __del__(self, _free=_release):   # bound at definition: safe at interpreter shutdown
        _free("mtp_batch_destroy", getattr(self, "h", None))
        self.h = None
