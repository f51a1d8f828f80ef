"""Full-size checks on the benchmark workloads: 32^3 x 6 Kuhn tets (196608) graded toward
one corner, and the jittered Delaunay cube (226989 tets, vertex patches up to 44: the 48-tet
P4 class), eps in {1, 2.25} split at x = 0.5, Gaussian-pulse E, P4, q = 5, m = 8, slab 0.05
(Delaunay: 0.01).  (1) Sampled tents of a mid-slab layer against the oracle started from
the GPU's state before that layer (FP64 <= 1e-10, mixed <= 1e-6), every element outside the
layer's patches untouched.  (2) One whole slab in the persistent DAG schedule (captured slab
graph) equals the per-layer launches bitwise, for both precisions."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from parity import assert_parity  # noqa: E402

pytestmark = pytest.mark.gpu
GRADE_A = 2.0 / 9.0


def _workload():
    from mtp_inputs import fields, meshes
    mm = meshes.cube_kuhn(32, axis_map=lambda g: GRADE_A * g + (1 - GRADE_A) * g * g)
    eps, mu = meshes.materials_split(mm)
    u0 = fields.GaussianPulse3D(seed=11030).u(meshes.equispaced_nodes(mm, 4), 0.0)
    return mm, eps, mu, u0


def _solver(mm, eps, mu, u0, precision, M=None, T=None):
    from paper_1906_11029_amd import mtp
    if M is None:
        M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu)
        T = mtp.Tents(M, 0.05, 0.5)
    S = mtp.Solver(M, T, 4, 5, 8, precision=precision)
    S.set_fields(u0, 0.0)
    return M, T, S


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-6)])
def test_full_size_p4_sampled_tents(precision, tol):
    from oracle.mesh import Mesh as OMesh
    from oracle.solve import OracleSolver
    print(f"[gpu full-size P4] sampled tents, precision {precision}", flush=True)
    mm, eps, mu, u0 = _workload()
    M, T, S = _solver(mm, eps, mu, u0, precision)
    L = T.n_layers // 2
    for layer in range(L):
        S.layer_advance(layer)
    w_before = S.get_state()
    S.layer_advance(L)
    w_after = S.get_state()
    tl = T.export()
    tau = np.zeros(M.info["nv"])
    sel = tl["layer"] < L
    tau[tl["vertex"][sel]] = tl["t_top"][sel]
    om = OMesh(mm["coords"], mm["cells"], eps=eps, mu=mu)
    O = OracleSolver(om, 4, 5, 8)
    O.set_nodal_w(w_before)
    O.tau[:] = tau
    idx = np.arange(T.layer_ptr[L], T.layer_ptr[L + 1])
    # 6 random tents of the layer, plus the first two whose patch has a PEC wall face
    # (their vertex lies on the boundary) and the first whose patch holds both media
    rng = np.random.default_rng(1)
    pick = list(rng.choice(idx, size=6, replace=False))
    xv = mm["coords"][tl["vertex"][idx]]
    on_wall = idx[np.any((xv < 1e-12) | (xv > 1 - 1e-12), axis=1)]
    on_jump = idx[[len(np.unique(eps[om.v2e[int(tl["vertex"][i])]])) == 2 for i in idx]]
    pick += [i for i in on_wall[:2] if i not in pick] + [i for i in on_jump[:1] if i not in pick]
    assert len(on_wall) >= 2 and len(on_jump) >= 1
    for i in pick:
        O.run_tent(int(tl["vertex"][i]), float(tl["t_top"][i]))
    w_or = O.nodal_w()
    for i in pick:
        es = om.v2e[int(tl["vertex"][i])]
        assert_parity(w_after[es], w_or[es], tol, f"tent {i}")
    touched = np.unique(np.concatenate([om.v2e[int(v)] for v in tl["vertex"][idx]]))
    mask = np.ones(len(w_after), bool)
    mask[touched] = False
    assert np.array_equal(w_after[mask], w_before[mask])


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_p4_dag_slab_equals_layers(precision):
    from paper_1906_11029_amd import mtp
    print(f"[gpu full-size P4] persistent slab vs layers, precision {precision}", flush=True)
    mm, eps, mu, u0 = _workload()
    M, T, A = _solver(mm, eps, mu, u0, precision)
    _, _, B = _solver(mm, eps, mu, u0, precision, M, T)
    A.set_schedule(mtp.MTP_SCHEDULE_DAG)
    A.advance_to(0.05)
    B.set_graph(False)
    for layer in range(T.n_layers):
        B.layer_advance(layer)
    wa, wb = A.get_state(), B.get_state()
    assert np.all(np.isfinite(wa))
    assert np.array_equal(wa, wb)


def _delaunay():
    from mtp_inputs import fields, meshes
    mm = meshes.graded_delaunay_cube()
    eps, mu = meshes.materials_split(mm)
    u0 = fields.GaussianPulse3D(seed=11030).u(meshes.equispaced_nodes(mm, 4), 0.0)
    return mm, eps, mu, u0


def _delaunay_solver(mm, eps, mu, u0, precision, M=None, T=None):
    from paper_1906_11029_amd import mtp
    if M is None:
        M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu)
        T = mtp.Tents(M, 0.01, 0.5, rule=mtp.MTP_PITCH_MIN_VERTEX)
    S = mtp.Solver(M, T, 4, 5, 8, precision=precision)
    S.set_fields(u0, 0.0)
    return M, T, S


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-6)])
def test_full_size_delaunay_p4_sampled_tents(precision, tol):
    """The Delaunay workload: a mid-slab layer holding a tent of more than 36 tets, a tent at
    a PEC wall and one across the material jump; 5 random tents of it and those three
    against the oracle."""
    from oracle.mesh import Mesh as OMesh
    from oracle.solve import OracleSolver
    print(f"[gpu full-size Delaunay P4] sampled tents, precision {precision}", flush=True)
    mm, eps, mu, u0 = _delaunay()
    M, T, S = _delaunay_solver(mm, eps, mu, u0, precision)
    assert M.info["max_patch"] > 36
    tl = T.export()
    om = OMesh(mm["coords"], mm["cells"], eps=eps, mu=mu)
    psize = np.array([len(om.v2e[int(v)]) for v in tl["vertex"]])
    xv_all = mm["coords"][tl["vertex"]]
    wall_all = np.any((xv_all < 1e-12) | (xv_all > 1 - 1e-12), axis=1)
    # the first layer from mid-slab on with a large patch, a wall tent and a jump tent
    L = T.n_layers // 2
    while True:
        idx = np.arange(T.layer_ptr[L], T.layer_ptr[L + 1])
        big = idx[psize[idx] > 36]
        on_wall = idx[wall_all[idx]]
        on_jump = idx[[len(np.unique(eps[om.v2e[int(tl["vertex"][i])]])) == 2 for i in idx]]
        if len(big) and len(on_wall) and len(on_jump):
            break
        L += 1
    print(f"[gpu full-size Delaunay P4] layer {L} of {T.n_layers}, {len(idx)} tents", flush=True)
    for layer in range(L):
        S.layer_advance(layer)
    w_before = S.get_state()
    S.layer_advance(L)
    w_after = S.get_state()
    tau = np.zeros(M.info["nv"])
    sel = tl["layer"] < L
    tau[tl["vertex"][sel]] = tl["t_top"][sel]
    O = OracleSolver(om, 4, 5, 8)
    O.set_nodal_w(w_before)
    O.tau[:] = tau
    rng = np.random.default_rng(2)
    pick = list(rng.choice(idx, size=min(5, len(idx)), replace=False))
    pick += [i for i in (big[0], on_wall[0], on_jump[0]) if i not in pick]
    for i in pick:
        O.run_tent(int(tl["vertex"][i]), float(tl["t_top"][i]))
    w_or = O.nodal_w()
    for i in pick:
        es = om.v2e[int(tl["vertex"][i])]
        assert_parity(w_after[es], w_or[es], tol, f"tent {i} ({len(es)} tets)")
    touched = np.unique(np.concatenate([om.v2e[int(v)] for v in tl["vertex"][idx]]))
    mask = np.ones(len(w_after), bool)
    mask[touched] = False
    assert np.array_equal(w_after[mask], w_before[mask])


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_delaunay_p4_dag_slab_equals_layers(precision):
    from paper_1906_11029_amd import mtp
    print(f"[gpu full-size Delaunay P4] persistent slab vs layers, precision {precision}", flush=True)
    mm, eps, mu, u0 = _delaunay()
    M, T, A = _delaunay_solver(mm, eps, mu, u0, precision)
    _, _, B = _delaunay_solver(mm, eps, mu, u0, precision, M, T)
    A.set_schedule(mtp.MTP_SCHEDULE_DAG)
    A.advance_to(0.01)
    B.set_graph(False)
    for layer in range(T.n_layers):
        B.layer_advance(layer)
    wa, wb = A.get_state(), B.get_state()
    assert np.all(np.isfinite(wa))
    assert np.array_equal(wa, wb)


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-6)])
def test_full_size_delaunay_p4_layers_wider_than_the_slots(precision, tol):
    """The Delaunay cube on colour tables over a short slab (0.0005: layers of up to 5765
    tents): the 48-tet class's per-layer launches run at most 1024 workgroups (one F/R slot
    each), so a workgroup takes several tents of a wide layer.  One slab equals the persistent
    schedule bitwise, and so does the slab run as a batch (per-layer and persistent); in the
    widest layer, tents at positions 1024, 2047 and the last (a workgroup's second and later
    tents) against the oracle."""
    from oracle.mesh import Mesh as OMesh
    from oracle.solve import OracleSolver
    from paper_1906_11029_amd import mtp
    print(f"[gpu full-size Delaunay P4] colour tables, wide layers, precision {precision}", flush=True)
    mm, eps, mu, u0 = _delaunay()
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu)
    T = mtp.Tents(M, 0.0005, 0.5, rule=mtp.MTP_PITCH_COLOUR)
    width = np.diff(T.layer_ptr)
    L = int(np.argmax(width))
    assert width[L] > 2048
    _, _, A = _delaunay_solver(mm, eps, mu, u0, precision, M, T)
    _, _, B = _delaunay_solver(mm, eps, mu, u0, precision, M, T)
    A.set_schedule(mtp.MTP_SCHEDULE_DAG)
    A.advance_to(0.0005)
    B.set_graph(False)
    for layer in range(L):
        B.layer_advance(layer)
    w_before = B.get_state()
    B.layer_advance(L)
    w_after = B.get_state()
    for layer in range(L + 1, T.n_layers):
        B.layer_advance(layer)
    assert np.array_equal(A.get_state(), B.get_state())
    # the same slab as a batch (its own slots; per-layer launches of up to 5765 tents on at
    # most 1024 workgroups, and the persistent schedule)
    for schedule in (mtp.MTP_SCHEDULE_LAYERS, mtp.MTP_SCHEDULE_DAG):
        _, _, C = _delaunay_solver(mm, eps, mu, u0, precision, M, T)
        Bt = mtp.Batch([C])
        Bt.set_schedule(schedule)
        Bt.advance(1)
        assert np.array_equal(C.get_state(), A.get_state()), f"batch, schedule {schedule}"
        del Bt, C
    tl = T.export()
    om = OMesh(mm["coords"], mm["cells"], eps=eps, mu=mu)
    tau = np.zeros(M.info["nv"])
    sel = tl["layer"] < L
    tau[tl["vertex"][sel]] = tl["t_top"][sel]
    O = OracleSolver(om, 4, 5, 8)
    O.set_nodal_w(w_before)
    O.tau[:] = tau
    first = int(T.layer_ptr[L])
    pick = [first + 1024, first + 2047, int(T.layer_ptr[L + 1]) - 1]
    for i in pick:
        O.run_tent(int(tl["vertex"][i]), float(tl["t_top"][i]))
    w_or = O.nodal_w()
    for i in pick:
        es = om.v2e[int(tl["vertex"][i])]
        assert_parity(w_after[es], w_or[es], tol, f"tent {i - first} of layer {L} ({len(es)} tets)")
