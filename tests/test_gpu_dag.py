"""GPU checks of the persistent DAG schedule (one launch per slab; workgroups take tents
from a device queue as their dependencies complete).  Every tent computes the same values
from the same inputs in either schedule, so the states must be bit-identical to the
layer schedule; the oracle parity of the layer schedule then carries over.  The failure
path (a wait for a released tent exceeding its bound) is forced from the host with a
zero bound: every workgroup must leave and the read-out must report the device error."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from cases import DATA, planewave_params, setup  # noqa: E402

pytestmark = pytest.mark.gpu


def solver(name, precision, schedule, graph=True, slabs=None):
    from paper_1906_11029_amd import mtp
    c, mm, dim, eps, mu, bc, ex, u0 = setup(name)
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc)
    T = mtp.Tents(M, c["T"], 0.5)
    S = mtp.Solver(M, T, c["p"], c["q"], c["m"], alpha=c["alpha"], precision=precision)
    S.set_fields(u0, 0.0)
    if c["kind"] == DATA:
        S.set_planewave_bc(*planewave_params(ex, dim))
    S.set_schedule(schedule)
    S.set_graph(graph)
    S.advance_to((slabs or max(2, c["slabs"])) * c["T"])
    return S


CASES = ["te_planewave_p2", "te_pmc_p5", "cav3d_p3", "cav3d_p4", "planewave3d_p2", "graded3d_p3_eps",
         "single_tet_p3"]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", CASES)
def test_dag_schedule_bit_identical_to_layers(name, precision):
    from paper_1906_11029_amd import mtp
    print(f"[gpu dag] {name} precision {precision}", flush=True)
    ref = solver(name, precision, mtp.MTP_SCHEDULE_LAYERS).get_state()
    got = solver(name, precision, mtp.MTP_SCHEDULE_DAG).get_state()
    assert np.array_equal(got, ref)


def test_dag_schedule_eager_and_graph_agree_over_slabs():
    from paper_1906_11029_amd import mtp
    print("[gpu dag] graded3d_p3_eps eager vs graph, 3 slabs", flush=True)
    a = solver("graded3d_p3_eps", 0, mtp.MTP_SCHEDULE_DAG, graph=False, slabs=3).get_state()
    b = solver("graded3d_p3_eps", 0, mtp.MTP_SCHEDULE_DAG, graph=True, slabs=3).get_state()
    c = solver("graded3d_p3_eps", 0, mtp.MTP_SCHEDULE_LAYERS, graph=True, slabs=3).get_state()
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_dag_schedule_switch_mid_run():
    """Layers for one slab, the persistent schedule for the next: same as layers only."""
    from paper_1906_11029_amd import mtp
    print("[gpu dag] cav3d_p3 schedule switch", flush=True)
    c, mm, dim, eps, mu, bc, ex, u0 = setup("cav3d_p3")
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc)
    T = mtp.Tents(M, c["T"], 0.5)
    S = mtp.Solver(M, T, c["p"], c["q"], c["m"], alpha=c["alpha"])
    S.set_fields(u0, 0.0)
    S.advance_to(c["T"])
    S.set_schedule(mtp.MTP_SCHEDULE_DAG)
    S.advance_to(2 * c["T"])
    ref = solver("cav3d_p3", 0, mtp.MTP_SCHEDULE_LAYERS, slabs=2).get_state()
    assert np.array_equal(S.get_state(), ref)


def test_dag_schedule_rejected_for_vector_alu_kernel():
    from paper_1906_11029_amd import mtp
    c, mm, dim, eps, mu, bc, ex, u0 = setup("cav3d_p2")
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc)
    T = mtp.Tents(M, c["T"], 0.5)
    S = mtp.Solver(M, T, c["p"], c["q"], c["m"], precision=mtp.MTP_FP64_VALU)
    with pytest.raises(mtp.MTPError) as e:
        S.set_schedule(mtp.MTP_SCHEDULE_DAG)
    assert e.value.code == -9


def test_dag_wait_bound_aborts_the_slab():
    """Zero wait bound: a workgroup that finds its queue slot empty gives up at once and
    raises the abort word; every workgroup leaves, and the read-out reports it."""
    from paper_1906_11029_amd import mtp
    print("[gpu dag] forced wait bound", flush=True)
    c, mm, dim, eps, mu, bc, ex, u0 = setup("cav3d_p3")
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc)
    T = mtp.Tents(M, c["T"], 0.5)
    assert T.dag()["n_ready"] < T.n_tents // 4
    S = mtp.Solver(M, T, c["p"], c["q"], c["m"])
    S.set_fields(u0, 0.0)
    S.set_schedule(mtp.MTP_SCHEDULE_DAG)
    S.set_dag_wait(0.0)
    S.advance_to(c["T"])
    with pytest.raises(mtp.MTPError) as e:
        S.get_fields()
    assert e.value.code == -6 and "bound" in str(e.value)


def _pw_solver(n, p, q, m, T, theta, k, phase, precision):
    from mtp_inputs import fields, meshes
    from paper_1906_11029_amd import mtp
    mm = meshes.square_tri(n)
    bc = meshes.uniform_bc(len(mm["cells"]), 2, meshes.DATA)
    ex = fields.PlaneWaveTE(direction=(np.cos(theta), np.sin(theta)), k=k, phase=phase)
    M = mtp.Mesh(mm["coords"], mm["cells"], face_bc=bc)
    Tt = mtp.Tents(M, T, 0.5)
    S = mtp.Solver(M, Tt, p, q, m, precision=precision)
    S.set_fields(ex.u(meshes.equispaced_nodes(mm, p), 0.0))
    S.set_planewave_bc(*planewave_params(ex, 2))
    return S


@pytest.mark.parametrize("graph", [True, False])
@pytest.mark.parametrize("precision", [0, 1])
def test_batch_dag_equals_single_solves(precision, graph):
    """Solves on different meshes, plane waves, q and m in one persistent launch per slab
    (one queue over all their tent DAGs): bitwise equal to the solves run one by one."""
    from paper_1906_11029_amd import mtp
    print(f"[gpu dag] batch precision {precision} graph {graph}", flush=True)
    specs = [(5, 2, 3, 4, 0.3, 0.2, 6.0, 0.1), (9, 2, 3, 4, 0.3, 1.3, 9.0, 2.0),
             (3, 2, 4, 2, 0.25, 2.9, 4.0, 0.7), (7, 2, 3, 6, 0.2, 4.4, 7.5, 5.1)]
    single = [_pw_solver(*sp, precision) for sp in specs]
    batched = [_pw_solver(*sp, precision) for sp in specs]
    for S, sp in zip(single, specs):
        S.advance_to(3 * sp[4])
    B = mtp.Batch(batched)
    B.set_schedule(mtp.MTP_SCHEDULE_DAG)
    B.set_graph(graph)
    B.advance(2)
    B.advance(1)
    for S1, S2, sp in zip(single, batched, specs):
        assert S2.front() == (3 * sp[4], 0)
        assert np.array_equal(S1.get_state(), S2.get_state())


def test_batch_dag_3d_uneven_patches():
    """3D solves of one degree with different patch sizes (Kuhn cubes of 2 and 3 cells per
    side, graded with two materials) in one persistent batch: equal to the layer batch."""
    from paper_1906_11029_amd import mtp
    print("[gpu dag] batch 3d", flush=True)

    def make():
        out = []
        for nm in ("cav3d_p3", "graded3d_p3_eps", "single_tet_p3"):
            c, mm, dim, eps, mu, bc, ex, u0 = setup(nm)
            M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc)
            T = mtp.Tents(M, c["T"], 0.5)
            S = mtp.Solver(M, T, c["p"], c["q"], c["m"], alpha=c["alpha"], precision=1)
            S.set_fields(u0, 0.0)
            out.append(S)
        return out
    a, b = make(), make()
    Ba, Bb = mtp.Batch(a), mtp.Batch(b)
    Bb.set_schedule(mtp.MTP_SCHEDULE_DAG)
    Ba.advance(2)
    Bb.advance(2)
    for S1, S2 in zip(a, b):
        assert np.array_equal(S1.get_state(), S2.get_state())
