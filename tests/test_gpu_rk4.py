"""GPU checks of the classical RK4 variant (the naive time stepping of the mapped system
that the paper contrasts with SAT, section 4): element-by-element parity with the
oracle's RK4 on the same tents (relative L2 <= 1e-10, FP64), both schedules, alone and in
batches; and, at
sizes the oracle would take long for, the order loss itself: on the 2D PMC cavity at
P4, SAT keeps the h-convergence rate p + 1 while RK4 falls clearly behind."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from parity import assert_parity, rel  # noqa: E402
from cases import DATA, RK4_CASES, planewave_params, setup  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-10




def fixture(name):
    path = os.path.join(HERE, "golden", f"oracle_{name}.npz")
    if os.path.exists(path):
        return np.load(path)
    pytest.skip(f"missing oracle fixture {path}")


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("name", list(RK4_CASES))
def test_rk4_parity_against_oracle(name, schedule):
    from paper_1906_11029_amd import mtp
    print(f"[gpu rk4] {name} schedule {schedule}", flush=True)
    ref = fixture(name)
    c, mm, dim, eps, mu, bc, ex, u0 = setup(name)
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc)
    T = mtp.Tents(M, c["T"], 0.5)
    S = mtp.Solver(M, T, c["p"], c["q"], c["m"], alpha=c["alpha"])
    S.set_method(mtp.MTP_METHOD_RK4)
    S.set_schedule(schedule)
    S.set_fields(u0, 0.0)
    if c["kind"] == DATA:
        S.set_planewave_bc(*planewave_params(ex, dim))
    S.advance_to(c["slabs"] * c["T"])
    assert_parity(S.get_state(), ref["w"], TOL, name)
    assert_parity(S.get_fields(), ref["u"], TOL, name)


def _cavity_error(n, p, method):
    from mtp_inputs import fields, meshes
    from paper_1906_11029_amd import mtp
    mm = meshes.square_tri(n, length=np.pi)
    ex = fields.CavityTE_PMC()
    M = mtp.Mesh(mm["coords"], mm["cells"], face_bc=meshes.uniform_bc(len(mm["cells"]), 2, meshes.PMC))
    T = mtp.Tents(M, 0.5, 0.5)
    S = mtp.Solver(M, T, p, p + 1, 2 * p)
    S.set_method(method)
    S.set_schedule(mtp.MTP_SCHEDULE_DAG)
    nodes = meshes.equispaced_nodes(mm, p)
    S.set_fields(ex.u(nodes, 0.0), 0.0)
    S.advance_to(0.5)
    return rel(S.get_fields(), ex.u(nodes, 0.5))


def test_rk4_loses_order_at_scale():
    from paper_1906_11029_amd import mtp
    p, ns = 4, (8, 16, 32)
    sat = [_cavity_error(n, p, mtp.MTP_METHOD_SAT) for n in ns]
    rk4 = [_cavity_error(n, p, mtp.MTP_METHOD_RK4) for n in ns]
    rs = [np.log2(sat[i] / sat[i + 1]) for i in range(2)]
    rr = [np.log2(rk4[i] / rk4[i + 1]) for i in range(2)]
    print(f"[gpu rk4] P{p} PMC cavity, n = {ns}: SAT errors {sat} rates {rs}; RK4 errors {rk4} rates {rr}",
          flush=True)
    assert min(rs) > p + 1 - 0.5
    assert rr[-1] < rs[-1] - 1.0
    assert rk4[-1] > 3 * sat[-1]


def test_rk4_rejected_where_unsupported():
    from paper_1906_11029_amd import mtp
    c, mm, dim, eps, mu, bc, ex, u0 = setup("cav3d_p2_rk4")
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc)
    T = mtp.Tents(M, c["T"], 0.5)
    S = mtp.Solver(M, T, c["p"], c["q"], c["m"], precision=mtp.MTP_MIXED_FP32)
    with pytest.raises(mtp.MTPError) as e:
        S.set_method(mtp.MTP_METHOD_RK4)
    assert e.value.code == -9
    # a batch runs one method: SAT and RK4 solvers do not mix, and a member that changes its
    # method after the batch was made stops the batch
    S2 = mtp.Solver(M, T, c["p"], c["q"], c["m"])
    S2.set_method(mtp.MTP_METHOD_RK4)
    S3 = mtp.Solver(M, T, c["p"], c["q"], c["m"])
    with pytest.raises(mtp.MTPError) as e:
        mtp.Batch([S2, S3])
    assert e.value.code == -9
    B = mtp.Batch([S2])
    S2.set_method(mtp.MTP_METHOD_SAT)
    with pytest.raises(mtp.MTPError):
        B.advance(1)


# batches of RK4 solvers (one system each; degree groups where the degrees differ)
RK4_BATCHES = {"maxwell2d": ["te_planewave_p2_rk4", "te_pmc_p3_rk4", "te_pec_p2_eps_rk4"],
               "maxwell3d": ["cav3d_p2_rk4", "delaunay3d_p4_rk4"],
               "acoustic2d": ["ac2d_rigid_p3_rk4"],
               "acoustic3d": ["ac3d_release_eps_p3_rk4"]}


def _rk4_solver(name):
    from paper_1906_11029_amd import mtp
    c, mm, dim, eps, mu, bc, ex, u0 = setup(name)
    system = mtp.MTP_SYSTEM_ACOUSTIC if c["system"] == "acoustic" else mtp.MTP_SYSTEM_MAXWELL
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc, system=system)
    T = mtp.Tents(M, c["T"], 0.5)
    S = mtp.Solver(M, T, c["p"], c["q"], c["m"], alpha=c["alpha"])
    S.set_method(mtp.MTP_METHOD_RK4)
    S.set_fields(u0, 0.0)
    if c["kind"] == DATA:
        S.set_planewave_bc(*planewave_params(ex, dim))
    return S


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("batch", list(RK4_BATCHES))
def test_rk4_batches_against_oracle(batch, schedule):
    """RK4 solvers advanced one slab together in a batch (per-layer launches or one persistent
    launch per degree group) against the oracle's RK4 fixtures, element by element."""
    from paper_1906_11029_amd import mtp
    names = RK4_BATCHES[batch]
    print(f"[gpu rk4] batch {batch} ({', '.join(names)}) schedule {schedule}", flush=True)
    refs = [fixture(n) for n in names]
    solvers = [_rk4_solver(n) for n in names]
    B = mtp.Batch(solvers)
    B.set_schedule(schedule)
    B.advance(1)
    for S, n, ref in zip(solvers, names, refs):
        assert_parity(S.get_state(), ref["w"], TOL, f"batch {batch}: {n}")
