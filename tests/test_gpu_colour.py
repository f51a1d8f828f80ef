"""GPU parity of solves on tables of the colour pitching rule: the library pitches the same
table as the oracle (bit-exact), and the solve on it matches the oracle's FP64 solve element
by element (<= 1e-10), on both FP64 kernels, under the persistent schedule, in a batch, and
on the curved disk."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from cases import COLOUR_CASES, DATA, planewave_params, setup  # noqa: E402
from parity import assert_parity  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-10


def colour_solver(name, precision=0):
    from paper_1906_11029_amd import mtp
    c, mm, dim, eps, mu, bc, ex, u0 = setup(name)
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc, curved=mm.get("geo"))
    T = mtp.Tents(M, c["T"], 0.5, rule=mtp.MTP_PITCH_COLOUR)
    S = mtp.Solver(M, T, c["p"], c["q"], c["m"], alpha=c["alpha"], precision=precision)
    S.set_fields(u0, 0.0)
    if c["kind"] == DATA:
        S.set_planewave_bc(*planewave_params(ex, dim))
    return c, S, T


def fixture(name):
    path = os.path.join(HERE, "golden", f"oracle_{name}.npz")
    if os.path.exists(path):
        return np.load(path)
    pytest.skip(f"missing oracle fixture {path}")


@pytest.mark.parametrize("precision", [0, 2])
@pytest.mark.parametrize("name", list(COLOUR_CASES))
def test_colour_tables_against_oracle(name, precision):
    print(f"[gpu colour] {name} precision {precision}", flush=True)
    ref = fixture(name)
    c, S, T = colour_solver(name, precision)
    ex = T.export()
    for k in ("vertex", "t_top", "layer"):
        assert np.array_equal(ex[k], ref[k]), f"tent list differs in {k}"
    S.advance_to(c["slabs"] * c["T"])
    assert_parity(S.get_state(), ref["w"], TOL, f"{name} w")


@pytest.mark.parametrize("name", [n for n in COLOUR_CASES if not COLOUR_CASES[n].get("curved")])
def test_colour_tables_under_the_persistent_schedule(name):
    """The tent DAG of a colour table drains to the layer schedule's result bit for bit."""
    from paper_1906_11029_amd import mtp
    print(f"[gpu colour] {name} dag", flush=True)
    c, A, _ = colour_solver(name)
    _, B, _ = colour_solver(name)
    B.set_schedule(mtp.MTP_SCHEDULE_DAG)
    A.advance_to(c["T"])
    B.advance_to(c["T"])
    assert np.array_equal(A.get_state(), B.get_state())


def test_colour_tables_in_a_batch():
    from paper_1906_11029_amd import mtp
    names = ["disk_colour_p2", "te_planewave_p2_colour"]
    print("[gpu colour] batch", flush=True)
    solvers = [colour_solver(nm)[1] for nm in names]
    mtp.Batch(solvers).advance(1)
    for S, nm in zip(solvers, names):
        assert_parity(S.get_state(), fixture(nm)["w"], TOL, f"batch {nm}")


def test_colour_tables_stay_bounded_on_the_graded_p4_mesh():
    """The 32^3 x 6 Kuhn cube graded 1:8 toward a corner with eps in {1, 2.25}, P4, q = 5,
    m = 8, slab 0.05, Gaussian pulse: the colour table (with its pole cap) runs three slabs in
    FP64 and stays within the minimum-vertex table's solution (both approximate the same
    field).  Without the cap, poles of two edge steps next to the material jump grew the
    state by ~1e14 per slab on this mesh."""
    import torch
    from mtp_inputs import fields, meshes
    from paper_1906_11029_amd import mtp
    a = 2.0 / 9.0
    mm = meshes.cube_kuhn(32, axis_map=lambda g: a * g + (1 - a) * g * g)
    eps, mu = meshes.materials_split(mm)
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu)
    u0 = fields.GaussianPulse3D(seed=11030).u(meshes.equispaced_nodes(mm, 4), 0.0)
    out = {}
    for rule in (mtp.MTP_PITCH_MIN_VERTEX, mtp.MTP_PITCH_COLOUR):
        T = mtp.Tents(M, 0.05, 0.5, rule=rule)
        S = mtp.Solver(M, T, 4, 5, 8, precision=mtp.MTP_FP64)
        S.set_tuning(mtp.MTP_SCHEDULE_LAYERS)
        S.set_fields(u0, 0.0)
        w = torch.empty(S.shape, dtype=torch.float64, device="cuda")
        peaks = []
        for k in range(1, 4):
            S.advance_to(0.05 * k)
            S.get_fields(w)
            peaks.append(w.abs().max().item())
        print(f"[gpu colour] graded P4 rule {rule}: tents {T.n_tents} layers {T.n_layers} max|u| {peaks}", flush=True)
        out[rule] = (w.cpu().numpy(), peaks)
        del S
    (ua, pa), (ub, pb) = out[mtp.MTP_PITCH_MIN_VERTEX], out[mtp.MTP_PITCH_COLOUR]
    assert max(pb) < 1.5 * max(pa)
    diff = np.linalg.norm(ub - ua) / np.linalg.norm(ua)
    print(f"[gpu colour] colour vs minimum-vertex after 3 slabs: relative L2 {diff:.3e}", flush=True)
    assert diff < 1e-3


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("name", [n for n in COLOUR_CASES if not COLOUR_CASES[n].get("curved")])
def test_colour_tables_mixed_precision(name, schedule):
    """Mixed precision on colour tables, per-layer and persistent: the state against the
    oracle's FP64 solve within 1e-6, element by element."""
    from paper_1906_11029_amd import mtp
    print(f"[gpu colour] {name} mixed schedule {schedule}", flush=True)
    ref = fixture(name)
    c, S, T = colour_solver(name, mtp.MTP_MIXED_FP32)
    assert S.kernel() == 2
    S.set_schedule(schedule)
    S.advance_to(c["slabs"] * c["T"])
    assert_parity(S.get_state(), ref["w"], 1e-6, f"{name} mixed")
