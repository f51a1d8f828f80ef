"""GPU parity of the second system, linear acoustics u = (p, v) (the method as stated for
linear hyperbolic systems in conservation form): the HIP path against the oracle on the
same tents, element by element (FP64 <= 1e-10 in both schedules, mixed <= 1e-6), rigid and
pressure-release walls, plane-wave data, two media with the impedance-matched flux; and
the h-convergence rate p + 1 of SAT on the rigid-wall cavity at GPU sizes."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from parity import assert_parity, rel  # noqa: E402
from cases import AC_CASES, DATA, planewave_params, setup  # noqa: E402

pytestmark = pytest.mark.gpu




def fixture(name):
    path = os.path.join(HERE, "golden", f"oracle_{name}.npz")
    if os.path.exists(path):
        return np.load(path)
    pytest.skip(f"missing oracle fixture {path}")


def make(name, precision):
    from paper_1906_11029_amd import mtp
    c, mm, dim, eps, mu, bc, ex, u0 = setup(name)
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc, system=mtp.MTP_SYSTEM_ACOUSTIC)
    T = mtp.Tents(M, c["T"], 0.5)
    S = mtp.Solver(M, T, c["p"], c["q"], c["m"], alpha=c["alpha"], precision=precision)
    if c["flux"] == "impedance":
        S.set_flux(mtp.MTP_FLUX_IMPEDANCE)
    S.set_fields(u0, 0.0)
    if c["kind"] == DATA:
        S.set_planewave_bc(*planewave_params(ex, dim))
    return c, S, T


def run(name, precision, schedule):
    c, S, T = make(name, precision)
    S.set_schedule(schedule)
    S.advance_to(c["slabs"] * c["T"])
    return S, T


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("name", list(AC_CASES))
def test_acoustic_parity_fp64(name, schedule):
    print(f"[gpu acoustic] {name} fp64 schedule {schedule}", flush=True)
    ref = fixture(name)
    S, T = run(name, 0, schedule)
    ex = T.export()
    for k in ("vertex", "t_top", "layer"):
        assert np.array_equal(ex[k], ref[k]), k
    assert_parity(S.get_state(), ref["w"], 1e-10, name)
    assert_parity(S.get_fields(), ref["u"], 1e-10, name)


@pytest.mark.parametrize("name", list(AC_CASES))
def test_acoustic_parity_mixed(name):
    print(f"[gpu acoustic] {name} mixed", flush=True)
    ref = fixture(name)
    S, _ = run(name, 1, 1)
    assert_parity(S.get_state(), ref["w"], 1e-6, name)


def test_acoustic_cavity_convergence_at_scale():
    from mtp_inputs import fields, meshes
    from paper_1906_11029_amd import mtp
    p, errs = 3, []
    for n in (8, 16, 32):
        mm = meshes.square_tri(n)
        M = mtp.Mesh(mm["coords"], mm["cells"], face_bc=meshes.uniform_bc(len(mm["cells"]), 2, meshes.PMC),
                     system=mtp.MTP_SYSTEM_ACOUSTIC)
        T = mtp.Tents(M, 0.5, 0.5)
        S = mtp.Solver(M, T, p, p + 1, 2 * p)
        S.set_schedule(mtp.MTP_SCHEDULE_DAG)
        ex = fields.AcousticCavity(2)
        nodes = meshes.equispaced_nodes(mm, p)
        S.set_fields(ex.u(nodes, 0.0), 0.0)
        S.advance_to(0.5)
        errs.append(rel(S.get_fields(), ex.u(nodes, 0.5)))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print(f"[gpu acoustic] P{p} rigid cavity errors {errs} rates {rates}", flush=True)
    assert min(rates) > p + 1 - 0.5


def test_acoustic_rejected_where_unsupported():
    from paper_1906_11029_amd import mtp
    c, mm, dim, eps, mu, bc, ex, u0 = setup("ac3d_rigid_p2")
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc, system=mtp.MTP_SYSTEM_ACOUSTIC)
    T = mtp.Tents(M, c["T"], 0.5)
    S = mtp.Solver(M, T, c["p"], c["q"], c["m"], precision=mtp.MTP_MIXED_FP32)
    with pytest.raises(mtp.MTPError):   # RK4 runs on the FP64 kernel only
        S.set_method(mtp.MTP_METHOD_RK4)
    with pytest.raises(mtp.MTPError):   # acoustics has no vector-ALU kernel
        mtp.Solver(M, T, c["p"], c["q"], c["m"], precision=mtp.MTP_FP64_VALU)


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-6)])
@pytest.mark.parametrize("dim", [2, 3])
def test_acoustic_batches_against_oracle(dim, precision, tol, schedule):
    """The acoustic cases of one dimension (3D: P2, P3, P4 groups; rigid and pressure-release
    walls, two media, the impedance flux; 2D: P3 rigid walls and P2 plane-wave data) advanced
    as one batch, per-layer or persistent, against the oracle's fixtures."""
    from paper_1906_11029_amd import mtp
    names = [n for n in AC_CASES if n.startswith(f"ac{dim}d")]
    print(f"[gpu acoustic] batch {dim}D precision {precision} schedule {schedule}: {names}", flush=True)
    made = [make(n, precision) for n in names]
    B = mtp.Batch([S for _, S, _ in made])
    B.set_schedule(schedule)
    B.advance(1)
    for (c, S, _), n in zip(made, names):
        assert c["slabs"] == 1
        assert_parity(S.get_state(), fixture(n)["w"], tol, f"batch {n}")


def test_batches_refuse_mixed_systems():
    from paper_1906_11029_amd import mtp
    _, A, _ = make("ac3d_rigid_p2", 0)
    c, mm, dim, eps, mu, bc, ex, u0 = setup("ac3d_rigid_p2")
    M = mtp.Mesh(mm["coords"], mm["cells"])
    S = mtp.Solver(M, mtp.Tents(M, c["T"], 0.5), 2, 3, 4)
    with pytest.raises(mtp.MTPError) as e:
        mtp.Batch([A, S])
    assert e.value.code == -9


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("name", ["ac2d_rigid_p3_rk4", "ac3d_release_eps_p3_rk4"])
def test_acoustic_rk4_against_oracle(name, schedule):
    """Linear acoustics under the classical RK4 variant (FP64 matrix-core kernel), per-layer
    and persistent, against the oracle's RK4 solve: element by element <= 1e-10."""
    from paper_1906_11029_amd import mtp
    print(f"[gpu acoustic] {name} schedule {schedule}", flush=True)
    ref = fixture(name)
    c, S, T = make(name, 0)
    S.set_method(mtp.MTP_METHOD_RK4)
    S.set_schedule(schedule)
    S.advance_to(c["slabs"] * c["T"])
    assert_parity(S.get_state(), ref["w"], 1e-10, name)
    assert_parity(S.get_fields(), ref["u"], 1e-10, name)
