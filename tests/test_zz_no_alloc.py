"""The allocation-free advance (mtp_advance_to_static, scratch in the library's static
device array) against the existing entry point it varies (mtp_advance_to on the persistent
schedule, scratch in the solver's workspace): bit for bit, on two calls in a row, the second
with a smaller input (fewer tents, so stale scratch from the first call would show), in both
precisions; the first call also against the oracle; and a slab too large for the array is
refused before anything is enqueued."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from cases import DATA, planewave_params, setup  # noqa: E402
from parity import assert_parity  # noqa: E402

pytestmark = pytest.mark.gpu


def _solver(name, precision):
    from paper_1906_11029_amd import mtp
    c, mm, dim, eps, mu, bc, ex, u0 = setup(name)
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc)
    T = mtp.Tents(M, c["T"], 0.5)
    S = mtp.Solver(M, T, c["p"], c["q"], c["m"], alpha=c["alpha"], precision=precision)
    S.set_fields(u0, 0.0)
    if c["kind"] == DATA:
        S.set_planewave_bc(*planewave_params(ex, dim))
    return c, S, T


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-6)])
def test_static_scratch_advance_equals_advance_to(precision, tol):
    from paper_1906_11029_amd import mtp
    sizes = []
    for k, name in enumerate(("graded3d_p3_eps", "cav3d_p2")):
        print(f"[gpu no-alloc] call {k + 1}: {name} precision {precision}", flush=True)
        c, ref, T = _solver(name, precision)
        ref.set_schedule(mtp.MTP_SCHEDULE_DAG)
        ref.advance_to(c["T"])
        c, got, T2 = _solver(name, precision)
        got.advance_to_static(c["T"])
        assert got.front() == (c["T"], 0)
        w = got.get_state()
        assert np.array_equal(w, ref.get_state())
        assert_parity(w, np.load(os.path.join(HERE, "golden", f"oracle_{name}.npz"))["w"], tol, name)
        sizes.append(T2.n_tents)
    assert sizes[1] < sizes[0]


def test_static_scratch_refuses_a_slab_beyond_the_array():
    """1.68 million tents per slab need 13.4 MB of scratch, more than the 8 MiB array:
    refused with MTP_ERR_UNSUPPORTED, front unchanged."""
    from mtp_inputs import fields, meshes
    from paper_1906_11029_amd import mtp
    print("[gpu no-alloc] oversized slab refused", flush=True)
    mm = meshes.square_tri(200)
    M = mtp.Mesh(mm["coords"], mm["cells"], face_bc=meshes.uniform_bc(len(mm["cells"]), 2, meshes.PMC))
    T = mtp.Tents(M, 0.05, 0.5)
    assert T.n_tents * 8 > (8 << 20)
    S = mtp.Solver(M, T, 1, 2, 2)
    S.set_fields(fields.CavityTE_PEC().u(meshes.equispaced_nodes(mm, 1), 0.0))
    with pytest.raises(mtp.MTPError) as e:
        S.advance_to_static(0.05)
    assert e.value.code == -9 and "static array" in str(e.value)
    assert S.front() == (0.0, 0)
