"""GPU parity of the impedance-matched upwind flux (the material-jump variant): the HIP
path against the oracle run with the same flux, element by element (relative L2 <= 1e-10
in FP64 under both schedules, <= 1e-6 on the mixed path)."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from parity import assert_parity, rel  # noqa: E402
from cases import DATA, IMP_CASES, planewave_params, setup  # noqa: E402

pytestmark = pytest.mark.gpu




def fixture(name):
    path = os.path.join(HERE, "golden", f"oracle_{name}.npz")
    if os.path.exists(path):
        return np.load(path)
    pytest.skip(f"missing oracle fixture {path}")


def run(name, precision, schedule):
    from paper_1906_11029_amd import mtp
    c, mm, dim, eps, mu, bc, ex, u0 = setup(name)
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc)
    T = mtp.Tents(M, c["T"], 0.5)
    S = mtp.Solver(M, T, c["p"], c["q"], c["m"], alpha=c["alpha"], precision=precision)
    S.set_flux(mtp.MTP_FLUX_IMPEDANCE)
    S.set_schedule(schedule)
    S.set_fields(u0, 0.0)
    if c["kind"] == DATA:
        S.set_planewave_bc(*planewave_params(ex, dim))
    S.advance_to(c["slabs"] * c["T"])
    return S


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("name", list(IMP_CASES))
def test_impedance_flux_parity_fp64(name, schedule):
    print(f"[gpu flux] {name} fp64 schedule {schedule}", flush=True)
    ref = fixture(name)
    S = run(name, 0, schedule)
    assert_parity(S.get_state(), ref["w"], 1e-10, name)
    assert_parity(S.get_fields(), ref["u"], 1e-10, name)


@pytest.mark.parametrize("name", list(IMP_CASES))
def test_impedance_flux_parity_mixed(name):
    print(f"[gpu flux] {name} mixed", flush=True)
    ref = fixture(name)
    S = run(name, 1, 1)
    assert_parity(S.get_state(), ref["w"], 1e-6, name)


def test_impedance_flux_rejected_on_vector_alu_kernel():
    from paper_1906_11029_amd import mtp
    c, mm, dim, eps, mu, bc, ex, u0 = setup("te_pec_p2_eps_imp")
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc)
    T = mtp.Tents(M, c["T"], 0.5)
    S = mtp.Solver(M, T, c["p"], c["q"], c["m"], precision=mtp.MTP_FP64_VALU)
    with pytest.raises(mtp.MTPError) as e:
        S.set_flux(mtp.MTP_FLUX_IMPEDANCE)
    assert e.value.code == -9
