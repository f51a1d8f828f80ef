"""Write the oracle's results for the parity cases to tests/golden/oracle_<case>.npz.

Calls only the oracle and the shared input generators.  Usage:
    python tests/golden/make_oracle_fixtures.py [case ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

from cases import (AC_CASES, AC_RK4_CASES, CASES, COLOUR_CASES, CURVED_CASES, DATA, IMP_CASES,  # noqa: E402
                   LARGE_P4_CASES, RK4_CASES, setup)
from oracle import curved  # noqa: E402
from oracle.mesh import Mesh  # noqa: E402
from oracle.pitch import pitch  # noqa: E402
from oracle.solve import OracleSolver  # noqa: E402


def make_curved(name):
    """Quadratic boundary triangles: the oracle's weight-adjusted curved tent solve."""
    c, mm, dim, eps, mu, bc, ex, u0 = setup(name)
    cm = curved.CurvedMesh(mm["coords"], mm["cells"], mm["geo"], eps=eps, mu=mu, face_bc=bc)
    tents = pitch(cm.base, c["T"], 0.5, k_elem=cm.step_bounds(0.5), rule=c["rule"])
    S = curved.CurvedSolver(cm, c["p"], c["q"], c["m"], alpha=c["alpha"], recovery="wadg")
    S.set_nodal_u(u0)
    for k in range(c["slabs"]):
        S.run({**tents, "t_top": tents["t_top"] + k * c["T"]})
    order = np.argsort(tents["layer"], kind="stable")
    np.savez_compressed(os.path.join(HERE, f"oracle_{name}.npz"), w=S.nodal_w(),
                        vertex=tents["vertex"][order].astype(np.int32), t_top=tents["t_top"][order],
                        layer=tents["layer"][order].astype(np.int32))


def make(name):
    if setup(name)[0]["curved"]:
        return make_curved(name)
    c, mm, dim, eps, mu, bc, ex, u0 = setup(name)
    mesh = Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc)
    tents = pitch(mesh, c["T"], sigma=0.5, rule=c["rule"])
    S = OracleSolver(mesh, c["p"], c["q"], c["m"], alpha=c["alpha"], data=ex if c["kind"] == DATA else None,
                     method=c["method"], flux=c["flux"], system=c["system"])
    S.set_nodal_u(u0)
    for k in range(c["slabs"]):
        S.run(tents, t_offset=k * c["T"])
    order = np.argsort(tents["layer"], kind="stable")
    np.savez_compressed(os.path.join(HERE, f"oracle_{name}.npz"), w=S.nodal_w(), u=S.nodal_u(),
                        vertex=tents["vertex"][order].astype(np.int32), t_top=tents["t_top"][order],
                        layer=tents["layer"][order].astype(np.int32))


if __name__ == "__main__":
    names = sys.argv[1:] or (list(CASES) + list(RK4_CASES) + list(IMP_CASES) + list(AC_CASES) + list(CURVED_CASES)
                             + list(COLOUR_CASES) + list(LARGE_P4_CASES) + list(AC_RK4_CASES))
    for n in names:
        t0 = time.time()
        make(n)
        print(f"{n}: {time.time() - t0:.1f}s", flush=True)
