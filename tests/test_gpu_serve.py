"""GPU check of the stream server: solves served by continuous batching (batches rebuilt as
requests arrive and leave) end bit for bit where the same solves run alone."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


class Executor:
    def __init__(self):
        self.batch, self.members = None, ()

    def footprint(self, req):
        return 1

    def setup(self, req):
        from mtp_inputs import fields, meshes
        from paper_1906_11029_amd import mtp
        sp = req.spec
        mm = meshes.cube_kuhn(sp["n"])
        M = mtp.Mesh(mm["coords"], mm["cells"])
        T = mtp.Tents(M, sp["H"], 0.5)
        S = mtp.Solver(M, T, sp["p"], sp["p"] + 1, 2 * sp["p"])
        S.set_fields(fields.Cavity3D_PEC().u(meshes.equispaced_nodes(mm, sp["p"]), 0.0), 0.0)
        return {"rid": req.rid, "S": S, "n": sp["slabs"], "M": M, "T": T}

    def slabs(self, h):
        return h["n"]

    def step(self, hs):
        from paper_1906_11029_amd import mtp
        key = tuple(h["rid"] for h in hs)
        if key != self.members:
            self.batch = None
            self.batch = mtp.Batch([h["S"] for h in hs])
            self.members = key
        self.batch.advance(1)

    def run(self, h):
        h["S"].advance_to(h["n"] * h["S"].tents.t_end)

    def finish(self, h):
        return {"w": h["S"].get_state()}


def test_continuous_batching_equals_solves_alone():
    from paper_1906_11029_amd import mtp
    from paper_1906_11029_amd.serve import Request, StreamServer
    specs = [dict(n=3, p=2, H=0.2, slabs=3), dict(n=2, p=3, H=0.25, slabs=1), dict(n=3, p=3, H=0.1, slabs=2)]
    print("[gpu serve] 3 requests, continuous batching vs alone", flush=True)
    reqs = [Request(i, 0.002 * i, sp) for i, sp in enumerate(specs)]
    ex = Executor()
    recs = StreamServer(ex, budget_bytes=10, batched=True).run(reqs)
    ex.batch = None
    alone = Executor()
    for r, sp in zip(recs, specs):
        h = alone.setup(Request(r.rid, 0.0, sp))
        h["S"].set_tuning(mtp.MTP_SCHEDULE_LAYERS)
        alone.run(h)
        assert np.array_equal(r.result["w"], h["S"].get_state()), f"request {r.rid}"
