"""Checkpoint / restart and solver statistics through the C interface: a run stopped at a
flat front (and in the middle of a slab), written out, restored into a fresh solver and
continued equals the uninterrupted run bit for bit; foreign, corrupted and mismatched
checkpoints are refused."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from cases import setup  # noqa: E402

pytestmark = pytest.mark.gpu


def _solver(name="graded3d_p3_eps", precision=1, p=None):
    from paper_1906_11029_amd import mtp
    c, mm, dim, eps, mu, bc, ex, u0 = setup(name)
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc)
    T = mtp.Tents(M, c["T"], 0.5)
    S = mtp.Solver(M, T, p or c["p"], c["q"], c["m"], precision=precision)
    if p is None:
        S.set_fields(u0, 0.0)
    S.set_schedule(mtp.MTP_SCHEDULE_DAG)
    return c, M, T, S


def test_checkpoint_restart_bitwise(tmp_path):
    print("[gpu checkpoint] restart at a flat front", flush=True)
    c, M, T, A = _solver()
    A.advance_to(3 * c["T"])
    ref = A.get_state()
    _, _, _, B = _solver()
    B.advance_to(c["T"])
    path = str(tmp_path / "ck.bin")
    B.checkpoint_write(path)
    _, _, _, C = _solver()
    C.checkpoint_read(path)
    assert C.front() == (c["T"], 0)
    C.advance_to(3 * c["T"])
    assert np.array_equal(C.get_state(), ref)
    st = C.stats()
    assert st["slabs_done"] == 3 and st["layers_done"] == 0 and st["n_tents"] == T.n_tents
    assert st["schedule"] == 1 and st["kernel"] == 2 and st["persistent_workgroups"] > 0
    assert st["dof_updates_per_slab"] == C.slab_dof_updates()[0]


def test_checkpoint_mid_slab(tmp_path):
    print("[gpu checkpoint] restart in the middle of a slab", flush=True)
    c, M, T, A = _solver(precision=0)
    A.advance_to(c["T"])
    ref = A.get_state()
    _, _, _, B = _solver(precision=0)
    half = T.n_layers // 2
    for layer in range(half):
        B.layer_advance(layer)
    path = str(tmp_path / "mid.bin")
    B.checkpoint_write(path)
    _, _, _, C = _solver(precision=0)
    C.checkpoint_read(path)
    assert C.front()[1] == half
    for layer in range(half, T.n_layers):
        C.layer_advance(layer)
    assert np.array_equal(C.get_state(), ref)


def test_checkpoint_refusals(tmp_path):
    from paper_1906_11029_amd import mtp
    c, M, T, A = _solver()
    A.advance_to(c["T"])
    path = str(tmp_path / "ck.bin")
    A.checkpoint_write(path)
    with pytest.raises(mtp.MTPError) as e:          # another degree: another discretisation
        _solver(p=2)[3].checkpoint_read(path)
    assert e.value.code == -7
    raw = bytearray(open(path, "rb").read())
    raw[len(raw) // 2] ^= 0x40                       # one flipped bit in the state
    bad = str(tmp_path / "bad.bin")
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(mtp.MTPError) as e:
        _solver()[3].checkpoint_read(bad)
    assert e.value.code == -1 and "checksum" in str(e.value)
    junk = str(tmp_path / "junk.bin")
    open(junk, "wb").write(b"not a checkpoint")
    with pytest.raises(mtp.MTPError):
        _solver()[3].checkpoint_read(junk)
    with pytest.raises(mtp.MTPError):
        _solver()[3].checkpoint_read(str(tmp_path / "missing.bin"))
