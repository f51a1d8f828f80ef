"""The parity check used by the GPU tests catches an error confined to one element that
the global relative L2 alone would let through (a planted mistake in a copy of an oracle
fixture, on the CPU)."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from parity import assert_parity, rel  # noqa: E402


@pytest.mark.parametrize("name,tol", [("te_planewave_p2", 1e-10), ("cav3d_p3", 1e-10), ("graded3d_p3_eps", 1e-6)])
def test_single_element_error_fails_parity(name, tol):
    ref = np.load(os.path.join(HERE, "golden", f"oracle_{name}.npz"))["w"]
    assert_parity(ref.copy(), ref, tol)
    bad = ref.copy()
    e = len(ref) // 3
    bad[e, -1, 0] += 2 * tol * np.abs(ref).max()   # one face-adjacent node of one element
    assert rel(bad, ref) <= tol                       # invisible to the global norm ...
    with pytest.raises(AssertionError, match=f"element {e} "):
        assert_parity(bad, ref, tol)                  # ... but not to the per-element bound
