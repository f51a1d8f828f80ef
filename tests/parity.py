"""Parity checks shared by the GPU tests: a nodal array from the HIP path against the
oracle's, both as one relative L2 over the whole array and node by node, so that an error
confined to one element (one face node, say) cannot hide in the global norm."""
import numpy as np


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def parity_errors(got, ref):
    """(relative L2, worst element, that element's largest nodal difference / max |ref|)."""
    got, ref = np.asarray(got), np.asarray(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    scale = float(np.abs(ref).max())
    per_el = np.abs(got - ref).reshape(len(ref), -1).max(axis=1) / scale
    worst = int(np.argmax(per_el))
    return rel(got, ref), worst, float(per_el[worst])


def assert_parity(got, ref, tol, what=""):
    """Relative L2 <= tol and, for every element e, max over its nodal values of
    |got - ref| <= tol * max |ref|."""
    g, worst, el = parity_errors(got, ref)
    assert g <= tol, f"{what}: relative L2 {g:.3e} > {tol:.1e}"
    assert el <= tol, f"{what}: element {worst} differs by {el:.3e} (relative to max |ref|) > {tol:.1e}"
    return g, el
