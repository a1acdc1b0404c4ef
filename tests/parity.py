"""Comparison helpers of the GPU parity tests (imported by the test modules).

`close` is the parity bar: every element of a GPU result must agree with
the oracle's to `tol` relative to the largest magnitude of the oracle's
array (numpy's assert_allclose with rtol = tol and atol = tol * max|ref|),
and the relative Frobenius norm of the whole difference must be below `tol`
as well.  The element-wise bound is what catches a single wrong tile or row
that a norm over tens of thousands of entries would hide.
"""
import numpy as np


def as_np(x):
    if hasattr(x, "detach"):
        x = x.detach().cpu().numpy()
    return np.asarray(x, np.float64)


def rel(a, b) -> float:
    a, b = as_np(a), as_np(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def close(got, ref, tol, what="") -> float:
    """Asserts element-wise and Frobenius agreement to `tol`; returns the
    Frobenius figure (for reports)."""
    got, ref = as_np(got), as_np(ref)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    scale = float(np.abs(ref).max()) if ref.size else 0.0
    np.testing.assert_allclose(got, ref, rtol=tol, atol=tol * scale, err_msg=str(what))
    f = rel(got, ref)
    assert f < tol, (what, f, tol)
    return f


def close_scaled(got, ref, tol, scale, what="") -> float:
    """Element-wise agreement to `tol` relative to a given magnitude `scale`
    (for a quantity that passes close to zero, such as the state of a bar
    coming to rest: the scale is the largest magnitude along the
    trajectory).  Returns max |got - ref| / scale."""
    got, ref = as_np(got), as_np(ref)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    np.testing.assert_allclose(got, ref, rtol=tol, atol=tol * scale, err_msg=str(what))
    return float(np.abs(got - ref).max() / scale)
