"""Comparison helpers shared by the GPU parity tests.

Two measures are used side by side:
  * relf: relative Frobenius error ||X - X_ref|| / ||X_ref||;
  * colscaled: max over entries of |X_ij - X_ref_ij| / ||X_ref[:, j]||, i.e.
    every entry judged against the norm of its own column.  On joins whose
    columns are scaled over six orders of magnitude, a Frobenius check is
    dominated by the largest columns and cannot see an error confined to a
    small one; the column-scaled check can.  R is unique for a full-rank join
    (positive diagonal), so its columns are comparable one by one.
"""
import numpy as np


def relf(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def colscaled(a, b, axis=0):
    """max |a - b| / ||b along `axis`||: axis=0 judges each entry against the
    norm of its column (matrices such as R), axis=1 against the norm of its
    row (the (columns x rows) layout of relation values and gradients)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nrm = np.linalg.norm(b, axis=axis, keepdims=True)
    diff = np.abs(a - b)
    # a column of zeros must be matched exactly
    out = np.where(nrm > 0, diff / np.where(nrm > 0, nrm, 1.0), np.where(diff > 0, np.inf, 0.0))
    return float(out.max()) if out.size else 0.0
