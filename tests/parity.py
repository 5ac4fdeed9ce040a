"""Error measures for the GPU parity tests.

``rel(a, b)`` is the larger of two ratios against the reference b:
  * the relative 2-norm error ||a - b||_2 / ||b||_2, and
  * the element-wise max-abs error max_i |a_i - b_i| / max_i |b_i|, so that
    a wrong row confined to a few elements (one face, one orientation) cannot
    hide below the tolerance in the global norm.
Every assertion ``rel(a, b) <= tol`` therefore checks both."""

from __future__ import annotations

import numpy as np


def rel2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / (nb if nb > 0 else 1.0)


def relinf(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.size == 0:
        return 0.0
    nb = float(np.abs(b).max())
    return float(np.abs(a - b).max()) / (nb if nb > 0 else 1.0)


def rel(a, b) -> float:
    return max(rel2(a, b), relinf(a, b))


def worst_element(a, b, off):
    """(element, max-abs error of its rows / max |b|) of the element whose rows
    differ most; off = dof offsets [n_elems + 1]."""
    d = np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))
    per = np.maximum.reduceat(d, np.asarray(off[:-1], dtype=np.int64)) if d.size else np.zeros(0)
    e = int(np.argmax(per)) if per.size else -1
    nb = float(np.abs(b).max()) if d.size else 1.0
    return e, (float(per[e]) / nb if per.size else 0.0)


def rows_of(off, elems):
    return np.concatenate([np.arange(off[e], off[e + 1]) for e in elems])
