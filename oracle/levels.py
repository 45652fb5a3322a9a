"""Level schedule of triangular factors (oracle).

A row of a lower-triangular solve can be computed once every row it reads
has been; its level is 1 + the largest level among the columns of its
strictly-lower entries (0 if it has none).  For an upper-triangular solve,
run from the last row, the same holds with the strictly-upper entries.  The
depth of the schedule (number of levels) bounds the number of sequential
steps of a level-scheduled substitution.

Pins (tests/test_oracle_levels.py): diagonal, bidiagonal and dense triangles
(depth 1, n, n) and a hand-made pattern.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def lower_levels(Lf: sp.spmatrix) -> np.ndarray:
    L = sp.csr_matrix(Lf)
    n = L.shape[0]
    lev = np.zeros(n, dtype=np.int64)
    for i in range(n):
        cols = L.indices[L.indptr[i]:L.indptr[i + 1]]
        cols = cols[cols < i]
        lev[i] = 1 + int(lev[cols].max()) if cols.size else 0
    return lev


def upper_levels(Uf: sp.spmatrix) -> np.ndarray:
    U = sp.csr_matrix(Uf)
    n = U.shape[0]
    lev = np.zeros(n, dtype=np.int64)
    for i in range(n - 1, -1, -1):
        cols = U.indices[U.indptr[i]:U.indptr[i + 1]]
        cols = cols[cols > i]
        lev[i] = 1 + int(lev[cols].max()) if cols.size else 0
    return lev


def depth(levels: np.ndarray) -> int:
    return int(levels.max()) + 1 if levels.size else 0
