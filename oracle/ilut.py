"""Dual-threshold incomplete LU factorisation and its application (oracle).

Sec. II describes the preconditioner: an incomplete LU of the (reordered)
constrained matrix in which fill-in smaller than d times the infinity norm of
a row is dropped and at most p * NNZ(L_tilde) nonzeros are kept; d = 0 gives
the complete LU.  This is the row-wise ILUT of Saad ("Iterative Methods for
Sparse Linear Systems", ILUT), read as follows:

  for each row i, with tau_i = d * max_j |a_ij| and w = a_i:
    for k < i in increasing order with w_k != 0 (fill created during the
    loop included):
      w_k <- w_k / u_kk
      if |w_k| < tau_i: w_k <- 0           (first dropping rule)
      else: w <- w - w_k * u_k             (u_k = row k of U, columns > k)
    drop every off-diagonal w_j with |w_j| < tau_i  (second dropping rule)
    keep the lfil_i largest |w_j| among j < i and among j > i, ties to the
    lower column, with lfil_i = floor((p * nnz(a_i) - 1) / 2), so that
    nnz(L) + nnz(U) <= p * nnz(A)
    l_ij = w_j (j < i, unit diagonal implied), u_ij = w_j (j >= i)

Readings where Sec. II is silent: no pivoting (the "P" of iLUTP is not
used: the constrained matrix has a zero-free diagonal); a pivot with
|u_ii| < 1e-14 * ||a_i||_inf is replaced by that floor times the phase of
u_ii (1 if u_ii == 0) and counted; magnitudes are compared as squared
moduli (re^2 + im^2 against tau^2), which is the same test without a root.

Pins (tests/test_oracle_ilut.py): d = 0 with no cap reproduces the complete
LU (L U == A to rounding); a hand-worked 4x4 example of both dropping rules
and of the cap (tests/golden/ilut_hand_4x4.txt); every kept entry passes the
threshold; nnz bound.
"""
from __future__ import annotations

import heapq
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

PIVOT_FLOOR = 1e-14


def _abs2(z: complex) -> float:
    return z.real * z.real + z.imag * z.imag


def ilut(A: sp.spmatrix, drop_tol: float, fill_factor: float):
    """Return (Lf, Uf, stats).

    Lf: strictly lower part (unit diagonal implied), CSR.
    Uf: upper part with the diagonal, CSR.
    stats: fill, nnz_L, nnz_U, repaired_pivots.
    """
    A = sp.csr_matrix(A, dtype=np.complex128)
    A.sort_indices()
    n = A.shape[0]
    indptr, indices, data = A.indptr, A.indices, A.data
    unbounded = not math.isfinite(fill_factor)

    U_rows = [None] * n          # (cols > k, vals) per row, for elimination
    U_diag = np.zeros(n, dtype=np.complex128)
    L_cols, L_vals, U_cols, U_vals = [], [], [], []
    L_ptr, U_ptr = [0], [0]
    repaired = 0

    for i in range(n):
        cols = indices[indptr[i]:indptr[i + 1]]
        vals = data[indptr[i]:indptr[i + 1]]
        w = {}
        for c, v in zip(cols, vals):
            w[int(c)] = complex(v)
        row_inf = max((abs(complex(v)) for v in vals), default=0.0)
        tau = drop_tol * row_inf
        tau2 = tau * tau
        lfil = None if unbounded else max(0, int(math.floor((fill_factor * len(cols) - 1) / 2)))

        heap = [c for c in w if c < i]
        heapq.heapify(heap)
        in_heap = set(heap)
        while heap:
            k = heapq.heappop(heap)
            wk = w.get(k, 0j)
            if wk == 0:
                w.pop(k, None)
                continue
            wk = wk / U_diag[k]
            if _abs2(wk) < tau2:
                w.pop(k, None)        # first dropping rule
                continue
            w[k] = wk
            ucols, uvals = U_rows[k]
            for c, u in zip(ucols, uvals):
                if c in w:
                    w[c] = w[c] - wk * u
                else:
                    w[c] = -(wk * u)
                    if c < i and c not in in_heap:
                        heapq.heappush(heap, c)
                        in_heap.add(c)

        # second dropping rule and the per-row cap
        diag = w.pop(i, 0j)
        lower = [(c, v) for c, v in w.items() if c < i and _abs2(v) >= tau2 and v != 0]
        upper = [(c, v) for c, v in w.items() if c > i and _abs2(v) >= tau2 and v != 0]
        if lfil is not None:
            if len(lower) > lfil:
                lower.sort(key=lambda cv: (-_abs2(cv[1]), cv[0]))
                lower = lower[:lfil]
            if len(upper) > lfil:
                upper.sort(key=lambda cv: (-_abs2(cv[1]), cv[0]))
                upper = upper[:lfil]
        lower.sort()
        upper.sort()

        floor = PIVOT_FLOOR * row_inf
        if abs(diag) < floor or diag == 0:
            phase = diag / abs(diag) if diag != 0 else 1.0 + 0j
            diag = floor * phase if floor > 0 else 1.0 + 0j
            repaired += 1
        U_diag[i] = diag
        U_rows[i] = ([c for c, _ in upper], [v for _, v in upper])

        for c, v in lower:
            L_cols.append(c)
            L_vals.append(v)
        L_ptr.append(len(L_cols))
        U_cols.append(i)
        U_vals.append(diag)
        for c, v in upper:
            U_cols.append(c)
            U_vals.append(v)
        U_ptr.append(len(U_cols))

    Lf = sp.csr_matrix((np.asarray(L_vals, dtype=np.complex128), np.asarray(L_cols, dtype=np.int64),
                        np.asarray(L_ptr, dtype=np.int64)), shape=(n, n))
    Uf = sp.csr_matrix((np.asarray(U_vals, dtype=np.complex128), np.asarray(U_cols, dtype=np.int64),
                        np.asarray(U_ptr, dtype=np.int64)), shape=(n, n))
    stats = {
        "nnz_L": int(Lf.nnz),
        "nnz_U": int(Uf.nnz),
        "fill": (Lf.nnz + Uf.nnz) / A.nnz,
        "repaired_pivots": repaired,
    }
    return Lf, Uf, stats


def apply(Lf: sp.spmatrix, Uf: sp.spmatrix, x: np.ndarray, adjoint: bool = False) -> np.ndarray:
    """Preconditioner solve y = (Lf Uf)^{-1} x, with Lf unit lower (strict part
    stored).  adjoint=True gives y = (Lf Uf)^{-H} x = Lf^{-H} Uf^{-H} x."""
    n = Lf.shape[0]
    I = sp.identity(n, dtype=np.complex128, format="csr")
    Lu = (sp.csr_matrix(Lf) + I).tocsr()
    Uc = sp.csr_matrix(Uf)
    x = np.asarray(x, dtype=np.complex128)
    if not adjoint:
        z = spla.spsolve_triangular(Lu, x, lower=True, unit_diagonal=True)
        return spla.spsolve_triangular(Uc, z, lower=False)
    z = spla.spsolve_triangular(Uc.conj().T.tocsr(), x, lower=True)
    return spla.spsolve_triangular(Lu.conj().T.tocsr(), z, lower=False, unit_diagonal=True)


def condest(Lf: sp.spmatrix, Uf: sp.spmatrix) -> float:
    """Condition estimate of the preconditioner used in Sec. IV, read as
    ||(L U)^{-1} e||_inf with e the all-ones vector."""
    e = np.ones(Lf.shape[0], dtype=np.complex128)
    return float(np.max(np.abs(apply(Lf, Uf, e))))
