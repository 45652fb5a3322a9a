"""Optomechanical Lindblad Liouvillian in the Fock basis (oracle).

Follows Eq. (1) (Hamiltonian in the frame rotating at the pump), Eq. (3)
(Lindblad master equation with dissipators D[a], D[b], D[b^dag]) and Eq. (4)
(column-stacked vectorisation), with the operator ordering of Sec. III:
a = a (x) I_b and b = I_a (x) b, so the Hilbert index is k = i*N_m + j
(i cavity, j mechanical).  The trace-constrained system is Eq. (5) with the
weight w of Sec. IV (mean of the diagonal of L).

Everything is built from Kronecker products of small sparse matrices using the
identity vec(A X B) = (B^T (x) A) vec(X) for column stacking.  Entries that
evaluate to exactly zero are not stored.

Pins (tests/test_oracle_model.py): the closed-form nonzero count and the
Fig. 1 count 8957; trace preservation t^T L = 0; Hermiticity preservation;
upper bandwidth N^2 - 1 of the constrained matrix (Sec. III).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

TRACE_NONE = 0      # L itself (singular)
TRACE_REPLACE = 1   # row 0 := w * t^T, rhs = w e_0
TRACE_ADD = 2       # row 0 := L_0 + w * t^T, rhs = w e_0  (Eq. (5) as printed)


def destroy(dim: int) -> sp.csr_matrix:
    """Annihilation operator on a dim-level Fock space: a|i> = sqrt(i)|i-1>."""
    if dim < 1:
        raise ValueError("Fock dimension must be >= 1")
    vals = np.sqrt(np.arange(1, dim, dtype=np.float64)).astype(np.complex128)
    return sp.diags(vals, offsets=1, shape=(dim, dim), format="csr", dtype=np.complex128)


def mode_operators(nc: int, nm: int):
    """a = a_c (x) I_m and b = I_c (x) b_m on the joint Hilbert space
    (Sec. III operator ordering)."""
    ac = destroy(nc)
    bm = destroy(nm)
    a = sp.kron(ac, sp.identity(nm, dtype=np.complex128, format="csr"), format="csr")
    b = sp.kron(sp.identity(nc, dtype=np.complex128, format="csr"), bm, format="csr")
    return a, b


def _dag(op: sp.spmatrix) -> sp.csr_matrix:
    return op.conj().T.tocsr()


def hamiltonian(p) -> sp.csr_matrix:
    """Eq. (1): H = -Delta a^dag a + omega_m b^dag b + g0 (b + b^dag) a^dag a
    + E (a + a^dag), hbar = 1; plus g2 (b + b^dag)^2 a^dag a when p has a
    nonzero g2 (the quadratic coupling the conclusion (Sec. V) names as a
    variant), with the truncated operators multiplied as matrices."""
    a, b = mode_operators(p.nc, p.nm)
    ad, bd = _dag(a), _dag(b)
    na = ad @ a
    nb = bd @ b
    H = (-p.delta) * na + p.omega_m * nb + p.g0 * ((b + bd) @ na) + p.E * (a + ad)
    g2 = getattr(p, "g2", 0.0)
    if g2:
        x = b + bd
        H = H + g2 * ((x @ x) @ na)
    return H.tocsr()


def collapse_operators(p):
    """The three collapse operators of Eq. (3): sqrt(kappa) a,
    sqrt(Gamma (1 + n_th)) b and sqrt(Gamma n_th) b^dag.  Operators with a
    zero rate are omitted (their dissipator vanishes identically)."""
    a, b = mode_operators(p.nc, p.nm)
    ops = []
    if p.kappa != 0.0:
        ops.append(np.sqrt(p.kappa) * a)
    if p.gamma_m * (1.0 + p.n_th) != 0.0:
        ops.append(np.sqrt(p.gamma_m * (1.0 + p.n_th)) * b)
    if p.gamma_m * p.n_th != 0.0:
        ops.append(np.sqrt(p.gamma_m * p.n_th) * _dag(b))
    return ops


def liouvillian_from(H: sp.spmatrix, c_ops) -> sp.csr_matrix:
    """Matrix of L[rho] = -i[H, rho] + sum_c (C rho C^dag - 1/2 {C^dag C, rho})
    acting on the column-stacked vec(rho) (Eq. (3), Eq. (4)).

    With vec(A X B) = (B^T (x) A) vec(X):
      H rho        -> I (x) H
      rho H        -> H^T (x) I
      C rho C^dag  -> conj(C) (x) C
      C^dag C rho  -> I (x) C^dag C
      rho C^dag C  -> (C^dag C)^T (x) I
    """
    N = H.shape[0]
    I = sp.identity(N, dtype=np.complex128, format="csr")
    L = -1j * (sp.kron(I, H) - sp.kron(H.T, I))
    for C in c_ops:
        C = sp.csr_matrix(C)
        CdC = (_dag(C) @ C).tocsr()
        L = L + sp.kron(C.conj(), C) - 0.5 * sp.kron(I, CdC) - 0.5 * sp.kron(CdC.T, I)
    L = sp.csr_matrix(L, dtype=np.complex128)
    L.sum_duplicates()
    L.eliminate_zeros()
    L.sort_indices()
    return L


def liouvillian(p) -> sp.csr_matrix:
    """L of Eq. (3)-(4) for the optomechanical model with parameters p."""
    return liouvillian_from(hamiltonian(p), collapse_operators(p))


def trace_vector(N: int) -> np.ndarray:
    """t with t^T vec(rho) = Tr rho: ones at the diagonal positions k(N+1)
    of the column-stacked vector (the single row of the matrix T in Eq. (5))."""
    t = np.zeros(N * N, dtype=np.complex128)
    t[np.arange(N) * (N + 1)] = 1.0
    return t


def weight(L: sp.spmatrix) -> complex:
    """w of Eq. (5), chosen as the average of the diagonal elements of L
    (Sec. IV)."""
    return complex(L.diagonal().mean())


def constrained_system(L: sp.spmatrix, mode: int = TRACE_REPLACE, w: complex | None = None):
    """Return (L_tilde, rhs, w) for the trace-constrained system Eq. (5).

    TRACE_ADD     -- row 0 becomes L_0 + w t^T, as Eq. (5) is printed.
    TRACE_REPLACE -- row 0 becomes w t^T.  Row 0 of L is minus the sum of the
                     rows k(N+1), k >= 1 (trace preservation), so it carries no
                     information and both forms give the same solution.
    TRACE_NONE    -- L itself with a zero right-hand side.
    """
    n = L.shape[0]
    N = int(round(np.sqrt(n)))
    if N * N != n:
        raise ValueError("Liouvillian dimension is not a perfect square")
    if w is None:
        w = weight(L)
    rhs = np.zeros(n, dtype=np.complex128)
    if mode == TRACE_NONE:
        return sp.csr_matrix(L, dtype=np.complex128), rhs, w
    t = trace_vector(N)
    Lt = sp.lil_matrix(L, dtype=np.complex128)
    if mode == TRACE_REPLACE:
        Lt[0, :] = 0.0
        Lt[0, :] = w * t[None, :]
    elif mode == TRACE_ADD:
        Lt[0, :] = Lt[0, :].toarray() + w * t[None, :]
    else:
        raise ValueError(f"unknown trace mode {mode}")
    Lt = Lt.tocsr()
    Lt.eliminate_zeros()
    Lt.sort_indices()
    rhs[0] = w
    return Lt, rhs, w


def build_system(p, mode: int = TRACE_REPLACE):
    """Convenience: (L, L_tilde, rhs, w) for parameters p."""
    L = liouvillian(p)
    Lt, rhs, w = constrained_system(L, mode)
    return L, Lt, rhs, w
