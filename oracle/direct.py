"""Direct solve of the trace-constrained system Eq. (5) and the observables
of Sec. IV (oracle).

The method's result has a plain definition: the unique vec(rho_ss) with
L vec(rho) = 0 and Tr rho = 1.  Here it is computed by LU factorisation,
the direct route of Sec. II: dense LAPACK (partial pivoting) for small
systems, scipy's sparse LU (SuperLU) above that.

Pins (tests/test_oracle_solve.py): coherent cavity state at g0 = 0; truncated
thermal mechanical state at E = 0; Tr rho = 1, Hermiticity and positive
semidefiniteness; agreement with the null vector of a dense eigensolve;
invariance under a symmetric permutation (Sec. V).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import model

DENSE_LIMIT = 6000


def solve(Lt: sp.spmatrix, rhs: np.ndarray) -> np.ndarray:
    """x = L_tilde^{-1} rhs by LU (dense below DENSE_LIMIT rows, else sparse)."""
    n = Lt.shape[0]
    if n <= DENSE_LIMIT:
        return sla.solve(Lt.toarray(), rhs)
    lu = spla.splu(sp.csc_matrix(Lt))
    return lu.solve(rhs.astype(np.complex128))


def steady_state_vector(p, mode: int = model.TRACE_REPLACE) -> np.ndarray:
    """vec(rho_ss) for parameters p, by Eq. (5) and a direct solve."""
    L = model.liouvillian(p)
    Lt, rhs, _ = model.constrained_system(L, mode)
    return solve(Lt, rhs)


def to_density_matrix(x: np.ndarray, N: int, normalise: bool = True) -> np.ndarray:
    """rho from the column-stacked vector (Eq. (4)); optionally rho /= Tr rho."""
    rho = np.asarray(x, dtype=np.complex128).reshape((N, N), order="F")
    if normalise:
        rho = rho / np.trace(rho)
    return rho


def observable_weights(nc: int, nm: int):
    """Real diagonals of a^dag a, b^dag b and (b^dag b)^2 on the joint
    Hilbert space (index k = i*N_m + j)."""
    i = np.repeat(np.arange(nc, dtype=np.float64), nm)
    j = np.tile(np.arange(nm, dtype=np.float64), nc)
    return i, j, j * j


def observables(rho: np.ndarray, nc: int, nm: int) -> dict:
    """<a^dag a>, <b^dag b> and the mechanical Fano factor
    F = <(Delta N_b)^2> / <N_b> (Sec. IV) of a density matrix."""
    na_d, nb_d, nb2_d = observable_weights(nc, nm)
    d = np.real(np.diag(rho))
    n_a = float(d @ na_d)
    n_b = float(d @ nb_d)
    n_b2 = float(d @ nb2_d)
    fano = (n_b2 - n_b * n_b) / n_b if n_b != 0.0 else float("nan")
    return {"n_a": n_a, "n_b": n_b, "n_b2": n_b2, "fano": fano}


def relative_residual(Lt: sp.spmatrix, rhs: np.ndarray, x: np.ndarray) -> float:
    """||rhs - L_tilde x||_2 / ||rhs||_2 in complex128."""
    r = rhs - Lt @ x
    return float(np.linalg.norm(r) / np.linalg.norm(rhs))


def backward_error(L: sp.spmatrix, x: np.ndarray) -> float:
    """w-free backward error ||L x|| / (||L||_F ||x||) of a candidate rho."""
    return float(np.linalg.norm(L @ x) / (spla.norm(L, "fro") * np.linalg.norm(x)))


def hermiticity_error(rho: np.ndarray) -> float:
    return float(np.linalg.norm(rho - rho.conj().T) / np.linalg.norm(rho))


def steady_state(p, mode: int = model.TRACE_REPLACE):
    """(rho, observables) for parameters p."""
    N = p.nc * p.nm
    x = steady_state_vector(p, mode)
    rho = to_density_matrix(x, N)
    return rho, observables(rho, p.nc, p.nm)
