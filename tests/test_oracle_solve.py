"""Pins of the oracle steady state (Eq. (2), (4), (5)) against closed forms,
invariants and an independent eigen-solve."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import direct, model, ordering


def coherent_state(alpha, dim):
    """Fock amplitudes of |alpha>, normalised on the truncated space."""
    from math import factorial
    c = np.array([alpha ** n / np.sqrt(float(factorial(n))) for n in range(dim)], dtype=np.complex128)
    return c / np.linalg.norm(c)


def test_coherent_cavity_at_zero_coupling():
    """g0 = 0: the driven damped cavity relaxes to the coherent state with
    alpha = E / (Delta + i kappa / 2), <a^dag a> = E^2 / (Delta^2 + kappa^2/4),
    and the state factorises into cavity (x) mechanics."""
    p = W.TINY.replace(nc=14, nm=3, g0=0.0)
    N = p.nc * p.nm
    rho, obs = direct.steady_state(p)
    alpha = p.E / (p.delta + 0.5j * p.kappa)
    assert abs(obs["n_a"] - abs(alpha) ** 2) <= 1e-10 * abs(alpha) ** 2
    r4 = rho.reshape(p.nc, p.nm, p.nc, p.nm)
    rho_c = np.einsum("imjm->ij", r4)
    rho_m = np.einsum("iaib->ab", r4)
    c = coherent_state(alpha, p.nc)
    assert np.max(np.abs(rho_c - np.outer(c, c.conj()))) <= 1e-10
    assert np.max(np.abs(rho - np.kron(rho_c, rho_m))) <= 1e-12


@pytest.mark.parametrize("g2", [0.0, 0.25])
@pytest.mark.parametrize("n_th", [0.5, 2.0])
def test_thermal_mechanics_without_drive(n_th, g2):
    """E = 0: cavity in vacuum, mechanics in the truncated thermal state
    p_n proportional to r^n with r = n_th / (n_th + 1) (detailed balance of the
    b and b^dag jumps, exact in the truncated space).  Both couplings act
    through a^dag a, which vanishes on the vacuum, so a quadratic coupling g2
    leaves this state unchanged."""
    p = W.TINY.replace(nc=3, nm=9, E=0.0, n_th=n_th, g2=g2)
    rho, obs = direct.steady_state(p)
    r = n_th / (n_th + 1.0)
    pn = r ** np.arange(p.nm)
    pn /= pn.sum()
    expect = np.kron(np.diag([1.0, 0.0, 0.0]), np.diag(pn))
    assert np.max(np.abs(rho - expect)) <= 1e-12
    assert abs(obs["n_b"] - float(np.arange(p.nm) @ pn)) <= 1e-12
    assert abs(obs["n_a"]) <= 1e-14


@pytest.mark.parametrize("case", range(5))
def test_density_matrix_invariants(case):
    p = W.small_cases()[case]
    if p.n > 4000:
        p = p.replace(nm=max(3, int(np.sqrt(4000) // p.nc)))
    rho, _ = direct.steady_state(p)
    assert abs(np.trace(rho) - 1.0) <= 1e-13
    assert direct.hermiticity_error(rho) <= 1e-10
    assert np.linalg.eigvalsh(0.5 * (rho + rho.conj().T)).min() >= -1e-10


def test_null_vector_of_dense_eigensolve():
    """The kernel of L (Eq. (4)), found by a dense eigen-decomposition, is the
    same vector as the solution of the constrained system Eq. (5)."""
    p = W.TINY.replace(nm=6)
    N = p.nc * p.nm
    L = model.liouvillian(p).toarray()
    ev, V = sla.eig(L)
    v = V[:, np.argmin(np.abs(ev))]
    rho_eig = v.reshape(N, N, order="F")
    rho_eig = rho_eig / np.trace(rho_eig)
    rho, _ = direct.steady_state(p)
    assert np.max(np.abs(rho - rho_eig)) <= 1e-10


def test_trace_forms_give_the_same_state():
    p = W.TINY
    x1 = direct.steady_state_vector(p, model.TRACE_REPLACE)
    x2 = direct.steady_state_vector(p, model.TRACE_ADD)
    assert np.max(np.abs(x1 - x2)) <= 1e-12


def test_symmetric_permutation_is_a_similarity():
    """Solving P A P^T (P b) and un-permuting returns the same solution
    (Sec. V)."""
    p = W.TINY
    L = model.liouvillian(p)
    Lt, b, _ = model.constrained_system(L)
    x = direct.solve(Lt, b)
    perm = ordering.rcm(Lt)
    xp = direct.solve(ordering.permute(Lt, perm), b[perm])
    y = np.empty_like(xp)
    y[perm] = xp
    assert np.max(np.abs(x - y)) <= 1e-12


def test_tiny_thermal_occupation_matches_zero_temperature():
    """Sec. IV: n_th = 1e-15 gives a density matrix numerically identical to
    n_th = 0."""
    p = W.ADJOINT.replace(nc=4, nm=8)
    assert p.n_th == 0.0
    r0, _ = direct.steady_state(p)
    r1, _ = direct.steady_state(p.replace(n_th=1e-15))
    assert np.max(np.abs(r0 - r1)) <= 1e-12


def test_sparse_and_dense_direct_agree():
    p = W.TINY
    L = model.liouvillian(p)
    Lt, b, _ = model.constrained_system(L)
    xd = direct.solve(Lt, b)
    import scipy.sparse.linalg as spla
    import scipy.sparse as sp
    xs = spla.splu(sp.csc_matrix(Lt)).solve(b)
    assert np.max(np.abs(xd - xs)) <= 1e-11
    assert direct.relative_residual(Lt, b, xd) <= 1e-14
