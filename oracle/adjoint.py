"""Gradients of steady-state observables by the adjoint of Eq. (5) (oracle).

For an objective f = Re o^T x, with x the solution of L_tilde x = w e_0 and
o = vec(O^T) for a diagonal observable O (so that o^T vec(rho) = Tr rho O),
differentiating Eq. (5) with respect to a model parameter theta gives
    L_tilde dx = -P0 (dL/dtheta) x,
where P0 zeroes row 0: with row 0 replaced by w t^T, its derivative
contributes (dw) (t^T x - 1) = 0 because Tr rho = 1.  Hence
    df/dtheta = -Re lambda^H P0 (dL/dtheta) x,   L_tilde^H lambda = conj(o).
The Fano factor F = <N_b^2>/<N_b> - <N_b> has the objective vector
o_F = o_2 / m_1 - (2 + F / m_1) o_1 with m_1 = <N_b>.

dL/dtheta is linear in the Hamiltonian and in the rates of Eq. (3):
    Delta -> -i[-a^dag a, .]       g0 -> -i[(b + b^dag) a^dag a, .]
    E     -> -i[a + a^dag, .]      kappa -> D[a]
    Gamma -> (1 + n_th) D[b] + n_th D[b^dag]

Pins (tests/test_oracle_adjoint.py): central finite differences of the direct
oracle solve with h = 1e-6.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import direct, model

PARAMS = ("delta", "g0", "E", "kappa", "gamma_m")


def dL_dtheta(p, name: str) -> sp.csr_matrix:
    a, b = model.mode_operators(p.nc, p.nm)
    ad = a.conj().T.tocsr()
    bd = b.conj().T.tocsr()
    N = p.nc * p.nm
    zero = sp.csr_matrix((N, N), dtype=np.complex128)
    if name == "delta":
        return model.liouvillian_from(-(ad @ a), [])
    if name == "g0":
        return model.liouvillian_from((b + bd) @ (ad @ a), [])
    if name == "E":
        return model.liouvillian_from(a + ad, [])
    if name == "kappa":
        return model.liouvillian_from(zero, [a])
    if name == "gamma_m":
        ops = [np.sqrt(1.0 + p.n_th) * b]
        if p.n_th != 0.0:
            ops.append(np.sqrt(p.n_th) * bd)
        return model.liouvillian_from(zero, ops)
    raise ValueError(name)


def objective_vectors(p, x: np.ndarray):
    """(o_a, o_b, o_F) and the observable values at x (Tr rho = 1)."""
    N = p.nc * p.nm
    n = N * N
    na_d, nb_d, nb2_d = direct.observable_weights(p.nc, p.nm)
    diag_pos = np.arange(N) * (N + 1)
    o_a = np.zeros(n, dtype=np.complex128)
    o_b = np.zeros(n, dtype=np.complex128)
    o_2 = np.zeros(n, dtype=np.complex128)
    o_a[diag_pos] = na_d
    o_b[diag_pos] = nb_d
    o_2[diag_pos] = nb2_d
    m_a = float(np.real(o_a @ x))
    m_1 = float(np.real(o_b @ x))
    m_2 = float(np.real(o_2 @ x))
    F = (m_2 - m_1 * m_1) / m_1
    o_F = o_2 / m_1 - (2.0 + F / m_1) * o_b
    return (o_a, o_b, o_F), (m_a, m_1, F)


def gradients(p, params=PARAMS):
    """Values (n_a, n_b, F) and their gradients with respect to params, by the
    dense adjoint solve.  Returns (values[3], grads[3, len(params)])."""
    L = model.liouvillian(p)
    Lt, rhs, _ = model.constrained_system(L, model.TRACE_REPLACE)
    D = Lt.toarray()
    lu = sla.lu_factor(D)
    x = sla.lu_solve(lu, rhs)
    objs, vals = objective_vectors(p, x)
    grads = np.zeros((3, len(params)))
    for fi, o in enumerate(objs):
        lam = sla.lu_solve(lu, np.conj(o), trans=2)      # L_tilde^H lam = conj(o)
        for ti, name in enumerate(params):
            v = dL_dtheta(p, name) @ x
            v[0] = 0.0                                   # P0
            grads[fi, ti] = -float(np.real(np.vdot(lam, v)))
    return np.asarray(vals), grads


def finite_differences(p, params=PARAMS, h: float = 1e-6):
    """Central differences of (n_a, n_b, F) over the direct oracle."""
    grads = np.zeros((3, len(params)))
    for ti, name in enumerate(params):
        vals = []
        for s in (+1.0, -1.0):
            q = p.replace(**{name: getattr(p, name) + s * h})
            _, o = direct.steady_state(q)
            vals.append(np.array([o["n_a"], o["n_b"], o["fano"]]))
        grads[:, ti] = (vals[0] - vals[1]) / (2.0 * h)
    return grads
