"""Pins of the oracle ILUT (Sec. II) and level schedule."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from conftest import read_golden
from oracle import ilut, levels, model, ordering


def _dict(M):
    C = sp.coo_matrix(M)
    return {(int(i), int(j)): complex(v) for i, j, v in zip(C.row, C.col, C.data)}


@pytest.mark.parametrize("phase", [1.0, 1j])
def test_hand_worked_ilut(phase):
    g = read_golden("ilut_hand_4x4.txt")
    A = sp.csr_matrix(np.array(g["A"], dtype=np.complex128) * phase)
    for fill, lk, uk in [(np.inf, "L_inf", "U_inf"), (1.0, "L_p1", "U_p1")]:
        Lf, Uf, _ = ilut.ilut(A, g["d"], fill)
        Ld, Ud = _dict(Lf), _dict(Uf)
        assert set(Ld) == set(g[lk]) and set(Ud) == set(g[uk])
        for k, v in g[lk].items():
            assert abs(Ld[k] - v) <= 1e-15
        for k, v in g[uk].items():
            assert abs(Ud[k] - phase * v) <= 1e-15


def test_zero_drop_is_complete_lu():
    """Sec. II: d = 0 (and no fill cap) returns the complete LU factorisation,
    so L U reproduces A."""
    p = W.TINY.replace(nm=6)
    Lt, _, _ = model.constrained_system(model.liouvillian(p))
    A = ordering.permute(Lt, ordering.rcm(Lt))
    Lf, Uf, st = ilut.ilut(A, 0.0, np.inf)
    n = A.shape[0]
    LU = (Lf + sp.identity(n)) @ Uf
    assert abs(LU - A).max() <= 1e-13 * abs(A).max()
    assert st["repaired_pivots"] == 0
    x = np.random.default_rng(1).standard_normal(n) + 0j
    y = ilut.apply(Lf, Uf, A @ x)
    assert np.max(np.abs(y - x)) <= 1e-9 * np.max(np.abs(x))


def test_threshold_and_cap_properties():
    p = W.TINY.replace(nm=6)
    Lt, _, _ = model.constrained_system(model.liouvillian(p))
    A = ordering.permute(Lt, ordering.rcm(Lt))
    d, fill = 1e-3, 3.0
    Lf, Uf, st = ilut.ilut(A, d, fill)
    A = sp.csr_matrix(A)
    assert Lf.nnz + Uf.nnz <= fill * A.nnz
    for i in range(A.shape[0]):
        row = A.getrow(i)
        tau = d * np.abs(row.data).max()
        lfil = int(np.floor((fill * row.nnz - 1) / 2))
        lv = Lf.getrow(i)
        uv = Uf.getrow(i)
        off_u = uv.data[uv.indices != i]
        assert lv.nnz <= lfil and off_u.size <= lfil
        assert np.all(np.abs(lv.data) >= tau) and np.all(np.abs(off_u) >= tau)
        assert uv.indices.min() == i       # diagonal stored first-in-row
    assert np.all(sp.tril(Lf, k=0).diagonal() == 0)


def test_adjoint_apply_is_conjugate_transpose():
    p = W.TINY.replace(nm=5)
    Lt, _, _ = model.constrained_system(model.liouvillian(p))
    A = ordering.permute(Lt, ordering.rcm(Lt))
    Lf, Uf, _ = ilut.ilut(A, 1e-4, 10.0)
    rng = np.random.default_rng(3)
    n = A.shape[0]
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    lhs = np.vdot(y, ilut.apply(Lf, Uf, x))
    rhs = np.vdot(ilut.apply(Lf, Uf, y, adjoint=True), x)
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_levels_simple_patterns():
    n = 7
    D = sp.identity(n, format="csr")
    assert levels.depth(levels.lower_levels(D)) == 1
    bid = sp.diags([np.ones(n - 1)], [-1], shape=(n, n), format="csr")
    assert levels.lower_levels(bid).tolist() == list(range(n))
    assert levels.depth(levels.upper_levels(bid.T.tocsr())) == n
    # hand pattern: rows 1,2 depend on 0; row 3 on 1 and 2; rows 4..6 independent
    r = [1, 2, 3, 3]
    c = [0, 0, 1, 2]
    M = sp.csr_matrix((np.ones(4), (r, c)), shape=(n, n))
    assert levels.lower_levels(M).tolist() == [0, 1, 1, 2, 0, 0, 0]
    assert levels.upper_levels(M.T.tocsr()).tolist() == [2, 1, 1, 0, 0, 0, 0]
