"""Pins of the oracle Liouvillian (Eq. (1), (3), (4), (5)) against facts fixed
by the paper and by the mathematics, not by re-typing the oracle."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from conftest import read_golden
from oracle import model, ordering


def nnz_closed_form(nc, nm, n_th):
    """Count of stored entries of L: diagonal (all but p = 0 when n_th = 0),
    ket- and bra-side Hamiltonian couplings, and the three jump terms.  Derived
    from Eq. (1) and Eq. (3) by counting, independently of the Kronecker build."""
    N = nc * nm
    z = 1 if n_th == 0 else 0
    return ((N * N - z) + 4 * N * (nc - 1) * (2 * nm - 1)
            + ((nc - 1) * nm) ** 2 + (1 + (1 - z)) * ((nm - 1) * nc) ** 2)


@pytest.mark.parametrize("nc,nm,n_th", [(2, 3, 0.5), (3, 4, 0.0), (4, 8, 3.0), (4, 10, 0.5), (5, 7, 0.0)])
def test_nnz_matches_counting_formula(nc, nm, n_th):
    p = W.TINY.replace(nc=nc, nm=nm, n_th=n_th)
    assert model.liouvillian(p).nnz == nnz_closed_form(nc, nm, n_th)


@pytest.mark.parametrize("nc,nm,n_th", [(2, 3, 0.5), (3, 5, 0.0), (4, 6, 3.0)])
def test_quadratic_coupling_nnz(nc, nm, n_th):
    """With the quadratic coupling g2 (b + b^dag)^2 a^dag a (Sec. V), every
    cavity level i >= 1 couples mechanical levels two apart, on the ket and
    on the bra side: 2 (nc - 1) 2 (nm - 2) new entries per column block of N,
    4 N (nc - 1)(nm - 2) in all; its diagonal part adds no entry."""
    p = W.TINY.replace(nc=nc, nm=nm, n_th=n_th, g2=0.3)
    N = nc * nm
    assert model.liouvillian(p).nnz == nnz_closed_form(nc, nm, n_th) + 4 * N * (nc - 1) * (nm - 2)


def test_quadratic_coupling_term():
    """H(g2) - H(0) = g2 (a^dag a) (x) (b + b^dag)^2, with the mechanical
    position operator written out densely from its matrix elements
    x[j, j+1] = x[j+1, j] = sqrt(j + 1) and squared in the truncated space."""
    p = W.TINY.replace(nc=3, nm=6)
    g2 = 0.37
    dH = (model.hamiltonian(p.replace(g2=g2)) - model.hamiltonian(p)).toarray() / g2
    x = np.zeros((p.nm, p.nm))
    for j in range(p.nm - 1):
        x[j, j + 1] = x[j + 1, j] = np.sqrt(j + 1.0)
    expect = np.kron(np.diag(np.arange(p.nc, dtype=float)), x @ x)
    assert np.max(np.abs(dH - expect)) <= 1e-13


def test_fig1_nnz_and_upper_bandwidth():
    g = read_golden("fig1_structure.txt")
    p = W.FIG1
    assert (p.nc, p.nm) == (g["nc"], g["nm"])
    L = model.liouvillian(p)
    Lt, _, _ = model.constrained_system(L, model.TRACE_ADD)
    assert Lt.nnz == g["nnz_constrained_additive"]
    st = ordering.bandwidth_profile(Lt)
    assert st["ub"] == g["upper_bandwidth"]
    assert st["B"] > (p.nc * p.nm) ** 2 - 1


@pytest.mark.parametrize("g2", [0.0, 0.2])
@pytest.mark.parametrize("n_th", [0.0, 0.5])
def test_trace_preservation(n_th, g2):
    """t^T L = 0: the Lindblad generator preserves the trace (Eq. (3))."""
    p = W.TINY.replace(nc=3, nm=5, n_th=n_th, g2=g2)
    L = model.liouvillian(p)
    t = model.trace_vector(p.nc * p.nm)
    row = L.T @ t
    assert np.max(np.abs(row)) <= 1e-14 * abs(L).max()


@pytest.mark.parametrize("g2", [0.0, 0.2])
def test_hermiticity_preservation(g2):
    """L[rho]^dag = L[rho^dag]: entry (p, q) equals conj of entry
    (sigma p, sigma q), where sigma swaps the ket and bra indices."""
    p = W.TINY.replace(nc=3, nm=4, g2=g2)
    N = p.nc * p.nm
    D = model.liouvillian(p).toarray()
    idx = np.arange(N * N)
    k, l = idx % N, idx // N
    sigma = k * N + l
    assert np.max(np.abs(D[np.ix_(sigma, sigma)] - D.conj())) <= 1e-15 * np.abs(D).max()


def test_spectrum_in_left_half_plane():
    p = W.TINY.replace(nc=3, nm=4)
    ev = np.linalg.eigvals(model.liouvillian(p).toarray())
    assert ev.real.max() <= 1e-12
    assert np.sort(np.abs(ev))[0] <= 1e-12          # a zero eigenvalue exists


def test_weight_closed_form():
    """Mean of diag(L): the Hamiltonian part cancels between ket and bra;
    the dissipative part is -mean(c_k) with c_k the decay rate of state k,
    giving w = -[kappa (N_c - 1) + Gamma (2 n_th + 1)(N_m - 1)] / 2."""
    for p in [W.TINY, W.FIG1, W.BATCH_BASE.replace(nc=4, nm=9)]:
        w = model.weight(model.liouvillian(p))
        expect = -(p.kappa * (p.nc - 1) + p.gamma_m * (2 * p.n_th + 1) * (p.nm - 1)) / 2
        assert abs(w - expect) <= 1e-13 * abs(expect)


def test_single_entries_from_the_master_equation():
    """A few entries of L written out from Eq. (3) by hand, at positions
    p = l*N + k (column stacking), k = i*N_m + j."""
    p = W.TINY.replace(nc=3, nm=4)
    N, nm = p.nc * p.nm, p.nm
    D = model.liouvillian(p).toarray()

    def pos(ik, jk, il, jl):
        return (il * nm + jl) * N + (ik * nm + jk)

    # kappa a rho a^dag feeds rho[(1,0),(1,0)] into rho[(0,0),(0,0)] with rate kappa*1
    assert np.isclose(D[pos(0, 0, 0, 0), pos(1, 0, 1, 0)], p.kappa)
    # Gamma(1+n_th) b rho b^dag: rho[(0,2),(0,1)] -> rho[(0,1),(0,0)], sqrt(2*1)
    assert np.isclose(D[pos(0, 1, 0, 0), pos(0, 2, 0, 1)], p.gamma_m * (1 + p.n_th) * np.sqrt(2.0))
    # Gamma n_th b^dag rho b: rho[(0,0),(0,1)] -> rho[(0,1),(0,2)], sqrt(1*2)
    assert np.isclose(D[pos(0, 1, 0, 2), pos(0, 0, 0, 1)], p.gamma_m * p.n_th * np.sqrt(2.0))
    # -i H rho, drive E a^dag: ket index (0,0) <- (1,0)?  (H rho)[k,l] = H[k,k'] rho[k',l]
    assert np.isclose(D[pos(0, 0, 2, 1), pos(1, 0, 2, 1)], -1j * p.E)
    # +i rho H, coupling g0 i (b + b^dag): bra index (1,1) <- (1,2): rho[k,l'] H[l',l]
    assert np.isclose(D[pos(0, 3, 1, 1), pos(0, 3, 1, 2)], 1j * p.g0 * 1 * np.sqrt(2.0))
    # diagonal at k = (1,2), l = (0,1)
    hk = -p.delta * 1 + 2.0
    hl = 1.0
    ck = p.kappa * 1 + p.gamma_m * (1 + p.n_th) * 2 + p.gamma_m * p.n_th * 3
    cl = p.gamma_m * (1 + p.n_th) * 1 + p.gamma_m * p.n_th * 2
    assert np.isclose(D[pos(1, 2, 0, 1), pos(1, 2, 0, 1)], -1j * (hk - hl) - 0.5 * (ck + cl))
    # top mechanical level: b^dag b^... (b b^dag) at j = N_m - 1 is zero
    ctop = p.kappa * 0 + p.gamma_m * (1 + p.n_th) * 3 + 0.0
    assert np.isclose(D[pos(0, 3, 0, 3), pos(0, 3, 0, 3)], -ctop)


def test_trace_forms_and_row_zero():
    p = W.TINY
    N = p.nc * p.nm
    L = model.liouvillian(p)
    Lr, br, w = model.constrained_system(L, model.TRACE_REPLACE)
    La, ba, _ = model.constrained_system(L, model.TRACE_ADD)
    row = Lr.getrow(0)
    assert set(row.indices.tolist()) == set((np.arange(N) * (N + 1)).tolist())
    assert np.allclose(row.data, w)
    assert br[0] == w and not np.any(br[1:])
    # the additive row differs from the replaced one by exactly row 0 of L
    d = (La - Lr).getrow(0).toarray().ravel() - L.getrow(0).toarray().ravel()
    assert np.max(np.abs(d)) <= 1e-15
