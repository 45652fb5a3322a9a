"""Host-side checks of libomss.so that need no GPU: the library loads and
exports every entry point declared in include/omss.h; the host algorithms
(RCM, ILUT, level depth) agree with the oracle exactly."""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from conftest import ROOT, read_golden
from oracle import ilut as oilut
from oracle import levels, model, ordering


@pytest.fixture(scope="module")
def P():
    import paper_1411_4356_amd as P
    P.lib()
    return P


def declared_functions():
    src = open(os.path.join(ROOT, "include", "omss.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(?:om_status|void|const char\*)\s+(\w+)\s*\(", src)
    return sorted(set(names))


def test_exports_every_declared_symbol(P):
    names = declared_functions()
    assert len(names) >= 20
    L = P.lib()
    for name in names:
        assert hasattr(L, name), name


def test_version(P):
    assert b"gfx950" in P.lib().om_version()


def _cases():
    out = []
    for p in (W.TINY, W.FIG1, W.ADJOINT.replace(nc=4, nm=9), W.TINY.replace(nc=3, nm=7)):
        for mode in (model.TRACE_REPLACE, model.TRACE_ADD):
            out.append((p, mode))
    return out


@pytest.mark.parametrize("case", range(8))
def test_host_rcm_matches_oracle(P, case):
    p, mode = _cases()[case]
    Lt, _, _ = model.constrained_system(model.liouvillian(p), mode)
    perm = P.host_rcm(Lt.indptr, Lt.indices)
    assert np.array_equal(perm, ordering.rcm(Lt))


def test_host_rcm_hand_graph_and_random_pattern(P):
    g = read_golden("rcm_hand_graph.txt")
    n = g["n"]
    r = list(range(n)) + [a for a, b in g["edges"]] + [b for a, b in g["edges"]]
    c = list(range(n)) + [b for a, b in g["edges"]] + [a for a, b in g["edges"]]
    A = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(n, n))
    A.sort_indices()
    assert P.host_rcm(A.indptr, A.indices).tolist() == g["rcm"]
    # a random non-symmetric pattern with several components
    rng = np.random.default_rng(7)
    B = sp.random(300, 300, density=0.01, random_state=rng, format="csr") + sp.identity(300, format="csr")
    B.sort_indices()
    assert np.array_equal(P.host_rcm(B.indptr, B.indices), ordering.rcm(B))


@pytest.mark.parametrize("d,fill", [(1e-5, 60.0), (1e-3, 5.0), (0.0, np.inf)])
def test_host_ilut_matches_oracle(P, d, fill):
    p = W.TINY.replace(nc=3, nm=7)
    Lt, _, _ = model.constrained_system(model.liouvillian(p))
    A = ordering.permute(Lt, ordering.rcm(Lt))
    Lf, Uf, st = P.host_ilut(A, d, fill)
    Lo, Uo, so = oilut.ilut(A, d, fill)
    for X, Y in ((Lf, Lo), (Uf, Uo)):
        assert np.array_equal(X.indptr, Y.indptr) and np.array_equal(X.indices, Y.indices)
        rel = np.abs(X.data - Y.data) / np.maximum(np.abs(Y.data), 1e-300)
        assert np.median(rel) <= 1e-14 and rel.max() <= 1e-8
    assert st["nnz_L"] == so["nnz_L"] and st["nnz_U"] == so["nnz_U"]
    assert st["repaired_pivots"] == so["repaired_pivots"]
    assert st["depth_L"] == levels.depth(levels.lower_levels(Lo))
    assert st["depth_U"] == levels.depth(levels.upper_levels(Uo))
    x = np.random.default_rng(2).standard_normal(A.shape[0]) + 0j
    y1, y2 = oilut.apply(Lf, Uf, x), oilut.apply(Lo, Uo, x)
    assert np.linalg.norm(y1 - y2) <= 1e-11 * np.linalg.norm(y2)


def test_host_ilut_hand_example(P):
    g = read_golden("ilut_hand_4x4.txt")
    A = sp.csr_matrix(np.array(g["A"], dtype=np.complex128))
    Lf, Uf, _ = P.host_ilut(A, g["d"], 1.0)
    Ld = dict(zip(zip(*sp.find(Lf)[:2]), sp.find(Lf)[2]))
    Ud = dict(zip(zip(*sp.find(Uf)[:2]), sp.find(Uf)[2]))
    assert set(Ld) == set(g["L_p1"]) and set(Ud) == set(g["U_p1"])
    for k, v in g["U_p1"].items():
        assert abs(Ud[k] - v) <= 1e-15


def test_host_entry_points_reject_bad_input(P):
    from paper_1411_4356_amd._lib import OmError
    A = sp.identity(4, format="csr", dtype=np.complex128)
    with pytest.raises(OmError):
        P.host_ilut(A, -1.0, 10.0)
    with pytest.raises(OmError):
        P.host_ilut(A, 1e-3, 0.0)
    with pytest.raises(OmError):
        P.host_rcm(np.array([0, 1]), np.array([5]))


@pytest.mark.parametrize("threads", ["1", "3", "8"])
def test_host_ilut_threads_bit_identical(P, threads, monkeypatch):
    """The row-pipelined multi-threaded factorisation gives the same factor,
    bit for bit, as the sequential one (and as the oracle's pattern)."""
    p = W.BATCH_BASE.replace(nc=4, nm=9)
    Lt, _, _ = model.constrained_system(model.liouvillian(p))
    A = ordering.permute(Lt, ordering.rcm(Lt))
    monkeypatch.setenv("OMSS_HOST_THREADS", "1")
    L1, U1, s1 = P.host_ilut(A, 1e-6, 20.0)
    monkeypatch.setenv("OMSS_HOST_THREADS", threads)
    L2, U2, s2 = P.host_ilut(A, 1e-6, 20.0)
    for X, Y in ((L1, L2), (U1, U2)):
        assert np.array_equal(X.indptr, Y.indptr) and np.array_equal(X.indices, Y.indices)
        assert np.array_equal(X.data, Y.data)
    Lo, Uo, _ = oilut.ilut(A, 1e-6, 20.0)
    assert np.array_equal(L2.indices, Lo.indices) and np.array_equal(U2.indices, Uo.indices)


def test_host_ilut_reports_breakdown(P):
    """An unstable incomplete factorisation (too little fill) is reported as
    breakdown rather than returned with non-finite entries."""
    from paper_1411_4356_amd._lib import OmError, OM_EBREAKDOWN
    A = sp.csr_matrix(np.array([[1.0, 1e300, 0.0], [1e300, 1.0, 1e300], [0.0, 1e300, 1.0]], dtype=np.complex128))
    with pytest.raises(OmError) as e:
        P.host_ilut(A, 0.0, float("inf"))
    assert e.value.status == OM_EBREAKDOWN
