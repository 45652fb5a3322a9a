"""Pins of the oracle bandwidth/profile (Sec. II) and RCM (Sec. III)."""
import numpy as np
import scipy.sparse as sp

import workloads as W
from conftest import read_golden
from oracle import model, ordering


def _graph(g):
    n = g["n"]
    rows = list(range(n))
    cols = list(range(n))
    for a, b in g["edges"]:
        rows += [a, b]
        cols += [b, a]
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))


def test_hand_worked_rcm():
    g = read_golden("rcm_hand_graph.txt")
    A = _graph(g)
    assert ordering.cuthill_mckee(A).tolist() == g["cm"]
    assert ordering.rcm(A).tolist() == g["rcm"]


def test_hand_worked_bandwidth_profile():
    g = read_golden("rcm_hand_graph.txt")
    r, c = zip(*g["pattern"])
    A = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(4, 4))
    st = ordering.bandwidth_profile(A)
    for k in ("ub", "lb", "B", "up", "lp", "P"):
        assert st[k] == g[k], k


def test_fig1_reductions():
    """Fig. 1: RCM lowers the total bandwidth about 5x and the profile about
    2.5x."""
    g = read_golden("fig1_structure.txt")
    L = model.liouvillian(W.FIG1)
    Lt, _, _ = model.constrained_system(L, model.TRACE_ADD)
    s0 = ordering.bandwidth_profile(Lt)
    s1 = ordering.bandwidth_profile(ordering.permute(Lt, ordering.rcm(Lt)))
    rb = s0["B"] / s1["B"]
    rp = s0["P"] / s1["P"]
    assert 0.8 * g["bandwidth_reduction_approx"] <= rb <= 1.25 * g["bandwidth_reduction_approx"]
    assert 0.8 * g["profile_reduction_approx"] <= rp <= 1.25 * g["profile_reduction_approx"]


def test_bfs_order_properties_on_model_graph():
    """Brute-force checks of the Cuthill-McKee order: it is a permutation; the
    first node has minimum degree; BFS levels never decrease along the order;
    the children of each parent appear in ascending (degree, index)."""
    p = W.TINY.replace(nc=3, nm=5)
    Lt, _, _ = model.constrained_system(model.liouvillian(p))
    S = ordering.symmetrised_pattern(Lt)
    deg = np.diff(S.indptr)
    cm = ordering.cuthill_mckee(Lt)
    n = S.shape[0]
    assert sorted(cm.tolist()) == list(range(n))
    assert deg[cm[0]] == deg.min()
    pos = np.empty(n, dtype=int)
    pos[cm] = np.arange(n)
    # parent of each node = earliest-ordered neighbour ordered before it
    parent = {}
    for v in cm[1:]:
        nb = S.indices[S.indptr[v]:S.indptr[v + 1]]
        earlier = [u for u in nb if pos[u] < pos[v] and u != v]
        assert earlier, "connected graph: every later node has an earlier neighbour"
        parent[v] = min(earlier, key=lambda u: pos[u])
    # BFS: parents are non-decreasing along the order
    ps = [pos[parent[v]] for v in cm[1:]]
    assert all(a <= b for a, b in zip(ps, ps[1:]))
    # children of one parent sorted by (degree, index)
    for par in set(parent.values()):
        kids = [v for v in cm[1:] if parent[v] == par]
        assert kids == sorted(kids, key=lambda u: (deg[u], u))


def test_rcm_is_reverse_of_cm_and_permute_roundtrip():
    p = W.TINY
    Lt, _, _ = model.constrained_system(model.liouvillian(p))
    perm = ordering.rcm(Lt)
    assert np.array_equal(perm, ordering.cuthill_mckee(Lt)[::-1])
    B = ordering.permute(Lt, perm)
    inv = ordering.inverse_permutation(perm)
    back = ordering.permute(B, inv)
    assert (back != Lt).nnz == 0
