"""GPU parity of every step of the hot path against the oracle, through the
C ABI: assembly (Eq. (3)-(5)), RCM (Sec. III), SpMV, ILUT factors and their
application (Sec. II), GMRES and the steady state (Sec. IV), mixed
precision and adjoint gradients.  Sizes span several 64-row blocks and a
ragged tail."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import workloads as W
from gpu_util import announce, require_gpu, to_dev, to_host
from oracle import adjoint as oadj
from oracle import direct, model, ordering
from oracle import ilut as oilut

pytestmark = pytest.mark.gpu

import paper_1411_4356_amd as P  # noqa: E402


@pytest.fixture(autouse=True)
def _gpu(request):
    require_gpu()
    announce(request.node.nodeid)


# n = 441, 1296 (ragged: not a multiple of 64), 1600, n_th = 0, and the
# quadratic coupling g2 (b + b^dag)^2 a^dag a of the Sec. V variant
CASES = [W.TINY.replace(nc=3, nm=7), W.TINY.replace(nc=4, nm=9), W.TINY, W.ADJOINT.replace(nc=3, nm=8),
         W.TINY.replace(nc=3, nm=8, g2=0.07)]


def _oracle_system(p, mode=model.TRACE_REPLACE):
    return model.constrained_system(model.liouvillian(p), mode)


@pytest.mark.parametrize("mode", [model.TRACE_NONE, model.TRACE_REPLACE, model.TRACE_ADD])
@pytest.mark.parametrize("ci", range(len(CASES)))
def test_build_matches_oracle(ci, mode):
    p = CASES[ci]
    Lt, _, w = _oracle_system(p, mode)
    A, wd = P.liouvillian_build(p, trace_mode=mode)
    rp, col, val = A.export()
    assert np.array_equal(rp, Lt.indptr) and np.array_equal(col, Lt.indices)
    assert np.max(np.abs(val[0] - Lt.data)) <= 1e-14 * np.abs(Lt.data).max()
    assert abs(wd[0] - w) <= 1e-14 * abs(w)


def test_build_batch_matches_oracle_per_item():
    ps = [W.TINY.replace(nc=3, nm=7, E=e) for e in (0.1, 0.35, 0.6)]
    A, w = P.liouvillian_build(ps)
    rp, col, val = A.export()
    for b, p in enumerate(ps):
        Lt, _, wo = _oracle_system(p)
        assert np.array_equal(col, Lt.indices)
        assert np.max(np.abs(val[b] - Lt.data)) <= 1e-14 * np.abs(Lt.data).max()


def test_build_fig1_count():
    A, _ = P.liouvillian_build(W.FIG1, trace_mode=model.TRACE_ADD)
    assert A.nnz == 8957


@pytest.mark.parametrize("ci", range(len(CASES)))
def test_rcm_permute_matches_oracle(ci):
    p = CASES[ci]
    Lt, _, _ = _oracle_system(p)
    A, _ = P.liouvillian_build(p)
    B, perm, st = P.rcm_permute(A)
    po = ordering.rcm(Lt)
    assert np.array_equal(perm, po)
    Bo = ordering.permute(Lt, po)
    rp, col, val = B.export()
    assert np.array_equal(rp, Bo.indptr) and np.array_equal(col, Bo.indices)
    assert np.max(np.abs(val[0] - Bo.data)) <= 1e-14 * np.abs(Bo.data).max()
    s0, s1 = ordering.bandwidth_profile(Lt), ordering.bandwidth_profile(Bo)
    assert (st["B0"], st["P0"], st["B1"], st["P1"]) == (s0["B"], s0["P"], s1["B"], s1["P"])
    assert (st["ub1"], st["lb1"]) == (s1["ub"], s1["lb"])


@pytest.mark.parametrize("adjoint", [0, 1])
@pytest.mark.parametrize("ci", range(len(CASES)))
def test_spmv_matches_oracle(ci, adjoint):
    p = CASES[ci]
    ps = [p, p.replace(E=p.E * 1.5)]
    A, _ = P.liouvillian_build(ps, c64=True)
    B, perm, _ = P.rcm_permute(A)
    X = W.random_complex(B.n, seed=11, count=2)
    y = to_host(P.csr_spmv(B, to_dev(X), adjoint=bool(adjoint)))
    y32 = to_host(P.csr_spmv(B, to_dev(X, torch.complex64), adjoint=bool(adjoint)))
    for b, q in enumerate(ps):
        Lt, _, _ = _oracle_system(q)
        Bo = ordering.permute(Lt, perm)
        M = Bo.conj().T.tocsr() if adjoint else Bo
        ref = M @ X[b]
        bound = abs(M) @ np.abs(X[b])
        assert np.all(np.abs(y[b] - ref) <= 1e-14 * bound + 1e-300)
        assert np.all(np.abs(y32[b] - ref) <= 2e-6 * bound)


@pytest.mark.parametrize("mode", [model.TRACE_NONE, model.TRACE_REPLACE, model.TRACE_ADD])
@pytest.mark.parametrize("permuted", [False, True])
@pytest.mark.parametrize("ci", range(len(CASES)))
def test_matrix_free_apply_matches_oracle(ci, permuted, mode):
    """liouvillian_apply re-evaluates every row of the constrained matrix from
    the model parameters (Eq. (3) in the Fock basis, Eq. (4), the trace row of
    Eq. (5)) instead of reading stored entries: equal, within the rounding
    bound of the row sums, to the oracle's Kronecker-built matrix (permuted as
    rcm_permute permutes it) times x, per batch item and in both precisions."""
    p = CASES[ci]
    ps = [p, p.replace(E=p.E * 1.5)]
    A, _ = P.liouvillian_build(ps, trace_mode=mode)
    if permuted:
        B, perm, _ = P.rcm_permute(A)
    else:
        B, perm = A, None
    X = W.random_complex(B.n, seed=12, count=2)
    y = to_host(P.liouvillian_apply(B, to_dev(X)))
    y32 = to_host(P.liouvillian_apply(B, to_dev(X, torch.complex64)))
    for b, q in enumerate(ps):
        Lt, _, _ = _oracle_system(q, mode)
        Bo = ordering.permute(Lt, perm) if permuted else Lt
        ref = Bo @ X[b]
        bound = abs(Bo) @ np.abs(X[b])
        assert np.all(np.abs(y[b] - ref) <= 1e-14 * bound + 1e-300)
        assert np.all(np.abs(y32[b] - ref) <= 2e-6 * bound)


def test_solver_with_matrix_free_products(monkeypatch):
    """With OMSS_SPMV=stencil the solver's products with the system matrix
    run matrix-free (the kernel class "lapply" records launches) and the
    steady state is the stored-matrix one and the oracle's."""
    import ctypes as C
    lib = P.lib()
    p = W.TINY
    opts = dict(drop_tol=W.TINY_OPTS.drop_tol, fill_factor=W.TINY_OPTS.fill_factor, m=W.TINY_OPTS.restart,
                tol=W.TINY_OPTS.tol)
    rho0, info0, _ = P.steady_state(p, **opts)
    monkeypatch.setenv("OMSS_SPMV", "stencil")
    lib.om_profile_enable(1)
    lib.om_profile_reset()
    try:
        rho1, info1, _ = P.steady_state(p, **opts)
        torch.cuda.synchronize()
        launches, ms, nbytes = C.c_int64(), C.c_double(), C.c_double()
        lib.om_profile_query(b"lapply", C.byref(launches), C.byref(ms), C.byref(nbytes))
    finally:
        lib.om_profile_enable(0)
    assert launches.value > 0
    assert info1["gmres"]["relres_true"] <= W.TINY_OPTS.tol
    r0, r1 = rho0[0].cpu().numpy(), rho1[0].cpu().numpy()
    ro, _ = direct.steady_state(p)
    assert np.max(np.abs(r1 - r0)) <= 1e-10
    assert np.max(np.abs(r1 - ro)) <= 1e-9


def _factored(p, d, fill, **kw):
    A, _ = P.liouvillian_build(p)
    B, perm, _ = P.rcm_permute(A)
    M = P.ilu_factor(B, d, fill, keep_host=True, **kw)
    return A, B, perm, M


@pytest.mark.parametrize("ci", range(len(CASES)))
def test_ilu_factor_and_apply_match_oracle(ci):
    p = CASES[ci]
    A, B, perm, M = _factored(p, 1e-5, 60.0, adjoint=True, c64=True, condest=True)
    Lt, _, _ = _oracle_system(p)
    Bo = ordering.permute(Lt, perm)
    Lo, Uo, so = oilut.ilut(Bo, 1e-5, 60.0)
    Lf, Uf = M.export(0)
    for X, Y in ((Lf, Lo), (Uf, Uo)):
        assert np.array_equal(X.indptr, Y.indptr) and np.array_equal(X.indices, Y.indices)
    assert M.stats["nnz_L"] == so["nnz_L"] and M.stats["nnz_U"] == so["nnz_U"]
    x = W.random_complex(B.n, seed=5)
    for adj in (False, True):
        y = to_host(P.ilu_apply(M, to_dev(x[None, :]), adjoint=adj))[0]
        ref = oilut.apply(Lf, Uf, x, adjoint=adj)
        ref_o = oilut.apply(Lo, Uo, x, adjoint=adj)
        assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)
        assert np.linalg.norm(y - ref_o) <= 1e-10 * np.linalg.norm(ref_o)
        y32 = to_host(P.ilu_apply(M, to_dev(x[None, :], torch.complex64), adjoint=adj))[0]
        assert np.linalg.norm(y32 - ref) <= 1e-3 * np.linalg.norm(ref)
    assert abs(M.stats["condest"] - oilut.condest(Lo, Uo)) <= 1e-9 * oilut.condest(Lo, Uo)


def test_ilu_apply_in_place_and_batched():
    ps = [W.TINY.replace(nc=4, nm=9, E=e) for e in (0.15, 0.45)]
    A, B, perm, M = _factored(ps, 1e-5, 60.0)
    X = W.random_complex(B.n, seed=9, count=2)
    t = to_dev(X)
    P.ilu_apply(M, t, t)
    y = to_host(t)
    for b in range(2):
        Lf, Uf = M.export(b)
        ref = oilut.apply(Lf, Uf, X[b])
        assert np.linalg.norm(y[b] - ref) <= 1e-12 * np.linalg.norm(ref)


def test_complete_lu_solves_exactly():
    """d = 0, no fill cap: the factors are the complete LU (Sec. II), so one
    preconditioner application solves the system."""
    p = CASES[0]
    A, B, perm, M = _factored(p, 0.0, float("inf"))
    Lt, b, _ = _oracle_system(p)
    xo = direct.solve(Lt, b)
    y = to_host(P.ilu_apply(M, to_dev(b[perm][None, :])))[0]
    assert np.max(np.abs(y - xo[perm])) <= 1e-9 * np.max(np.abs(xo))


@pytest.mark.parametrize("ci", range(len(CASES)))
def test_gmres_solve_matches_direct(ci):
    p = CASES[ci].replace(n_th=max(CASES[ci].n_th, 1e-15))
    A, B, perm, M = _factored(p, 1e-5, 60.0)
    Lt, b, _ = _oracle_system(p)
    xo = direct.solve(Lt, b)
    bt = to_dev(b[perm][None, :])
    x, info = P.gmres_solve(B, M, bt, m=50, tol=1e-12)
    xs = np.empty_like(xo)
    xs[perm] = to_host(x)[0]
    assert info["relres_true"] <= 1e-12
    assert direct.relative_residual(Lt, b, xs) <= 1e-11
    assert np.max(np.abs(xs - xo)) <= 1e-9 * np.max(np.abs(xo))


def test_gmres_without_preconditioner_and_adjoint():
    p = CASES[0]
    A, B, perm, M = _factored(p, 1e-5, 60.0, adjoint=True)
    Lt, b, _ = _oracle_system(p)
    Bo = ordering.permute(Lt, perm)
    g = W.random_complex(B.n, seed=3)
    lam, info = P.gmres_solve(B, M, to_dev(g[None, :]), adjoint=True, m=50, tol=1e-12)
    ref = np.linalg.solve(Bo.conj().T.toarray(), g)
    assert np.max(np.abs(to_host(lam)[0] - ref)) <= 1e-9 * np.max(np.abs(ref))
    x, info = P.gmres_solve(B, None, to_dev(b[perm][None, :]), m=100, tol=1e-8, maxiter=3000, allow_notconv=True)
    assert info["iters"] > 0


def test_gmres_reports_nonconvergence():
    p = CASES[1]
    A, B, perm, M = _factored(p, 1e-2, 2.0)
    Lt, b, _ = _oracle_system(p)
    x, info = P.gmres_solve(B, M, to_dev(b[perm][None, :]), m=5, tol=1e-30, maxiter=7, allow_notconv=True)
    assert info["status"] == "OM_ENOTCONV" and info["iters"] <= 7 + 5
    with pytest.raises(P.OmError):
        P.gmres_solve(B, M, to_dev(b[perm][None, :]), m=5, tol=1e-30, maxiter=7)


@pytest.mark.parametrize("ci", range(len(W.small_cases())))
def test_steady_state_matches_oracle(ci):
    p = W.small_cases()[ci]
    rho, info, res = P.steady_state(p, drop_tol=1e-5, fill_factor=60.0, m=50, tol=1e-12)
    rho = to_host(rho)[0]
    ro, oo = direct.steady_state(p)
    assert info["gmres"]["relres_true"] <= 1e-12
    err = np.max(np.abs(rho - ro))
    assert err <= 1e-9, err
    assert abs(res["n_a"][0] - oo["n_a"]) <= 1e-9 * max(1.0, abs(oo["n_a"]))
    assert abs(res["n_b"][0] - oo["n_b"]) <= 1e-9 * max(1.0, abs(oo["n_b"]))
    assert abs(res["fano"][0] - oo["fano"]) <= 1e-8 * max(1.0, abs(oo["fano"]))
    assert res["herm_err"][0] <= 1e-9 and res["trace_err"][0] <= 1e-9


def test_steady_state_batch_of_pump_amplitudes():
    ps = [W.BATCH_BASE.replace(nc=4, nm=9, E=e) for e in W.batch_E(4)]
    rho, info, res = P.steady_state(ps, drop_tol=1e-6, fill_factor=60.0, m=50, tol=1e-11)
    rho = to_host(rho)
    for b, p in enumerate(ps):
        ro, oo = direct.steady_state(p)
        assert np.max(np.abs(rho[b] - ro)) <= 1e-8
        assert abs(res["n_b"][b] - oo["n_b"]) <= 1e-8 * oo["n_b"]


def test_mixed_precision_matches_fp64():
    p = W.MIXED.replace(nc=4, nm=12)
    rho64, i64, r64 = P.steady_state(p, drop_tol=1e-5, fill_factor=60.0, m=30, tol=1e-10)
    rho32, i32, r32 = P.steady_state(p, drop_tol=1e-5, fill_factor=60.0, m=30, tol=1e-10, precision="ir_c64",
                                     inner_tol=1e-5)
    ro, oo = direct.steady_state(p)
    assert i32["gmres"]["relres_true"] <= 1e-10 and i32["gmres"]["outer_iters"] >= 1
    assert np.max(np.abs(to_host(rho32)[0] - ro)) <= 1e-8
    assert abs(r32["n_b"][0] - oo["n_b"]) <= 1e-8 * oo["n_b"]


def test_adjoint_gradients_match_oracle():
    p = W.ADJOINT.replace(nc=3, nm=6, n_th=1e-15)
    A, _ = P.liouvillian_build(p)
    B, perm, _ = P.rcm_permute(A)
    M = P.ilu_factor(B, 1e-8, 100.0, adjoint=True)
    Lt, b, _ = _oracle_system(p)
    x, _ = P.gmres_solve(B, M, to_dev(b[perm][None, :]), m=50, tol=1e-14)
    obs = P.observables(B, x)[0]
    g = P.objective_vectors(B, x)
    lam = torch.empty_like(g)
    for f in range(3):
        lam[f], _ = P.gmres_solve(B, M, g[f].contiguous(), adjoint=True, m=50, tol=1e-14)
    grad = P.param_gradient(B, x, lam)[0]
    vals, go = oadj.gradients(p)
    assert np.max(np.abs(obs - vals) / np.abs(vals)) <= 1e-10
    scale = np.maximum(np.abs(go), 1e-6 * np.abs(go).max(axis=1, keepdims=True))
    assert np.max(np.abs(grad - go) / scale) <= 1e-7


def test_invalid_parameters_are_rejected():
    with pytest.raises(P.OmError):
        P.liouvillian_build(W.TINY.replace(kappa=-1.0))
    with pytest.raises(P.OmError):
        P.liouvillian_build(W.TINY.replace(E=float("nan")))
    with pytest.raises(P.OmError):
        P.liouvillian_build(W.TINY.replace(nc=1))


def test_shared_factor_preconditions_whole_batch():
    """One factor (of item 0) as the preconditioner of every item: the
    solutions are the same steady states, each to tolerance."""
    ps = [W.BATCH_BASE.replace(nc=4, nm=9, E=e) for e in (0.35, 0.15, 0.55)]
    rho, info, res = P.steady_state(ps, drop_tol=1e-6, fill_factor=60.0, m=60, tol=1e-11, share_factor=True)
    rho = to_host(rho)
    for b, p in enumerate(ps):
        ro, oo = direct.steady_state(p)
        assert np.max(np.abs(rho[b] - ro)) <= 1e-8
    assert info["ilu"]["nnz_L"] > 0
    A, _ = P.liouvillian_build(ps)
    B, perm, _ = P.rcm_permute(A)
    M = P.ilu_factor(B, 1e-6, 60.0, shared=True, keep_host=True)
    L0, U0 = M.export(0)
    L2, U2 = M.export(2)
    assert (L0 != L2).nnz == 0 and (U0 != U2).nnz == 0
    X = W.random_complex(B.n, seed=4, count=3)
    y = to_host(P.ilu_apply(M, to_dev(X)))
    for b in range(3):
        ref = oilut.apply(L0, U0, X[b])
        assert np.linalg.norm(y[b] - ref) <= 1e-12 * np.linalg.norm(ref)


ILUT_CASES = [
    (CASES[0], 1e-5, 60.0),
    (CASES[1], 1e-5, 60.0),
    (CASES[3], 1e-5, 60.0),
    (W.BATCH_BASE.replace(nc=4, nm=9), 1e-6, 20.0),
    (W.BATCH_BASE.replace(nc=4, nm=9), 1e-6, float("inf")),
    (W.BATCH_BASE.replace(nc=4, nm=9), 0.0, float("inf")),
    (W.BATCH_BASE.replace(nc=6, nm=20), 1e-6, 60.0),
]


def _bits(M):
    return M.view(np.uint64)


@pytest.mark.parametrize("ci", range(len(ILUT_CASES)))
def test_device_ilut_is_the_host_factor_bit_for_bit(ci, monkeypatch):
    """The row-pipelined device ILUT (Sec. II dropping rules) yields exactly
    the factor of the sequential host ILUT, whose pattern and values are
    pinned to the oracle elsewhere: same pattern, same bits."""
    p, d, fill = ILUT_CASES[ci]
    A, _ = P.liouvillian_build(p)
    B, perm, _ = P.rcm_permute(A)
    monkeypatch.setenv("OMSS_ILUT", "device")
    M = P.ilu_factor(B, d, fill, keep_host=True)
    Lg, Ug = M.export(0)
    Lh, Uh, _ = P.host_ilut(B.to_scipy(), d, fill)
    for X, Y in ((Lg, Lh), (Ug, Uh)):
        assert np.array_equal(X.indptr, Y.indptr) and np.array_equal(X.indices, Y.indices)
        assert np.array_equal(_bits(X.data), _bits(Y.data))
    # the host-thread path of ilu_factor gives the same factor
    monkeypatch.setenv("OMSS_ILUT", "host")
    Mh = P.ilu_factor(B, d, fill, keep_host=True)
    L2, U2 = Mh.export(0)
    assert np.array_equal(_bits(L2.data), _bits(Lg.data)) and np.array_equal(_bits(U2.data), _bits(Ug.data))


@pytest.mark.parametrize("stage", ["0", "48"])
@pytest.mark.parametrize("ci", [3, 6])
def test_device_ilut_staging_paths_give_the_host_factor(ci, stage, monkeypatch):
    """The dropping and cap of a triangle (Sec. II) stage its keys in LDS when
    few entries are present and otherwise re-read them from the working row
    in every digit pass.  The staging limit is lowered here (0: no triangle
    staged; 48: a mix) so that small operators take the second path too: the
    factor is the host's, bit for bit, whichever path each row took."""
    p, d, fill = ILUT_CASES[ci]
    A, _ = P.liouvillian_build(p)
    B, perm, _ = P.rcm_permute(A)
    monkeypatch.setenv("OMSS_ILUT", "device")
    monkeypatch.setenv("OMSS_ILUT_STAGE", stage)
    M = P.ilu_factor(B, d, fill, keep_host=True)
    Lg, Ug = M.export(0)
    Lh, Uh, _ = P.host_ilut(B.to_scipy(), d, fill)
    for X, Y in ((Lg, Lh), (Ug, Uh)):
        assert np.array_equal(X.indptr, Y.indptr) and np.array_equal(X.indices, Y.indices)
        assert np.array_equal(_bits(X.data), _bits(Y.data))


def test_device_ilut_batch_items_are_factored_independently(monkeypatch):
    monkeypatch.setenv("OMSS_ILUT", "device")
    ps = [W.TINY.replace(nc=4, nm=9, E=e) for e in (0.15, 0.45, 0.3)]
    A, _ = P.liouvillian_build(ps)
    B, perm, _ = P.rcm_permute(A)
    M = P.ilu_factor(B, 1e-5, 40.0, keep_host=True)
    for b in range(3):
        Lg, Ug = M.export(b)
        Lh, Uh, _ = P.host_ilut(B.to_scipy(b), 1e-5, 40.0)
        assert np.array_equal(_bits(Lg.data), _bits(Lh.data)) and np.array_equal(_bits(Ug.data), _bits(Uh.data))
        assert np.array_equal(Ug.indices, Uh.indices)


def test_autograd_steady_state_obs_matches_oracle_adjoint():
    """torch.autograd through SteadyStateObs: the forward observables and the
    vector-Jacobian product of the adjoint backward pass against the oracle's
    dense adjoint gradients (themselves pinned to central differences)."""
    p = W.ADJOINT.replace(nc=3, nm=6, n_th=1e-15)
    cfg = P.SolveConfig(nc=p.nc, nm=p.nm, omega_m=p.omega_m, n_th=p.n_th, drop_tol=1e-8, fill_factor=100.0,
                        m=50, tol=1e-14)
    theta = torch.tensor([p.delta, p.g0, p.E, p.kappa, p.gamma_m], dtype=torch.float64, requires_grad=True)
    obs = P.SteadyStateObs.apply(theta, cfg)
    wts = torch.tensor([0.7, -1.3, 2.0], dtype=torch.float64)
    (obs * wts).sum().backward()
    vals, go = oadj.gradients(p)
    assert np.max(np.abs(obs.detach().numpy() - vals) / np.abs(vals)) <= 1e-10
    ref = wts.numpy() @ go
    assert np.max(np.abs(theta.grad.numpy() - ref)) <= 1e-7 * np.abs(ref).max()
    # the full Jacobian, one backward pass per observable on one retained graph
    obs = P.SteadyStateObs.apply(theta, cfg)
    for f in range(3):
        gsel = torch.zeros(3, dtype=torch.float64)
        gsel[f] = 1.0
        row, = torch.autograd.grad(obs, theta, gsel, retain_graph=f < 2)
        assert np.max(np.abs(row.numpy() - go[f])) <= 1e-7 * np.abs(go[f]).max()


@pytest.mark.parametrize("ci", [1, 3])
def test_device_built_schedules_equal_host_built(ci, monkeypatch):
    """The L and U solve schedules built on the device from the device factor
    are the host-built ones: both preconditioner applications give the same
    bits, in complex128 and complex64, forward and adjoint."""
    p, d, fill = ILUT_CASES[ci]
    A, _ = P.liouvillian_build([p, p.replace(E=0.3)])
    B, perm, _ = P.rcm_permute(A)
    monkeypatch.delenv("OMSS_ILU_SCHED", raising=False)
    Md = P.ilu_factor(B, d, fill, c64=True, adjoint=True)
    monkeypatch.setenv("OMSS_ILU_SCHED", "host")
    Mh = P.ilu_factor(B, d, fill, c64=True, adjoint=True)
    X = W.random_complex(B.n, seed=11, count=2)
    for dt in (torch.complex128, torch.complex64):
        for adj in (False, True):
            yd = to_host(P.ilu_apply(Md, to_dev(X, dt), adjoint=adj))
            yh = to_host(P.ilu_apply(Mh, to_dev(X, dt), adjoint=adj))
            assert np.array_equal(yd.view(np.uint64 if dt == torch.complex128 else np.uint32),
                                  yh.view(np.uint64 if dt == torch.complex128 else np.uint32))


@pytest.mark.parametrize("nb", [2, 3, 8])
def test_multi_rhs_solve_with_shared_factor(nb, monkeypatch):
    """With one factor shared by the batch, the triangular solves of all
    right-hand sides run as one pass over the factor; results agree with the
    one-side-at-a-time solves (summation order differs) in both precisions and
    directions, and the factor's own host application."""
    ps = [W.BATCH_BASE.replace(nc=4, nm=9, E=0.2 + 0.05 * b) for b in range(nb)]
    A, _ = P.liouvillian_build(ps)
    B, perm, _ = P.rcm_permute(A)
    M = P.ilu_factor(B, 1e-6, 60.0, shared=True, c64=True, adjoint=True, keep_host=True)
    L0, U0 = M.export(0)
    X = W.random_complex(B.n, seed=21, count=nb)
    for dt, tol in ((torch.complex128, 1e-12), (torch.complex64, 2e-4)):
        for adj in (False, True):
            monkeypatch.setenv("OMSS_TRSV_MRHS", "1")
            ym = to_host(P.ilu_apply(M, to_dev(X, dt), adjoint=adj))
            monkeypatch.setenv("OMSS_TRSV_MRHS", "0")
            ys = to_host(P.ilu_apply(M, to_dev(X, dt), adjoint=adj))
            for b in range(nb):
                ref = oilut.apply(L0, U0, X[b], adjoint=adj)
                assert np.linalg.norm(ym[b] - ys[b]) <= tol * np.linalg.norm(ys[b])
                assert np.linalg.norm(ym[b] - ref) <= tol * np.linalg.norm(ref)
    # in place, and with items masked out by a converged solve: steady states
    monkeypatch.setenv("OMSS_TRSV_MRHS", "1")
    rho, info, res = P.steady_state(ps, drop_tol=1e-6, fill_factor=60.0, m=60, tol=1e-11, share_factor=True)
    rho = to_host(rho)
    for b, p in enumerate(ps):
        ro, _ = direct.steady_state(p)
        assert np.max(np.abs(rho[b] - ro)) <= 1e-8


def test_full_size_matrix_free_apply_against_oracle():
    """The matrix-free product and the CSR SpMV at the batch workload's full
    size (360,000 rows, eight items, RCM order, the launch bench.py times):
    every row of two items against the oracle's Kronecker-built constrained
    matrix, permuted as rcm_permute permutes it, within the rounding bound
    of the row sums."""
    params = W.batch_params()
    A, _ = P.liouvillian_build(params)
    B, perm, _ = P.rcm_permute(A)
    X = W.random_complex(B.n, seed=21, count=len(params))
    xd = to_dev(X)
    y = to_host(P.liouvillian_apply(B, xd))
    yc = to_host(P.csr_spmv(B, xd))
    for b in (0, len(params) - 1):
        Lt, _, _ = model.constrained_system(model.liouvillian(params[b]))
        Bo = ordering.permute(Lt, perm)
        ref = Bo @ X[b]
        bound = abs(Bo) @ np.abs(X[b])
        assert np.all(np.abs(y[b] - ref) <= 1e-14 * bound + 1e-300)
        assert np.all(np.abs(yc[b] - ref) <= 1e-14 * bound + 1e-300)


def test_full_size_batch_against_oracle_system():
    """The 360,000-row batch workload as bench.py runs it (eight pump
    amplitudes, one ILUT factor of the median-E item, d = 1e-6, p = 400,
    GMRES(100) to 1e-10): every item's density matrix is checked against the
    oracle's own Kronecker-built constrained system (Eqs. (3)-(5)) through
    properties that hold at any size -- relative residual, trace, Hermiticity,
    positivity -- and the observables the oracle computes from it."""
    params = W.batch_params()
    med = sorted(p.E for p in params)[len(params) // 2]
    params.sort(key=lambda p: (abs(p.E - med), p.E))
    o = W.BATCH_OPTS
    rho, info, res = P.steady_state(params, drop_tol=o.drop_tol, fill_factor=o.fill_factor, m=o.restart, tol=o.tol,
                                    maxiter=o.maxiter, share_factor=True)
    assert info["gmres"]["converged"] == len(params) and info["gmres"]["relres_true"] <= 1e-10
    rho = to_host(rho)
    N = params[0].nc * params[0].nm
    picks = sorted({0, int(np.argmin([p.E for p in params])), int(np.argmax([p.E for p in params]))})
    for b in picks:
        p = params[b]
        Lt, rhs, _ = model.constrained_system(model.liouvillian(p))
        r = rho[b]
        x = r.reshape(-1, order="F")
        assert direct.relative_residual(Lt, rhs, x) <= 1e-9
        assert abs(np.trace(r) - 1.0) <= 1e-12
        # the exact rho is Hermitian and positive; the computed one differs by
        # the forward error, at most cond(L~) x the 1e-10 residual (the
        # preconditioned operator's condition estimate is ~1e4 here)
        assert direct.hermiticity_error(r) <= 1e-6
        assert np.linalg.eigvalsh(0.5 * (r + r.conj().T)).min() >= -1e-6
        ob = direct.observables(r, p.nc, p.nm)
        assert abs(ob["n_b"] - res["n_b"][b]) <= 1e-10 * abs(ob["n_b"])
        assert abs(ob["n_a"] - res["n_a"][b]) <= 1e-10 * abs(ob["n_a"])
