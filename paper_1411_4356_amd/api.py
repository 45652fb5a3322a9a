"""Python binding of the C ABI (argument marshalling only).

Device arrays are contiguous torch tensors on the HIP device: complex128
(or complex64 where the call takes a dtype), batch-major.  Every numerical
step runs inside libomss.so; nothing here computes any part of the method.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass
from typing import Iterable, Sequence

import numpy as np
import torch

from . import _lib as L
from ._lib import check, lib


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _params_array(params) -> tuple:
    if not isinstance(params, (list, tuple)):
        params = [params]
    arr = (L.om_params * len(params))()
    for i, p in enumerate(params):
        g = (lambda k, d=None: p.get(k, d) if isinstance(p, dict) else getattr(p, k, d))
        arr[i] = L.om_params(int(g("nc")), int(g("nm")), float(g("delta")), float(g("omega_m", 1.0) or 1.0),
                             float(g("g0")), float(g("E")), float(g("kappa")), float(g("gamma_m")),
                             float(g("n_th")), float(g("g2", 0.0) or 0.0))
    return arr, len(params)


def _ptr(t: torch.Tensor) -> C.c_void_p:
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _check_dev(t: torch.Tensor, dtypes=(torch.complex128,)):
    if t.device.type != "cuda":
        raise ValueError("device tensor expected")
    if t.dtype not in dtypes:
        raise ValueError(f"dtype {t.dtype} not in {dtypes}")


class Csr:
    """Owner of an om_csr handle."""

    def __init__(self, handle: C.c_void_p):
        self.h = handle
        n, nnz, b, N = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int32()
        check(lib().om_csr_info(self.h, C.byref(n), C.byref(nnz), C.byref(b), C.byref(N)))
        self.n, self.nnz, self.batch, self.N = n.value, nnz.value, b.value, N.value

    def __del__(self):
        if getattr(self, "h", None):
            try:
                lib().om_csr_free(self.h)
            except Exception:
                pass
            self.h = None

    def export(self, stream=None):
        """(row_ptr int64[n+1], col int32[nnz], val complex128[batch, nnz]) on the host."""
        rp = np.empty(self.n + 1, dtype=np.int64)
        col = np.empty(self.nnz, dtype=np.int32)
        val = np.empty((self.batch, self.nnz), dtype=np.complex128)
        check(lib().om_csr_export(self.h, rp.ctypes.data_as(L._pi64), col.ctypes.data_as(L._pi32),
                                  val.ctypes.data_as(L._dp), _stream(stream)))
        return rp, col, val

    def to_scipy(self, item: int = 0):
        import scipy.sparse as sp
        rp, col, val = self.export()
        return sp.csr_matrix((val[item], col, rp), shape=(self.n, self.n))


class Ilu:
    """Owner of an om_ilu handle."""

    def __init__(self, handle: C.c_void_p, stats: L.om_ilu_stats, n: int, batch: int):
        self.h = handle
        self.stats = {k: getattr(stats, k) for k, _ in L.om_ilu_stats._fields_}
        self.n = n
        self.batch = batch

    def __del__(self):
        if getattr(self, "h", None):
            try:
                lib().om_ilu_free(self.h)
            except Exception:
                pass
            self.h = None

    def export(self, item: int = 0):
        """Host CSR factors (scipy): L strictly lower, U upper with diagonal."""
        import scipy.sparse as sp
        n, nl, nu = C.c_int64(), C.c_int64(), C.c_int64()
        check(lib().om_ilu_info(self.h, item, C.byref(n), C.byref(nl), C.byref(nu)))
        if nl.value < 0:
            raise RuntimeError("factors were not kept on the host")
        n = n.value
        lp, up = np.empty(n + 1, np.int64), np.empty(n + 1, np.int64)
        lc, uc = np.empty(nl.value, np.int32), np.empty(nu.value, np.int32)
        lv, uv = np.empty(nl.value, np.complex128), np.empty(nu.value, np.complex128)
        check(lib().om_ilu_export(self.h, item, lp.ctypes.data_as(L._pi64), lc.ctypes.data_as(L._pi32),
                                  lv.ctypes.data_as(L._dp), up.ctypes.data_as(L._pi64), uc.ctypes.data_as(L._pi32),
                                  uv.ctypes.data_as(L._dp)))
        return (sp.csr_matrix((lv, lc, lp), shape=(n, n)), sp.csr_matrix((uv, uc, up), shape=(n, n)))


def liouvillian_build(params, trace_mode: int = L.OM_TRACE_REPLACE_ROW0, c64: bool = False, stream=None):
    """Device CSR of the constrained Liouvillian for one or more parameter sets;
    returns (Csr, w[batch])."""
    arr, nb = _params_array(params)
    h = C.c_void_p()
    w = (C.c_double * nb)()
    check(lib().liouvillian_build(arr, nb, trace_mode, L.OM_BUILD_C64 if c64 else 0, C.byref(h),
                                  C.cast(w, L._dp), _stream(stream)))
    return Csr(h), np.array(list(w))


def rcm_permute(A: Csr, stream=None):
    """(A_perm, perm[new] = old, stats dict)."""
    perm = np.empty(A.n, dtype=np.int32)
    h = C.c_void_p()
    st = L.om_order_stats()
    check(lib().rcm_permute(A.h, perm.ctypes.data_as(L._pi32), C.byref(h), C.byref(st), _stream(stream)))
    return Csr(h), perm, {k: getattr(st, k) for k, _ in L.om_order_stats._fields_}


def csr_permute(A: Csr, perm, stream=None):
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    h = C.c_void_p()
    check(lib().csr_permute(A.h, perm.ctypes.data_as(L._pi32), C.byref(h), _stream(stream)))
    return Csr(h)


def ilu_factor(A: Csr, drop_tol: float, fill_factor: float, c64: bool = False, adjoint: bool = False,
               condest: bool = False, keep_host: bool = False, shared: bool = False, stream=None) -> Ilu:
    flags = ((L.OM_ILU_C64 if c64 else 0) | (L.OM_ILU_ADJOINT if adjoint else 0)
             | (L.OM_ILU_CONDEST if condest else 0) | (L.OM_ILU_KEEP_HOST if keep_host else 0)
             | (L.OM_ILU_SHARED if shared else 0))
    h = C.c_void_p()
    st = L.om_ilu_stats()
    check(lib().ilu_factor(A.h, float(drop_tol), float(fill_factor), flags, C.byref(h), C.byref(st), _stream(stream)))
    return Ilu(h, st, A.n, A.batch)


def ilu_apply(M: Ilu, x: torch.Tensor, y: torch.Tensor | None = None, adjoint: bool = False, stream=None):
    _check_dev(x, (torch.complex128, torch.complex64))
    y = torch.empty_like(x) if y is None else y
    dtype = L.OM_C64 if x.dtype == torch.complex64 else L.OM_C128
    check(lib().ilu_apply(M.h, int(adjoint), dtype, _ptr(x), _ptr(y), _stream(stream)))
    return y


def csr_spmv(A: Csr, x: torch.Tensor, y: torch.Tensor | None = None, adjoint: bool = False, stream=None):
    _check_dev(x, (torch.complex128, torch.complex64))
    y = torch.empty_like(x) if y is None else y
    dtype = L.OM_C64 if x.dtype == torch.complex64 else L.OM_C128
    check(lib().csr_spmv(A.h, int(adjoint), dtype, _ptr(x), _ptr(y), _stream(stream)))
    return y


def liouvillian_apply(A: Csr, x: torch.Tensor, y: torch.Tensor | None = None, stream=None):
    """y = A x evaluated matrix-free from A's model parameters (no stored
    entry is read); A comes from liouvillian_build, possibly permuted."""
    _check_dev(x, (torch.complex128, torch.complex64))
    y = torch.empty_like(x) if y is None else y
    dtype = L.OM_C64 if x.dtype == torch.complex64 else L.OM_C128
    check(lib().liouvillian_apply(A.h, dtype, _ptr(x), _ptr(y), _stream(stream)))
    return y


@dataclass
class GmresOpts:
    m: int = 50
    maxiter: int = 1000
    tol: float = 1e-10
    precision: str = "fp64"        # or "ir_c64"
    inner_tol: float = 1e-5
    max_outer: int = 20

    def c(self) -> L.om_gmres_opts:
        prec = {"fp64": L.OM_PREC_FP64, "ir_c64": L.OM_PREC_IR_C64}[self.precision]
        return L.om_gmres_opts(self.m, self.maxiter, prec, self.max_outer, self.tol, self.inner_tol)


def _info(st) -> dict:
    return {k: getattr(st, k) for k, _ in type(st)._fields_}


def gmres_solve(A: Csr, M: Ilu | None, b: torch.Tensor, x: torch.Tensor | None = None, adjoint: bool = False,
                opts: GmresOpts | None = None, allow_notconv: bool = False, stream=None, **kw):
    """Solve A x = b (or A^H x = b) for every batch item; returns (x, info)."""
    _check_dev(b)
    opts = opts or GmresOpts(**kw)
    x = torch.zeros_like(b) if x is None else x
    info = L.om_gmres_info()
    o = opts.c()
    st = lib().gmres_solve(A.h, M.h if M is not None else None, int(adjoint), _ptr(b), _ptr(x), C.byref(o),
                           C.byref(info), _stream(stream))
    check(st, allow=(L.OM_ENOTCONV,) if allow_notconv else ())
    d = _info(info)
    d["status"] = L.STATUS_NAMES[st]
    return x, d


def default_ss_opts() -> L.om_ss_opts:
    o = L.om_ss_opts()
    lib().om_ss_opts_default(C.byref(o))
    return o


def steady_state(params, drop_tol: float = 1e-6, fill_factor: float = 60.0, m: int = 50, tol: float = 1e-10,
                 maxiter: int = 1000, precision: str = "fp64", inner_tol: float = 1e-5, max_outer: int = 20,
                 trace_mode: int = L.OM_TRACE_REPLACE_ROW0, nth0_fix: bool = True, reorder: bool = True,
                 share_factor: bool = False, allow_notconv: bool = False, stream=None):
    """rho (complex128 [batch, N, N] on the device, rho[b][k, l]), info dict and
    per-item results (trace_err, herm_err, n_a, n_b, fano, relres)."""
    arr, nb = _params_array(params)
    N = arr[0].nc * arr[0].nm
    o = default_ss_opts()
    o.drop_tol, o.fill_factor = drop_tol, fill_factor
    o.gmres = GmresOpts(m=m, maxiter=maxiter, tol=tol, precision=precision, inner_tol=inner_tol,
                        max_outer=max_outer).c()
    o.trace_mode, o.nth0_fix, o.reorder = trace_mode, int(nth0_fix), int(reorder)
    o.share_factor = int(share_factor)
    # column-major N x N per item: element (k, l) at l*N + k
    rho_cm = torch.empty((nb, N, N), dtype=torch.complex128, device="cuda")
    info = L.om_ss_info()
    bufs = {k: (C.c_double * nb)() for k in ("trace_err", "herm_err", "n_a", "n_b", "fano", "relres")}
    res = L.om_ss_results(*[C.cast(bufs[k], L._dp) for k, _ in L.om_ss_results._fields_])
    st = lib().steady_state(arr, nb, C.byref(o), _ptr(rho_cm), C.byref(info), C.byref(res), _stream(stream))
    check(st, allow=(L.OM_ENOTCONV,) if allow_notconv else ())
    d = {"order": _info(info.order), "ilu": _info(info.ilu), "gmres": _info(info.gmres)}
    for k in ("t_build_s", "t_rcm_s", "t_factor_s", "t_solve_s", "t_post_s"):
        d[k] = getattr(info, k)
    d["status"] = L.STATUS_NAMES[st]
    results = {k: np.array(list(v)) for k, v in bufs.items()}
    rho = rho_cm.transpose(1, 2)   # rho[b][k, l]
    return rho, d, results


def observables(A: Csr, x: torch.Tensor, stream=None) -> np.ndarray:
    _check_dev(x)
    out = np.empty((A.batch, 3), dtype=np.float64)
    check(lib().om_observables(A.h, _ptr(x), out.ctypes.data_as(L._dp), _stream(stream)))
    return out


def objective_vectors(A: Csr, x: torch.Tensor, stream=None) -> torch.Tensor:
    """conj(o_f) for f = (n_a, n_b, F): complex128 [3, batch, n]."""
    _check_dev(x)
    g = torch.empty((3, A.batch, A.n), dtype=torch.complex128, device=x.device)
    check(lib().om_objective_vectors(A.h, _ptr(x), _ptr(g), _stream(stream)))
    return g


def param_gradient(A: Csr, x: torch.Tensor, lam: torch.Tensor, stream=None) -> np.ndarray:
    """-Re lambda_f^H P0 (dL/dtheta) x: float64 [batch, nrhs, 5] for
    theta = (Delta, g0, E, kappa, Gamma_m); lam is [nrhs, batch, n]."""
    _check_dev(x)
    _check_dev(lam)
    nrhs = lam.shape[0]
    out = np.empty((A.batch, nrhs, 5), dtype=np.float64)
    check(lib().om_param_gradient(A.h, _ptr(x), _ptr(lam.contiguous()), nrhs, out.ctypes.data_as(L._dp),
                                  _stream(stream)))
    return out


# ---- host-only entry points --------------------------------------------------

def host_rcm(row_ptr, col) -> np.ndarray:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    n = rp.size - 1
    perm = np.empty(n, dtype=np.int32)
    check(lib().om_host_rcm(n, rp.ctypes.data_as(L._pi64), cl.ctypes.data_as(L._pi32), perm.ctypes.data_as(L._pi32)))
    return perm


def host_ilut(A, drop_tol: float, fill_factor: float):
    """Host ILUT of a scipy CSR: (Lf, Uf, stats)."""
    import scipy.sparse as sp
    A = sp.csr_matrix(A, dtype=np.complex128)
    A.sort_indices()
    rp = A.indptr.astype(np.int64)
    cl = A.indices.astype(np.int32)
    v = np.ascontiguousarray(A.data)
    h = C.c_void_p()
    st = L.om_ilu_stats()
    check(lib().om_host_ilut(A.shape[0], rp.ctypes.data_as(L._pi64), cl.ctypes.data_as(L._pi32),
                             v.ctypes.data_as(L._dp), float(drop_tol), float(fill_factor), C.byref(h), C.byref(st)))
    M = Ilu(h, st, A.shape[0], 1)
    Lf, Uf = M.export(0)
    return Lf, Uf, M.stats
