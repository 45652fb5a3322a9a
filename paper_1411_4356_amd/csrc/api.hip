// C ABI of libomss (compiled as HIP: it holds one small kernel): argument checking, handle lifetime, the steady-state
// pipeline.  Every entry point catches C++ exceptions and reports them as a
// status; nothing throws across the ABI.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "common.hpp"
#include "gmres.hpp"
#include "ilu.hpp"
#include "ilut.hpp"
#include "kernels.hpp"
#include "ordering.hpp"
#include "post.hpp"

namespace omss {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}
const char* last_error() { return g_err.c_str(); }

template <typename F>
static om_status guarded(F&& f) {
    try {
        return f();
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return OM_ENOMEM;
    } catch (const std::exception& e) {
        set_error("internal error: %s", e.what());
        return OM_EINVAL;
    } catch (...) {
        set_error("internal error");
        return OM_EINVAL;
    }
}

static double secs_since(std::chrono::steady_clock::time_point t) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t).count();
}

static om_status check_gmres_opts(const om_gmres_opts* o) {
    if (!o) { set_error("gmres options are null"); return OM_EINVAL; }
    if (o->m < 1 || o->m > 127) { set_error("restart length m must be in 1..127 (got %d)", o->m); return OM_EINVAL; }
    if (!(o->tol > 0.0)) { set_error("tol must be > 0"); return OM_EINVAL; }
    if (o->maxiter < 1) { set_error("maxiter must be >= 1"); return OM_EINVAL; }
    if (o->precision != OM_PREC_FP64 && o->precision != OM_PREC_IR_C64) { set_error("unknown precision %d", o->precision); return OM_EINVAL; }
    if (o->precision == OM_PREC_IR_C64 && (!(o->inner_tol > 0.0) || o->max_outer < 1)) {
        set_error("GMRES-IR needs inner_tol > 0 and max_outer >= 1");
        return OM_EINVAL;
    }
    return OM_OK;
}

static void fill_gmres_info(const CoreResult& r, int outer, double t, om_gmres_info* info) {
    if (!info) return;
    std::memset(info, 0, sizeof *info);
    for (size_t i = 0; i < r.iters.size(); ++i) {
        info->iters = std::max(info->iters, r.iters[i]);
        info->restarts = std::max(info->restarts, r.cycles[i]);
        info->converged += r.converged[i];
        info->relres_true = std::max(info->relres_true, r.relres[i]);
        info->relres_est = std::max(info->relres_est, r.est[i]);
    }
    info->outer_iters = outer;
    info->t_total_s = t;
}

static om_status run_gmres(const om_csr* Ac, const om_ilu* M, int adjoint, const double2* b, double2* x,
                           const om_gmres_opts* o, om_gmres_info* info, std::vector<double>* relres, hipStream_t s) {
    om_csr* A = const_cast<om_csr*>(Ac);
    OM_TRY(check_gmres_opts(o));
    if (M && (M->host_only || M->n != A->n || M->batch != A->batch)) {
        set_error("preconditioner does not match the matrix (size, batch or host-only handle)");
        return OM_EINVAL;
    }
    if (adjoint) {
        if (M && !(M->flags & OM_ILU_ADJOINT)) { set_error("adjoint solve needs factors built with OM_ILU_ADJOINT"); return OM_EINVAL; }
        OM_TRY(ensure_transpose(A, s));
    }
    const auto t0 = std::chrono::steady_clock::now();
    CoreResult r;
    int outer = 0;
    if (o->precision == OM_PREC_IR_C64) {
        if (M && !(M->flags & OM_ILU_C64)) { set_error("GMRES-IR needs factors built with OM_ILU_C64"); return OM_EINVAL; }
        OM_TRY(make_c64(A, s));
        if (adjoint) OM_TRY(ensure_transpose(A, s));
        OM_TRY(gmres_ir(A, M, adjoint, b, x, *o, r, outer, s));
    } else {
        OM_TRY(gmres_core<double2>(A, M, adjoint, b, x, o->m, o->tol, o->maxiter, nullptr, r, s));
    }
    OM_HIP(hipStreamSynchronize(s));
    fill_gmres_info(r, outer, secs_since(t0), info);
    if (relres) *relres = r.relres;
    for (size_t i = 0; i < r.converged.size(); ++i)
        if (!r.converged[i]) {
            set_error("GMRES did not reach tol %g for item %zu (relres %g after %d steps)", o->tol, i, r.relres[i], r.iters[i]);
            return OM_ENOTCONV;
        }
    return OM_OK;
}

}  // namespace omss

using namespace omss;

extern "C" {

const char* om_last_error(void) { return omss::last_error(); }
const char* om_version(void) { return "omss 0.1 (gfx950)"; }

om_status liouvillian_build(const om_params* params, int32_t batch, int32_t trace_mode, uint32_t flags,
                            om_csr** A_out, double* w_out, void* stream) {
    return guarded([&]() -> om_status {
        if (!A_out) { set_error("A_out is null"); return OM_EINVAL; }
        *A_out = nullptr;
        std::unique_ptr<om_csr> A(new om_csr);
        OM_TRY(assemble(params, batch, trace_mode, flags, A.get(), w_out, as_stream(stream)));
        *A_out = A.release();
        return OM_OK;
    });
}

om_status om_csr_info(const om_csr* A, int64_t* n, int64_t* nnz, int32_t* batch, int32_t* N) {
    if (!A) { set_error("null handle"); return OM_EINVAL; }
    if (n) *n = A->n;
    if (nnz) *nnz = A->nnz;
    if (batch) *batch = A->batch;
    if (N) *N = A->N;
    return OM_OK;
}

om_status om_csr_export(const om_csr* A, int64_t* row_ptr, int32_t* col, double* val, void* stream) {
    return guarded([&]() -> om_status {
        if (!A) { set_error("null handle"); return OM_EINVAL; }
        hipStream_t s = as_stream(stream);
        if (row_ptr) {
            std::vector<int32_t> rp(A->n + 1);
            OM_HIP(hipMemcpyAsync(rp.data(), A->row_ptr.p, rp.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            OM_HIP(hipStreamSynchronize(s));
            for (int64_t i = 0; i <= A->n; ++i) row_ptr[i] = rp[i];
        }
        if (col) OM_HIP(hipMemcpyAsync(col, A->col.p, A->nnz * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        if (val) OM_HIP(hipMemcpyAsync(val, A->val.p, (size_t)A->batch * A->nnz * sizeof(double2), hipMemcpyDeviceToHost, s));
        OM_HIP(hipStreamSynchronize(s));
        return OM_OK;
    });
}

om_status rcm_permute(const om_csr* A, int32_t* perm_host, om_csr** A_perm_out, om_order_stats* st, void* stream) {
    return guarded([&]() -> om_status {
        if (!A || !A_perm_out) { set_error("null argument"); return OM_EINVAL; }
        *A_perm_out = nullptr;
        hipStream_t s = as_stream(stream);
        om_csr* Am = const_cast<om_csr*>(A);
        OM_TRY(ensure_host_pattern(Am, s));
        std::vector<int32_t> perm;
        rcm_order(A->n, Am->h_row_ptr.data(), Am->h_col.data(), perm);
        std::unique_ptr<om_csr> B(new om_csr);
        OM_TRY(permute_csr(A, perm.data(), B.get(), s));
        if (st) {
            BandStats s0 = band_stats(A->n, Am->h_row_ptr.data(), Am->h_col.data());
            BandStats s1 = band_stats(B->n, B->h_row_ptr.data(), B->h_col.data());
            *st = om_order_stats{s0.ub, s0.lb, s0.B, s0.P, s1.ub, s1.lb, s1.B, s1.P};
        }
        if (perm_host) std::memcpy(perm_host, perm.data(), perm.size() * sizeof(int32_t));
        *A_perm_out = B.release();
        return OM_OK;
    });
}

om_status csr_permute(const om_csr* A, const int32_t* perm_host, om_csr** A_perm_out, void* stream) {
    return guarded([&]() -> om_status {
        if (!A || !perm_host || !A_perm_out) { set_error("null argument"); return OM_EINVAL; }
        *A_perm_out = nullptr;
        std::unique_ptr<om_csr> B(new om_csr);
        OM_TRY(permute_csr(A, perm_host, B.get(), as_stream(stream)));
        *A_perm_out = B.release();
        return OM_OK;
    });
}

om_status ilu_factor(const om_csr* A, double drop_tol, double fill_factor, uint32_t flags, om_ilu** M_out,
                     om_ilu_stats* st, void* stream) {
    return guarded([&]() -> om_status {
        if (!A || !M_out) { set_error("null argument"); return OM_EINVAL; }
        *M_out = nullptr;
        return ilu_factor_impl(A, drop_tol, fill_factor, flags, M_out, st, as_stream(stream));
    });
}

om_status om_ilu_info(const om_ilu* M, int32_t b, int64_t* n, int64_t* nnz_L, int64_t* nnz_U) {
    if (!M || b < 0 || b >= M->batch) { set_error("bad handle or item"); return OM_EINVAL; }
    if (n) *n = M->n;
    const HostFactor* F = M->host[M->shared ? 0 : b].get();
    if (nnz_L) *nnz_L = F ? (int64_t)F->l_col.size() : -1;
    if (nnz_U) *nnz_U = F ? (int64_t)F->u_col.size() : -1;
    return OM_OK;
}

om_status om_ilu_export(const om_ilu* M, int32_t b, int64_t* l_ptr, int32_t* l_col, double* l_val, int64_t* u_ptr,
                        int32_t* u_col, double* u_val) {
    if (!M || b < 0 || b >= M->batch) { set_error("bad handle or item"); return OM_EINVAL; }
    const HostFactor* F = M->host[M->shared ? 0 : b].get();
    if (!F) { set_error("factors were not kept on the host (use OM_ILU_KEEP_HOST)"); return OM_EINVAL; }
    if (l_ptr) std::memcpy(l_ptr, F->l_ptr.data(), F->l_ptr.size() * sizeof(int64_t));
    if (l_col) std::memcpy(l_col, F->l_col.data(), F->l_col.size() * sizeof(int32_t));
    if (l_val) std::memcpy(l_val, F->l_val.data(), F->l_val.size() * sizeof(double));
    if (u_ptr) std::memcpy(u_ptr, F->u_ptr.data(), F->u_ptr.size() * sizeof(int64_t));
    if (u_col) std::memcpy(u_col, F->u_col.data(), F->u_col.size() * sizeof(int32_t));
    if (u_val) std::memcpy(u_val, F->u_val.data(), F->u_val.size() * sizeof(double));
    return OM_OK;
}

om_status ilu_apply(const om_ilu* M, int32_t adjoint, int32_t dtype, const void* x, void* y, void* stream) {
    return guarded([&]() -> om_status {
        if (!M || !x || !y) { set_error("null argument"); return OM_EINVAL; }
        if (M->host_only) { set_error("host-only factors cannot be applied on the device"); return OM_EINVAL; }
        if (adjoint && !(M->flags & OM_ILU_ADJOINT)) { set_error("factors were built without OM_ILU_ADJOINT"); return OM_EINVAL; }
        if (dtype == OM_C64 && !(M->flags & OM_ILU_C64)) { set_error("factors were built without OM_ILU_C64"); return OM_EINVAL; }
        if (dtype != OM_C64 && dtype != OM_C128) { set_error("bad dtype"); return OM_EINVAL; }
        OM_TRY(ilu_apply_dev(M, adjoint, dtype, x, y, nullptr, as_stream(stream)));
        return trsv_check(M, as_stream(stream));
    });
}

om_status csr_spmv(const om_csr* A, int32_t adjoint, int32_t dtype, const void* x, void* y, void* stream) {
    return guarded([&]() -> om_status {
        if (!A || !x || !y) { set_error("null argument"); return OM_EINVAL; }
        if (x == y) { set_error("x and y must not alias"); return OM_EINVAL; }
        hipStream_t s = as_stream(stream);
        om_csr* Am = const_cast<om_csr*>(A);
        if (dtype == OM_C64 && !A->val32.p) { set_error("matrix was built without OM_BUILD_C64"); return OM_EINVAL; }
        if (adjoint) OM_TRY(ensure_transpose(Am, s));
        if (dtype == OM_C128) return spmv<double2>(A, adjoint, (const double2*)x, (double2*)y, nullptr, s);
        if (dtype == OM_C64) return spmv<float2>(A, adjoint, (const float2*)x, (float2*)y, nullptr, s);
        set_error("bad dtype");
        return OM_EINVAL;
    });
}

om_status liouvillian_apply(const om_csr* A, int32_t dtype, const void* x, void* y, void* stream) {
    return guarded([&]() -> om_status {
        if (!A || !x || !y) { set_error("null argument"); return OM_EINVAL; }
        if (x == y) { set_error("x and y must not alias"); return OM_EINVAL; }
        hipStream_t s = as_stream(stream);
        if (dtype == OM_C128) return lapply<double2>(A, (const double2*)x, (double2*)y, nullptr, s);
        if (dtype == OM_C64) return lapply<float2>(A, (const float2*)x, (float2*)y, nullptr, s);
        set_error("bad dtype");
        return OM_EINVAL;
    });
}

om_status gmres_solve(const om_csr* A, const om_ilu* M, int32_t adjoint, const void* b, void* x,
                      const om_gmres_opts* opts, om_gmres_info* info, void* stream) {
    return guarded([&]() -> om_status {
        if (!A || !b || !x) { set_error("null argument"); return OM_EINVAL; }
        return run_gmres(A, M, adjoint, (const double2*)b, (double2*)x, opts, info, nullptr, as_stream(stream));
    });
}

void om_ss_opts_default(om_ss_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->drop_tol = 1e-6;
    o->fill_factor = 60.0;
    o->gmres.m = 50;
    o->gmres.maxiter = 1000;
    o->gmres.precision = OM_PREC_FP64;
    o->gmres.max_outer = 20;
    o->gmres.tol = 1e-10;
    o->gmres.inner_tol = 1e-5;
    o->trace_mode = OM_TRACE_REPLACE_ROW0;
    o->nth0_fix = 1;
    o->reorder = 1;
    o->want_adjoint = 0;
}

__global__ void set_rhs_kernel(double2* b, int64_t n, int64_t pos, const double* w, int batch) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < batch) b[(int64_t)i * n + pos] = make_double2(w[i], 0.0);
}

om_status steady_state(const om_params* params, int32_t batch, const om_ss_opts* opts, void* rho, om_ss_info* info,
                       om_ss_results* res, void* stream) {
    return guarded([&]() -> om_status {
        if (!opts || !rho) { set_error("null argument"); return OM_EINVAL; }
        OM_TRY(validate_params(params, batch));
        OM_TRY(check_gmres_opts(&opts->gmres));
        if (opts->trace_mode == OM_TRACE_NONE) { set_error("steady_state needs a trace condition"); return OM_EINVAL; }
        hipStream_t s = as_stream(stream);
        om_ss_info I;
        std::memset(&I, 0, sizeof I);
        std::vector<om_params> P(params, params + batch);
        if (opts->nth0_fix)
            for (auto& p : P)
                if (p.n_th == 0.0) p.n_th = 1e-15;
        const bool ir = opts->gmres.precision == OM_PREC_IR_C64;
        auto t = std::chrono::steady_clock::now();
        om_csr* A0 = nullptr;
        std::vector<double> w(batch);
        OM_TRY(liouvillian_build(P.data(), batch, opts->trace_mode, ir ? OM_BUILD_C64 : 0u, &A0, w.data(), stream));
        std::unique_ptr<om_csr> A(A0);
        OM_HIP(hipStreamSynchronize(s));
        I.t_build_s = secs_since(t);
        t = std::chrono::steady_clock::now();
        if (opts->reorder) {
            om_csr* B = nullptr;
            OM_TRY(rcm_permute(A.get(), nullptr, &B, &I.order, stream));
            A.reset(B);
        }
        I.t_rcm_s = secs_since(t);
        t = std::chrono::steady_clock::now();
        om_ilu* M0 = nullptr;
        uint32_t fl = (ir ? OM_ILU_C64 : 0u) | (opts->want_adjoint ? OM_ILU_ADJOINT : 0u) |
                      (opts->share_factor ? OM_ILU_SHARED : 0u);
        OM_TRY(ilu_factor(A.get(), opts->drop_tol, opts->fill_factor, fl, &M0, &I.ilu, stream));
        std::unique_ptr<om_ilu, void (*)(om_ilu*)> M(M0, om_ilu_free);
        I.t_factor_s = secs_since(t);
        t = std::chrono::steady_clock::now();
        const int64_t n = A->n;
        DevBuf<double2> bvec, x;
        OM_TRY(bvec.alloc((size_t)batch * n));
        OM_TRY(x.alloc((size_t)batch * n));
        OM_HIP(hipMemsetAsync(bvec.p, 0, bvec.bytes(), s));
        OM_HIP(hipMemsetAsync(x.p, 0, x.bytes(), s));
        DevBuf<double> dw;
        OM_TRY(dw.upload(w.data(), batch, s));
        int64_t pos0 = 0;   // position of natural row 0 (the trace row) in the ordering of A
        if (A->permuted)
            for (int64_t i = 0; i < n; ++i)
                if (A->perm[i] == 0) { pos0 = i; break; }
        hipLaunchKernelGGL(set_rhs_kernel, dim3(blocks_for(batch, 64)), dim3(64), 0, s, bvec.p, n, pos0, dw.p, batch);
        OM_HIP(hipGetLastError());
        std::vector<double> relres;
        om_status gs = run_gmres(A.get(), M.get(), 0, bvec.p, x.p, &opts->gmres, &I.gmres, &relres, s);
        if (gs != OM_OK && gs != OM_ENOTCONV) return gs;
        std::string gerr = gs == OM_ENOTCONV ? last_error() : "";
        I.t_solve_s = secs_since(t);
        t = std::chrono::steady_clock::now();
        DevBuf<double> obs, tr;
        OM_TRY(obs.alloc((size_t)batch * 3));
        OM_TRY(tr.alloc((size_t)batch * 2));
        OM_TRY(observables(A.get(), x.p, obs.p, tr.p, s));
        std::vector<double> herm(batch);
        OM_TRY(unvec(A.get(), x.p, tr.p, (double2*)rho, herm.data(), s));
        std::vector<double> ho((size_t)batch * 3), ht((size_t)batch * 2);
        OM_HIP(hipMemcpyAsync(ho.data(), obs.p, ho.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        OM_HIP(hipMemcpyAsync(ht.data(), tr.p, ht.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        OM_HIP(hipStreamSynchronize(s));
        I.t_post_s = secs_since(t);
        if (res) {
            for (int b = 0; b < batch; ++b) {
                if (res->trace_err) res->trace_err[b] = std::hypot(ht[2 * b] - 1.0, ht[2 * b + 1]);
                if (res->herm_err) res->herm_err[b] = herm[b];
                if (res->n_a) res->n_a[b] = ho[3 * b];
                if (res->n_b) res->n_b[b] = ho[3 * b + 1];
                if (res->fano) res->fano[b] = ho[3 * b + 2];
                if (res->relres) res->relres[b] = b < (int)relres.size() ? relres[b] : 0.0;
            }
        }
        if (info) *info = I;
        if (gs == OM_ENOTCONV) { set_error("%s", gerr.c_str()); return OM_ENOTCONV; }
        return OM_OK;
    });
}

om_status om_observables(const om_csr* A, const void* x, double* obs_host, void* stream) {
    return guarded([&]() -> om_status {
        if (!A || !x || !obs_host) { set_error("null argument"); return OM_EINVAL; }
        hipStream_t s = as_stream(stream);
        DevBuf<double> obs;
        OM_TRY(obs.alloc((size_t)A->batch * 3));
        OM_TRY(observables(A, (const double2*)x, obs.p, nullptr, s));
        OM_HIP(hipMemcpyAsync(obs_host, obs.p, (size_t)A->batch * 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        OM_HIP(hipStreamSynchronize(s));
        return OM_OK;
    });
}

om_status om_objective_vectors(const om_csr* A, const void* x, void* g, void* stream) {
    return guarded([&]() -> om_status {
        if (!A || !x || !g) { set_error("null argument"); return OM_EINVAL; }
        if (!A->has_model) { set_error("matrix carries no model description"); return OM_EINVAL; }
        return objective_vectors(A, (const double2*)x, (double2*)g, as_stream(stream));
    });
}

om_status om_param_gradient(const om_csr* A, const void* x, const void* lambda, int32_t nrhs, double* grad_host,
                            void* stream) {
    return guarded([&]() -> om_status {
        if (!A || !x || !lambda || !grad_host) { set_error("null argument"); return OM_EINVAL; }
        return param_gradient(A, (const double2*)x, (const double2*)lambda, nrhs, grad_host, as_stream(stream));
    });
}

void om_csr_free(om_csr* A) { delete A; }
void om_ilu_free(om_ilu* M) { delete M; }

om_status om_host_rcm(int64_t n, const int64_t* row_ptr, const int32_t* col, int32_t* perm) {
    return guarded([&]() -> om_status {
        if (n < 1 || !row_ptr || !col || !perm) { set_error("invalid argument"); return OM_EINVAL; }
        for (int64_t t = 0; t < row_ptr[n]; ++t)
            if (col[t] < 0 || col[t] >= n) { set_error("column index out of range"); return OM_EINVAL; }
        std::vector<int32_t> p;
        rcm_order(n, row_ptr, col, p);
        std::memcpy(perm, p.data(), n * sizeof(int32_t));
        return OM_OK;
    });
}

om_status om_host_ilut(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val, double drop_tol,
                       double fill_factor, om_ilu** M_out, om_ilu_stats* st) {
    return guarded([&]() -> om_status {
        if (!M_out) { set_error("M_out is null"); return OM_EINVAL; }
        *M_out = nullptr;
        return host_ilut_impl(n, row_ptr, col, val, drop_tol, fill_factor, M_out, st);
    });
}

}  // extern "C"
