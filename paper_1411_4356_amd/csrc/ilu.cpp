// ilu_factor: ILUT of every batch item (on the device, or on host threads, one
// per item), and the solve schedules of the factors.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cmath>
#include <mutex>
#include <string>
#include <thread>

#include "common.hpp"
#include "ilu.hpp"
#include "ilut.hpp"
#include "kernels.hpp"
#include "ordering.hpp"
#include "schedule.hpp"

namespace omss {

static om_status finish_views(om_ilu* M, hipStream_t s) {
    const int B = M->batch;
    std::vector<TriView<double2>> v64((size_t)B * 4);
    std::vector<TriView<float2>> v32((size_t)B * 4);
    for (int b = 0; b < B; ++b)
        for (int k = 0; k < 4; ++k) {
            const TriSched& S = M->sched[(size_t)(M->shared ? 0 : b) * 4 + k];
            TriView<double2>& a = v64[(size_t)b * 4 + k];
            a.far_off = S.far_off.p; a.mid_off = S.mid_off.p; a.near_off = S.near_off.p; a.far_col = S.far_col.p;
            a.mid_col = S.mid_col.p; a.near_col = S.near_col.p; a.far_need = S.far_need.p; a.far_val = S.far_val.p;
            a.mid_val = S.mid_val.p; a.near_val = S.near_val.p; a.dg = S.dg.p;
            a.dinv = S.dinv.p; a.n = S.n; a.nblk = S.nblk; a.rev = S.rev;
            TriView<float2>& c = v32[(size_t)b * 4 + k];
            c.far_off = S.far_off.p; c.mid_off = S.mid_off.p; c.near_off = S.near_off.p; c.far_col = S.far_col.p;
            c.mid_col = S.mid_col.p; c.near_col = S.near_col.p; c.far_need = S.far_need.p; c.far_val = S.far_val32.p;
            c.mid_val = S.mid_val32.p; c.near_val = S.near_val32.p; c.dg = S.dg32.p;
            c.dinv = S.dinv32.p; c.n = S.n; c.nblk = S.nblk; c.rev = S.rev;
        }
    OM_TRY(M->views64.upload(v64.data(), v64.size(), s));
    OM_TRY(M->views32.upload(v32.data(), v32.size(), s));
    const int64_t nblk = (M->n + 63) / 64;
    OM_TRY(M->scratch.far_buf.alloc((size_t)B * nblk * 64));
    OM_TRY(M->scratch.fdone.alloc((size_t)B * nblk));
    OM_TRY(M->scratch.progress.alloc(B));
    OM_TRY(M->scratch.abort_flag.alloc(1));
    OM_HIP(hipMemsetAsync(M->scratch.fdone.p, 0, M->scratch.fdone.bytes(), s));
    // far sums start unwritten (all bits set; see trsv.hip)
    OM_HIP(hipMemsetAsync(M->scratch.far_buf.p, 0xff, M->scratch.far_buf.bytes(), s));
    OM_HIP(hipMemsetAsync(M->scratch.progress.p, 0, M->scratch.progress.bytes(), s));
    OM_HIP(hipMemsetAsync(M->scratch.abort_flag.p, 0, M->scratch.abort_flag.bytes(), s));
    M->scratch.epoch = 0;
    OM_HIP(hipStreamSynchronize(s));
    return OM_OK;
}

om_status ilu_factor_impl(const om_csr* Ain, double drop_tol, double fill_factor, uint32_t flags, om_ilu** M_out,
                          om_ilu_stats* st, hipStream_t s) {
    if (!(drop_tol >= 0.0) || !(fill_factor > 0.0)) {
        set_error("drop_tol must be >= 0 and fill_factor > 0 (got %g, %g)", drop_tol, fill_factor);
        return OM_EINVAL;
    }
    om_csr* A = const_cast<om_csr*>(Ain);
    const auto t0 = std::chrono::steady_clock::now();
    OM_TRY(ensure_host_pattern(A, s));
    const int64_t n = A->n, nnz = A->nnz;
    const int B = A->batch;
    std::vector<double> vals((size_t)B * nnz * 2);
    OM_HIP(hipMemcpyAsync(vals.data(), A->val.p, vals.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    OM_HIP(hipStreamSynchronize(s));

    std::unique_ptr<om_ilu> M(new om_ilu);
    M->n = n;
    M->batch = B;
    M->flags = flags;
    M->shared = (flags & OM_ILU_SHARED) != 0;
    const int NF = M->shared ? 1 : B;   // factors to compute
    M->sched.resize((size_t)NF * 4);
    M->host.resize(NF);
    int dev = 0;
    OM_HIP(hipGetDevice(&dev));
    const bool adjoint = flags & OM_ILU_ADJOINT;
    const bool verbose = std::getenv("OMSS_VERBOSE") != nullptr;
    const bool c64 = flags & OM_ILU_C64;
    std::vector<om_status> status(NF, OM_OK);
    std::vector<std::string> errs(NF);
    std::vector<int64_t> nl(NF), nu(NF), dl(NF), du(NF), rep(NF);
    // Factorisation: on the device (one item at a time, the whole GPU), or on
    // host threads (items concurrently) with OMSS_ILUT=host or when the band
    // is wider than the device kernel's window.
    const char* ie = std::getenv("OMSS_ILUT");
    bool on_device = !(ie && std::strcmp(ie, "host") == 0);
    // host-side schedule build of the given kinds of a host factor, concurrently
    auto host_schedules = [&](const HostFactor& F, int b, int k0, int k1) -> om_status {
        std::vector<std::thread> kt;
        std::vector<om_status> krc(4, OM_OK);
        std::vector<std::string> kerr(4);
        for (int k = k0; k < k1; ++k)
            kt.emplace_back([&, k] {
                (void)hipSetDevice(dev);
                SolveCSR S;
                factor_to_solve(F, k, S);
                HostTri H;
                build_host_tri(S, H);
                S = SolveCSR();
                if (k == 0) dl[b] = H.depth;
                if (k == 1) du[b] = H.depth;
                krc[k] = upload_tri(H, c64, M->sched[(size_t)b * 4 + k]);
                if (krc[k] != OM_OK) kerr[k] = last_error();
            });
        for (auto& x : kt) x.join();
        for (int k = k0; k < k1; ++k)
            if (krc[k] != OM_OK) { set_error("%s", kerr[k].c_str()); return krc[k]; }
        return OM_OK;
    };
    if (on_device) {
        // the factor stays on the device: L and U schedules are built there;
        // the adjoint solves (transposes) and a kept host copy go through the host
        for (int b = 0; b < NF; ++b) {
            DevFactor D;
            std::string err;
            const om_status rc = ilut_factor_dev(A, b, drop_tol, fill_factor, &D, &err, s);
            if (rc == OM_EBREAKDOWN) { set_error("batch item %d: %s", b, err.c_str()); return rc; }
            if (rc == OM_EINVAL && b == 0) { on_device = false; break; }   // band too wide: host threads
            if (rc != OM_OK) return rc;
            nl[b] = D.nnz_l;
            nu[b] = D.nnz_u;
            rep[b] = D.repaired;
            dl[b] = du[b] = -1;
            if (verbose)
                fprintf(stderr, "[omss] ilu_factor: item %d factored on the device (fill %.1f)\n", b,
                        (double)(nl[b] + nu[b]) / (double)nnz);
            // OMSS_ILU_SCHED=host builds every schedule on the host (a cross-check)
            const char* se = std::getenv("OMSS_ILU_SCHED");
            const bool host_lu = se && std::strcmp(se, "host") == 0;
            if (!host_lu) {
                OM_TRY(build_tri_device(D, 0, c64, M->sched[(size_t)b * 4 + 0], s));
                OM_TRY(build_tri_device(D, 1, c64, M->sched[(size_t)b * 4 + 1], s));
            }
            if (host_lu || adjoint || (flags & OM_ILU_KEEP_HOST)) {
                std::unique_ptr<HostFactor> F(new HostFactor);
                OM_TRY(devfactor_to_host(D, F.get(), s));
                if (host_lu || adjoint) OM_TRY(host_schedules(*F, b, host_lu ? 0 : 2, adjoint ? 4 : 2));
                if (flags & OM_ILU_KEEP_HOST) M->host[b] = std::move(F);
            }
            if (verbose) fprintf(stderr, "[omss] ilu_factor: item %d schedules built\n", b);
        }
    }
    const int HT = host_threads();
    const int T = std::max(1, std::min(NF, HT));
    const int per_item = std::max(1, HT / T);
    auto work = [&](int t) {
        (void)hipSetDevice(dev);
        for (int b = t; b < NF; b += T) {
            std::unique_ptr<HostFactor> F(new HostFactor);
            std::string err;
            const int rc = per_item > 1
                ? ilut_factor_host_mt(n, A->h_row_ptr.data(), A->h_col.data(), vals.data() + (size_t)b * nnz * 2,
                                      drop_tol, fill_factor, per_item, F.get(), &err)
                : ilut_factor_host(n, A->h_row_ptr.data(), A->h_col.data(), vals.data() + (size_t)b * nnz * 2,
                                   drop_tol, fill_factor, 0.0, F.get(), &err);
            if (rc != 0) {
                status[b] = OM_EBREAKDOWN;
                errs[b] = "batch item " + std::to_string(b) + ": " + err;
                continue;
            }
            nl[b] = (int64_t)F->l_col.size();
            nu[b] = (int64_t)F->u_col.size();
            rep[b] = F->repaired;
            if (verbose)
                fprintf(stderr, "[omss] ilu_factor: item %d factored (fill %.1f), building solve schedules\n", b,
                        (double)(nl[b] + nu[b]) / (double)nnz);
            // the solve schedules of the factor are independent: build them concurrently
            const om_status krc = host_schedules(*F, b, 0, adjoint ? 4 : 2);
            if (krc != OM_OK) { status[b] = krc; errs[b] = last_error(); return; }
            if (verbose) fprintf(stderr, "[omss] ilu_factor: item %d schedules uploaded\n", b);
            if (flags & OM_ILU_KEEP_HOST) M->host[b] = std::move(F);
        }
    };
    if (!on_device) {
        std::vector<std::thread> th;
        for (int t = 1; t < T; ++t) th.emplace_back(work, t);
        work(0);
        for (auto& x : th) x.join();
    }
    for (int b = 0; b < NF; ++b)
        if (status[b] != OM_OK) { set_error("%s", errs[b].c_str()); return status[b]; }
    OM_TRY(finish_views(M.get(), s));

    om_ilu_stats S{};
    for (int b = 0; b < NF; ++b) {
        S.fill = std::max(S.fill, (double)(nl[b] + nu[b]) / (double)nnz);
        S.nnz_L += nl[b];
        S.nnz_U += nu[b];
        S.depth_L = std::max(S.depth_L, dl[b]);
        S.depth_U = std::max(S.depth_U, du[b]);
        S.repaired_pivots += rep[b];
    }
    S.t_factor_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (flags & OM_ILU_CONDEST) {
        DevBuf<double2> e;
        OM_TRY(e.alloc((size_t)B * n));
        std::vector<double2> ones((size_t)B * n, make_double2(1.0, 0.0));
        OM_HIP(hipMemcpyAsync(e.p, ones.data(), ones.size() * sizeof(double2), hipMemcpyHostToDevice, s));
        OM_TRY(ilu_apply_dev(M.get(), 0, OM_C128, e.p, e.p, nullptr, s));
        OM_HIP(hipMemcpyAsync(ones.data(), e.p, ones.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
        OM_HIP(hipStreamSynchronize(s));
        // a non-finite entry (an application that overflows) makes the estimate infinite
        double c = 0;
        for (const double2& v : ones) {
            const double a = std::sqrt(v.x * v.x + v.y * v.y);
            c = std::isfinite(a) ? std::max(c, a) : INFINITY;
            if (!std::isfinite(c)) break;
        }
        S.condest = c;
    }
    M->stats = S;
    if (st) *st = S;
    *M_out = M.release();
    return OM_OK;
}

om_status host_ilut_impl(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val, double drop_tol,
                         double fill_factor, om_ilu** M_out, om_ilu_stats* st) {
    if (!(drop_tol >= 0.0) || !(fill_factor > 0.0)) {
        set_error("drop_tol must be >= 0 and fill_factor > 0");
        return OM_EINVAL;
    }
    if (n < 1 || !row_ptr || !col || !val) { set_error("invalid CSR"); return OM_EINVAL; }
    const auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<om_ilu> M(new om_ilu);
    M->n = n;
    M->batch = 1;
    M->host_only = true;
    M->host.resize(1);
    M->host[0].reset(new HostFactor);
    std::string err;
    const int HT = host_threads();
    const int rc = HT > 1 ? ilut_factor_host_mt(n, row_ptr, col, val, drop_tol, fill_factor, HT, M->host[0].get(), &err)
                          : ilut_factor_host(n, row_ptr, col, val, drop_tol, fill_factor, 0.0, M->host[0].get(), &err);
    if (rc != 0) {
        set_error("%s", err.c_str());
        return OM_EBREAKDOWN;
    }
    const HostFactor& F = *M->host[0];
    om_ilu_stats S{};
    S.nnz_L = (int64_t)F.l_col.size();
    S.nnz_U = (int64_t)F.u_col.size();
    S.fill = (double)(S.nnz_L + S.nnz_U) / (double)row_ptr[n];
    S.repaired_pivots = F.repaired;
    S.depth_L = level_depth(n, F.l_ptr, F.l_col);
    SolveCSR T;
    factor_to_solve(F, 1, T);
    S.depth_U = level_depth(n, T.ptr, T.col);
    S.t_factor_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    M->stats = S;
    if (st) *st = S;
    *M_out = M.release();
    return OM_OK;
}

}  // namespace omss
