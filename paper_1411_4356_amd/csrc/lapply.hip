// Matrix-free product with the trace-constrained Liouvillian.
//
// y = A x where A is the matrix liouvillian_build assembles (Eq. (3) in the
// Fock basis with column-stacked rho, Eq. (4); row 0 carrying the trace
// condition of Eq. (5)), possibly symmetrically permuted, without reading
// any stored entry: every row evaluates its at most 16 stencil entries from
// the model parameters and gathers the matching unknowns.  Only x and y (and
// the permutation, if any) cross HBM -- 2s bytes per row instead of the
// 20 bytes per stored entry plus 2s per row of the CSR product (s = bytes of
// a complex value).  The values are the ones the build stores, so the result
// equals the CSR product up to the order of the additions.
#include "common.hpp"
#include "cplx.hpp"
#include "kernels.hpp"
#include "profile.hpp"
#include "stencil.hpp"

namespace omss {

namespace {

constexpr int LT = 256;

// the slots of the quadratic coupling g2 (b + b^dag)^2 a^dag a (stencil.hpp)
__host__ __device__ constexpr bool is_quadratic_slot(int sl) { return sl == 1 || sl == 5 || sl == 9 || sl == 13; }

// Rows of A other than the trace row.  Row i of A is model row perm[i]; the
// unknown of model column q is x[iperm[q]].  The row is decoded once (32-bit:
// n < 2^31), its candidate entries are evaluated into registers, and
// the index and value gathers of all of them are issued before any is used
// (a slot outside the truncated space gathers the row's own unknown and adds
// nothing), so a row waits for two rounds of loads rather than one per entry.
// QUAD = false: no item has a quadratic coupling, and its four slots (whose
// values would all be zero) are left out at compile time.
template <typename VT, bool PERM, bool QUAD>
__global__ __launch_bounds__(LT) void lapply_kernel(Dims d, const DevParams* __restrict__ P,
                                                    const int32_t* __restrict__ perm,
                                                    const int32_t* __restrict__ iperm, const VT* __restrict__ x,
                                                    VT* __restrict__ y, const int32_t* __restrict__ active,
                                                    int skip_row0) {
    using ST = typename Scalar<VT>::type;
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const int64_t i = (int64_t)blockIdx.x * LT + threadIdx.x;
    if (i >= d.n) return;
    const uint32_t p = PERM ? (uint32_t)perm[i] : (uint32_t)i;
    if (skip_row0 && p == 0) return;
    const uint32_t N = (uint32_t)d.N, nm = (uint32_t)d.nm;
    const uint32_t l = p / N, k = p - l * N;
    const int ik = (int)(k / nm), jk = (int)(k - (uint32_t)ik * nm);
    const int il = (int)(l / nm), jl = (int)(l - (uint32_t)il * nm);
    const DevParams Pb = P[b];
    const VT* xb = x + (int64_t)b * d.n;
    bool ok[NSLOT];
    int64_t q[NSLOT];
    double2 v[NSLOT];
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl) {
        ok[sl] = (QUAD || !is_quadratic_slot(sl)) && stencil_entry_at(sl, (int64_t)p, ik, jk, il, jl, d, Pb, q[sl], v[sl]);
        if (!ok[sl]) q[sl] = p;
    }
    int64_t j[NSLOT];
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl)
        if (QUAD || !is_quadratic_slot(sl)) j[sl] = PERM ? (int64_t)iperm[q[sl]] : q[sl];
    VT xv[NSLOT];
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl)
        if (QUAD || !is_quadratic_slot(sl)) xv[sl] = xb[j[sl]];
    ST ar = 0, ai = 0;
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl) {
        if (!ok[sl]) continue;
        const ST vr = (ST)v[sl].x, vi = (ST)v[sl].y;
        ar += vr * xv[sl].x - vi * xv[sl].y;
        ai += vr * xv[sl].y + vi * xv[sl].x;
    }
    VT r;
    r.x = ar;
    r.y = ai;
    y[(int64_t)b * d.n + i] = r;
}

// The trace row (model row 0), one block per item: w * sum_k x(k(N+1)), plus
// the model row itself when the condition is added (Eq. (5)) rather than
// substituted.
template <typename VT>
__global__ __launch_bounds__(LT) void lapply_trace_kernel(Dims d, const DevParams* __restrict__ P,
                                                          const double* __restrict__ w,
                                                          const int32_t* __restrict__ iperm,
                                                          const VT* __restrict__ x, VT* __restrict__ y,
                                                          const int32_t* __restrict__ active, int add_model_row) {
    using ST = typename Scalar<VT>::type;
    const int b = blockIdx.x;
    if (active && !active[b]) return;
    const VT* xb = x + (int64_t)b * d.n;
    ST sr = 0, si = 0;
    for (int64_t k = threadIdx.x; k < d.N; k += LT) {
        const int64_t q = k * (d.N + 1);
        const VT xv = xb[iperm ? (int64_t)iperm[q] : q];
        sr += xv.x;
        si += xv.y;
    }
    __shared__ ST red[2][LT / 64];
    for (int off = 32; off > 0; off >>= 1) {
        sr += __shfl_down(sr, off, 64);
        si += __shfl_down(si, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = sr;
        red[1][threadIdx.x >> 6] = si;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    ST tr = 0, ti = 0;
    for (int q = 0; q < LT / 64; ++q) {
        tr += red[0][q];
        ti += red[1][q];
    }
    const ST wb = (ST)w[b];
    ST ar = wb * tr, ai = wb * ti;
    if (add_model_row) {
        const DevParams Pb = P[b];
        for (int sl = 0; sl < NSLOT; ++sl) {
            int64_t q;
            double2 v;
            if (!stencil_entry(sl, 0, d, Pb, q, v)) continue;
            const VT xv = xb[iperm ? (int64_t)iperm[q] : q];
            const ST vr = (ST)v.x, vi = (ST)v.y;
            ar += vr * xv.x - vi * xv.y;
            ai += vr * xv.y + vi * xv.x;
        }
    }
    VT r;
    r.x = ar;
    r.y = ai;
    y[(int64_t)b * d.n + (iperm ? (int64_t)iperm[0] : 0)] = r;
}

}  // namespace

double lapply_bytes(const om_csr* A, size_t s, const int32_t* act_host) {
    int na = A->batch;
    if (act_host) {
        na = 0;
        for (int i = 0; i < A->batch; ++i) na += act_host[i] != 0;
    }
    // x read and y written once per item; the permutation (both directions) once
    return na * 2.0 * (double)A->n * (double)s + (A->permuted ? 8.0 * (double)A->n : 0.0);
}

template <typename VT>
om_status lapply(const om_csr* A, const VT* x, VT* y, const int32_t* active, hipStream_t s, const int32_t* act_host) {
    if (!A->has_model) { set_error("matrix-free product: the matrix carries no model description"); return OM_EINVAL; }
    if (A->permuted && (!A->perm_d.p || !A->iperm_d.p)) { set_error("matrix-free product: permutation missing"); return OM_EINVAL; }
    const om_params& p0 = A->params[0];
    const Dims d{p0.nc, p0.nm, p0.nc * p0.nm, A->n};
    om_csr* Am = const_cast<om_csr*>(A);
    // per-item parameters and weights, uploaded once per handle
    static_assert(sizeof(DevParams) == 8 * sizeof(double), "parameter record");
    if (!Am->lapply_params.p) {
        std::vector<double> hp;
        for (int b = 0; b < A->batch; ++b) {
            const om_params& q = A->params[b];
            for (double v : {q.delta, q.omega_m, q.g0, q.E, q.kappa, q.gamma_m, q.n_th, q.g2}) hp.push_back(v);
        }
        OM_TRY(Am->lapply_params.upload(hp.data(), hp.size(), s));
        OM_TRY(Am->lapply_w.upload(A->w.data(), A->w.size(), s));
        OM_HIP(hipStreamSynchronize(s));   // the host vectors go out of scope
    }
    const int32_t* perm = A->permuted ? A->perm_d.p : nullptr;
    const int32_t* iperm = A->permuted ? A->iperm_d.p : nullptr;
    const bool trace = A->trace_mode != OM_TRACE_NONE;
    ProfScope prof("lapply", s, profile_enabled() ? lapply_bytes(A, sizeof(VT), act_host) : 0.0);
    bool quad = false;
    for (const om_params& q : A->params) quad = quad || q.g2 != 0.0;
    const dim3 grid(blocks_for(A->n, LT), A->batch);
    const DevParams* dp = reinterpret_cast<const DevParams*>(Am->lapply_params.p);
    const int skip0 = trace ? 1 : 0;
    if (perm && quad)
        hipLaunchKernelGGL((lapply_kernel<VT, true, true>), grid, dim3(LT), 0, s, d, dp, perm, iperm, x, y, active, skip0);
    else if (perm)
        hipLaunchKernelGGL((lapply_kernel<VT, true, false>), grid, dim3(LT), 0, s, d, dp, perm, iperm, x, y, active, skip0);
    else if (quad)
        hipLaunchKernelGGL((lapply_kernel<VT, false, true>), grid, dim3(LT), 0, s, d, dp, perm, iperm, x, y, active, skip0);
    else
        hipLaunchKernelGGL((lapply_kernel<VT, false, false>), grid, dim3(LT), 0, s, d, dp, perm, iperm, x, y, active, skip0);
    OM_HIP(hipGetLastError());
    if (trace) {
        hipLaunchKernelGGL((lapply_trace_kernel<VT>), dim3(A->batch), dim3(LT), 0, s, d,
                           reinterpret_cast<const DevParams*>(Am->lapply_params.p),
                           Am->lapply_w.p, iperm, x, y, active, A->trace_mode == OM_TRACE_ADD_ROW0 ? 1 : 0);
        OM_HIP(hipGetLastError());
    }
    return OM_OK;
}
template om_status lapply<double2>(const om_csr*, const double2*, double2*, const int32_t*, hipStream_t,
                                   const int32_t*);
template om_status lapply<float2>(const om_csr*, const float2*, float2*, const int32_t*, hipStream_t, const int32_t*);

}  // namespace omss
