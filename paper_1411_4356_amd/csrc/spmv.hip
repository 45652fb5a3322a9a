// Complex CSR sparse matrix-vector products.
//
// A group of G consecutive lanes (G = 8 for the ~11 nonzeros per row of the
// Liouvillian) owns one row: the lanes stride over the row's entries, so the
// column and value loads of a wavefront are contiguous runs, and the partial
// sums are combined with cross-lane shuffles.  Batch items (blockIdx.y) share
// the column indices and row pointers; each has its own values.  The same
// kernel applies A^H through the stored conjugate transpose.
#include <cstdlib>
#include <cstring>

#include "common.hpp"
#include "cplx.hpp"
#include "kernels.hpp"
#include "profile.hpp"

namespace omss {

template <typename ST>
__device__ inline ST group_sum(ST v, int G) {
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_down(v, off, G);
    return v;
}

template <typename VT, int G>
__global__ __launch_bounds__(256) void spmv_kernel(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                                   const VT* __restrict__ val, int64_t nnz, const VT* __restrict__ x,
                                                   VT* __restrict__ y, int64_t n, const int32_t* __restrict__ active) {
    using ST = typename Scalar<VT>::type;
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int sub = threadIdx.x % G;
    const VT* vb = val + (int64_t)b * nnz;
    const VT* xb = x + (int64_t)b * n;
    ST ar = 0, ai = 0;
    if (row < n) {
        const int32_t t0 = row_ptr[row], t1 = row_ptr[row + 1];
        for (int32_t t = t0 + sub; t < t1; t += G) {
            const VT a = vb[t];
            const VT xv = xb[col[t]];
            ar += a.x * xv.x - a.y * xv.y;
            ai += a.x * xv.y + a.y * xv.x;
        }
    }
    ar = group_sum(ar, G);
    ai = group_sum(ai, G);
    if (row < n && sub == 0) {
        VT r;
        r.x = ar;
        r.y = ai;
        y[(int64_t)b * n + row] = r;
    }
}

double spmv_bytes(const om_csr* A, size_t s, const int32_t* act_host) {
    int na = A->batch;
    if (act_host) {
        na = 0;
        for (int i = 0; i < A->batch; ++i) na += act_host[i] != 0;
    }
    return na * ((double)A->nnz * (double)(s + 4) + 4.0 * (double)(A->n + 1) + 2.0 * (double)A->n * (double)s);
}

// OMSS_SPMV=stencil: products with a model matrix (not its adjoint) are
// evaluated matrix-free (lapply.hip)
static bool stencil_products() {
    const char* e = std::getenv("OMSS_SPMV");
    return e && std::strcmp(e, "stencil") == 0;
}

template <typename VT>
om_status spmv(const om_csr* A, int adjoint, const VT* x, VT* y, const int32_t* active, hipStream_t s,
               const int32_t* act_host) {
    if (!adjoint && A->has_model && stencil_products()) return lapply<VT>(A, x, y, active, s, act_host);
    constexpr int G = 8;
    const int TPB = 256;
    const int32_t* rp = adjoint ? A->t_row_ptr.p : A->row_ptr.p;
    const int32_t* cl = adjoint ? A->t_col.p : A->col.p;
    const void* v;
    if (sizeof(VT) == sizeof(double2)) v = adjoint ? (const void*)A->t_val.p : (const void*)A->val.p;
    else v = adjoint ? (const void*)A->t_val32.p : (const void*)A->val32.p;
    if (!rp || !cl || !v) { set_error("spmv: matrix storage for this product was not built"); return OM_EINVAL; }
    dim3 grid(blocks_for(A->n * G, TPB), A->batch);
    ProfScope prof("spmv", s, profile_enabled() ? spmv_bytes(A, sizeof(VT), act_host) : 0.0);
    hipLaunchKernelGGL((spmv_kernel<VT, G>), grid, dim3(TPB), 0, s, rp, cl, (const VT*)v, A->nnz, x, y, A->n, active);
    OM_HIP(hipGetLastError());
    return OM_OK;
}
template om_status spmv<double2>(const om_csr*, int, const double2*, double2*, const int32_t*, hipStream_t,
                                 const int32_t*);
template om_status spmv<float2>(const om_csr*, int, const float2*, float2*, const int32_t*, hipStream_t,
                                const int32_t*);

// r = b - A x with the squared norm of r accumulated per block:
// norm2[b * gridDim.x + blockIdx.x] (always in double precision).
template <typename VT, int G>
__global__ __launch_bounds__(256) void residual_kernel(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                                       const VT* __restrict__ val, int64_t nnz,
                                                       const VT* __restrict__ bvec, const VT* __restrict__ x,
                                                       VT* __restrict__ r, double* __restrict__ norm2, int64_t n,
                                                       const int32_t* __restrict__ active) {
    using ST = typename Scalar<VT>::type;
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int sub = threadIdx.x % G;
    const VT* vb = val + (int64_t)b * nnz;
    const VT* xb = x + (int64_t)b * n;
    ST ar = 0, ai = 0;
    if (row < n) {
        const int32_t t0 = row_ptr[row], t1 = row_ptr[row + 1];
        for (int32_t t = t0 + sub; t < t1; t += G) {
            const VT a = vb[t];
            const VT xv = xb[col[t]];
            ar += a.x * xv.x - a.y * xv.y;
            ai += a.x * xv.y + a.y * xv.x;
        }
    }
    ar = group_sum(ar, G);
    ai = group_sum(ai, G);
    double sq = 0.0;
    if (row < n && sub == 0) {
        const VT bb = bvec[(int64_t)b * n + row];
        VT rr;
        rr.x = bb.x - ar;
        rr.y = bb.y - ai;
        r[(int64_t)b * n + row] = rr;
        sq = (double)rr.x * (double)rr.x + (double)rr.y * (double)rr.y;
    }
    __shared__ double red[256 / 64];
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_down(sq, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int w = 0; w < 256 / 64; ++w) t += red[w];
        norm2[(int64_t)b * gridDim.x + blockIdx.x] = t;
    }
}

template <typename VT>
om_status residual(const om_csr* A, int adjoint, const VT* b, const VT* x, VT* r, double* norm2, int* nparts,
                   const int32_t* active, hipStream_t s, const int32_t* act_host) {
    constexpr int G = 8;
    const int TPB = 256;
    const int32_t* rp = adjoint ? A->t_row_ptr.p : A->row_ptr.p;
    const int32_t* cl = adjoint ? A->t_col.p : A->col.p;
    const void* v;
    if (sizeof(VT) == sizeof(double2)) v = adjoint ? (const void*)A->t_val.p : (const void*)A->val.p;
    else v = adjoint ? (const void*)A->t_val32.p : (const void*)A->val32.p;
    if (!rp || !cl || !v) { set_error("residual: matrix storage for this product was not built"); return OM_EINVAL; }
    dim3 grid(blocks_for(A->n * G, TPB), A->batch);
    if (nparts) *nparts = (int)grid.x;
    if (!b) return OM_OK;
    ProfScope prof("spmv", s, profile_enabled() ? spmv_bytes(A, sizeof(VT), act_host) + A->batch * (double)A->n * sizeof(VT) : 0.0);
    hipLaunchKernelGGL((residual_kernel<VT, G>), grid, dim3(TPB), 0, s, rp, cl, (const VT*)v, A->nnz, b, x, r, norm2,
                       A->n, active);
    OM_HIP(hipGetLastError());
    return OM_OK;
}
template om_status residual<double2>(const om_csr*, int, const double2*, const double2*, double2*, double*, int*,
                                     const int32_t*, hipStream_t, const int32_t*);
template om_status residual<float2>(const om_csr*, int, const float2*, const float2*, float2*, double*, int*,
                                    const int32_t*, hipStream_t, const int32_t*);

}  // namespace omss
