// CSR handle operations: host copy of the pattern, symmetric permutation
// P A P^T (pattern on the host, values gathered on the device) and the
// conjugate transpose used for A^H products.
#include <vector>

#include "common.hpp"
#include "cplx.hpp"
#include "kernels.hpp"
#include "ordering.hpp"

namespace omss {

__global__ void gather_values_kernel(const double2* __restrict__ src_val, int64_t src_nnz, const int32_t* __restrict__ src,
                                     double2* __restrict__ dst, int64_t nnz, int conj) {
    const int b = blockIdx.y;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nnz) return;
    double2 v = src_val[(int64_t)b * src_nnz + src[t]];
    if (conj) v.y = -v.y;
    dst[(int64_t)b * nnz + t] = v;
}

__global__ void to_c64_values_kernel(const double2* __restrict__ in, float2* __restrict__ out, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

om_status ensure_host_pattern(om_csr* A, hipStream_t s) {
    if ((int64_t)A->h_row_ptr.size() == A->n + 1) return OM_OK;
    std::vector<int32_t> rp(A->n + 1);
    A->h_col.resize(A->nnz);
    OM_HIP(hipMemcpyAsync(rp.data(), A->row_ptr.p, (A->n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    OM_HIP(hipMemcpyAsync(A->h_col.data(), A->col.p, A->nnz * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    OM_HIP(hipStreamSynchronize(s));
    A->h_row_ptr.assign(rp.begin(), rp.end());
    return OM_OK;
}

om_status permute_csr(const om_csr* Ain, const int32_t* perm, om_csr* B, hipStream_t s) {
    om_csr* A = const_cast<om_csr*>(Ain);
    OM_TRY(ensure_host_pattern(A, s));
    const int64_t n = A->n;
    std::vector<char> seen(n, 0);
    for (int64_t i = 0; i < n; ++i) {
        if (perm[i] < 0 || perm[i] >= n || seen[perm[i]]) { set_error("perm is not a permutation of 0..n-1"); return OM_EINVAL; }
        seen[perm[i]] = 1;
    }
    std::vector<int64_t> nptr;
    std::vector<int32_t> ncol, src;
    permute_pattern(n, A->h_row_ptr.data(), A->h_col.data(), perm, nptr, ncol, src);
    B->n = n;
    B->nnz = A->nnz;
    B->batch = A->batch;
    B->N = A->N;
    std::vector<int32_t> p32(nptr.begin(), nptr.end());
    OM_TRY(B->row_ptr.upload(p32.data(), n + 1, s));
    OM_TRY(B->col.upload(ncol.data(), ncol.size(), s));
    DevBuf<int32_t> dsrc;
    OM_TRY(dsrc.upload(src.data(), src.size(), s));
    OM_TRY(B->val.alloc((size_t)B->batch * B->nnz));
    dim3 grid(blocks_for(B->nnz, 256), B->batch);
    hipLaunchKernelGGL(gather_values_kernel, grid, dim3(256), 0, s, A->val.p, A->nnz, dsrc.p, B->val.p, B->nnz, 0);
    OM_HIP(hipGetLastError());
    if (A->val32.p) {
        OM_TRY(B->val32.alloc((size_t)B->batch * B->nnz));
        hipLaunchKernelGGL(to_c64_values_kernel, dim3(blocks_for((int64_t)B->batch * B->nnz, 256)), dim3(256), 0, s,
                           B->val.p, B->val32.p, (int64_t)B->batch * B->nnz);
    }
    B->h_row_ptr = nptr;
    B->h_col = ncol;
    B->has_model = A->has_model;
    B->params = A->params;
    B->trace_mode = A->trace_mode;
    B->w = A->w;
    B->permuted = true;
    B->perm.resize(n);
    for (int64_t i = 0; i < n; ++i) B->perm[i] = A->permuted ? A->perm[perm[i]] : perm[i];
    std::vector<int32_t> iperm(n);
    for (int64_t i = 0; i < n; ++i) iperm[B->perm[i]] = (int32_t)i;
    OM_TRY(B->perm_d.upload(B->perm.data(), n, s));
    OM_TRY(B->iperm_d.upload(iperm.data(), n, s));
    OM_HIP(hipStreamSynchronize(s));
    return OM_OK;
}

om_status ensure_transpose(om_csr* A, hipStream_t s) {
    if (A->has_t && (!A->val32.p || A->t_val32.p)) return OM_OK;
    if (!A->has_t) {
        OM_TRY(ensure_host_pattern(A, s));
        std::vector<int64_t> tptr, src64;
        std::vector<int32_t> tcol;
        transpose_pattern(A->n, A->h_row_ptr.data(), A->h_col.data(), tptr, tcol, src64);
        std::vector<int32_t> p32(tptr.begin(), tptr.end()), src(src64.begin(), src64.end());
        OM_TRY(A->t_row_ptr.upload(p32.data(), p32.size(), s));
        OM_TRY(A->t_col.upload(tcol.data(), tcol.size(), s));
        OM_TRY(A->t_src.upload(src.data(), src.size(), s));
        OM_TRY(A->t_val.alloc((size_t)A->batch * A->nnz));
        dim3 grid(blocks_for(A->nnz, 256), A->batch);
        hipLaunchKernelGGL(gather_values_kernel, grid, dim3(256), 0, s, A->val.p, A->nnz, A->t_src.p, A->t_val.p, A->nnz, 1);
        OM_HIP(hipGetLastError());
        OM_HIP(hipStreamSynchronize(s));
        A->has_t = true;
    }
    if (A->val32.p && !A->t_val32.p) {
        OM_TRY(A->t_val32.alloc((size_t)A->batch * A->nnz));
        hipLaunchKernelGGL(to_c64_values_kernel, dim3(blocks_for((int64_t)A->batch * A->nnz, 256)), dim3(256), 0, s,
                           A->t_val.p, A->t_val32.p, (int64_t)A->batch * A->nnz);
        OM_HIP(hipGetLastError());
    }
    return OM_OK;
}

}  // namespace omss
