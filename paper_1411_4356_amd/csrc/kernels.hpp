// Launch wrappers of the device kernels (internal).
#pragma once
#include <string>

#include "common.hpp"

namespace omss {

// assemble.hip
om_status validate_params(const om_params* params, int32_t batch);
om_status assemble(const om_params* params, int32_t batch, int32_t trace_mode, uint32_t flags, om_csr* A,
                   double* w_out, hipStream_t s);
om_status make_c64(om_csr* A, hipStream_t s);
double model_weight(const om_params& p);

// permute / transpose (csr.hip)
om_status ensure_host_pattern(om_csr* A, hipStream_t s);
om_status permute_csr(const om_csr* A, const int32_t* perm, om_csr* B, hipStream_t s);
om_status ensure_transpose(om_csr* A, hipStream_t s);

// spmv.hip: y = A x or A^H x; VT = double2 or float2
template <typename VT>
om_status spmv(const om_csr* A, int adjoint, const VT* x, VT* y, const int32_t* active, hipStream_t s,
               const int32_t* act_host = nullptr);
// r = b - A x and per-item partial |r|^2 into norm2 (*nparts per item); with
// b == nullptr only *nparts is returned.
template <typename VT>
om_status residual(const om_csr* A, int adjoint, const VT* b, const VT* x, VT* r, double* norm2, int* nparts,
                   const int32_t* active, hipStream_t s, const int32_t* act_host = nullptr);
double spmv_bytes(const om_csr* A, size_t s, const int32_t* act_host);

// lapply.hip: y = A x from the model's stencil (A built by liouvillian_build,
// possibly permuted); no stored entry is read
template <typename VT>
om_status lapply(const om_csr* A, const VT* x, VT* y, const int32_t* active, hipStream_t s,
                 const int32_t* act_host = nullptr);
double lapply_bytes(const om_csr* A, size_t s, const int32_t* act_host);


// trsv.hip
// act_host (nullable): host copy of the active mask, used for byte accounting
om_status ilu_apply_dev(const om_ilu* M, int adjoint, int dtype, const void* x, void* y, const int32_t* active,
                        hipStream_t s, const int32_t* act_host = nullptr);
om_status trsv_check(const om_ilu* M, hipStream_t s);

}  // namespace omss
