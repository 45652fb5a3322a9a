// GMRES drivers (internal).
#pragma once
#include <vector>

#include "common.hpp"

namespace omss {

struct CoreResult {
    std::vector<int32_t> iters, cycles, converged;
    std::vector<double> relres, est;
};

template <typename VT>
om_status gmres_core(const om_csr* A, const om_ilu* M, int adjoint, const VT* b, VT* x, int m, double tol,
                     int maxiter, const std::vector<int32_t>* item_mask, CoreResult& res, hipStream_t s);

om_status gmres_ir(const om_csr* A, const om_ilu* M, int adjoint, const double2* b, double2* x, const om_gmres_opts& o,
                   CoreResult& res, int& outer, hipStream_t s);

}  // namespace omss
