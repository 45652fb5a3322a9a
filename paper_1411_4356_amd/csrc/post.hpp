// Post-processing and gradient helpers (internal).
#pragma once
#include "common.hpp"

namespace omss {

om_status observables(const om_csr* A, const double2* x, double* obs_dev, double* trace_dev, hipStream_t s);
om_status unvec(const om_csr* A, const double2* x, const double* trace_dev, double2* rho, double* herm_err_host,
                hipStream_t s);
om_status objective_vectors(const om_csr* A, const double2* x, double2* g, hipStream_t s);
om_status param_gradient(const om_csr* A, const double2* x, const double2* lam, int nrhs, double* grad_host,
                         hipStream_t s);

}  // namespace omss
