// ILU factor drivers (internal).
#pragma once
#include "common.hpp"

namespace omss {
om_status ilu_factor_impl(const om_csr* A, double drop_tol, double fill_factor, uint32_t flags, om_ilu** M_out,
                          om_ilu_stats* st, hipStream_t s);
om_status host_ilut_impl(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val, double drop_tol,
                         double fill_factor, om_ilu** M_out, om_ilu_stats* st);
}  // namespace omss
