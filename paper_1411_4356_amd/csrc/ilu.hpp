// ILU factor drivers (internal).
#pragma once
#include <string>

#include "common.hpp"

namespace omss {

struct HostFactor;

// An ILU factor held on the device, row by row with capacity offsets:
// row i of L at l_col/l_val[l_off[i] ..] (l_len[i] entries, strictly lower,
// columns increasing), row i of U at u_off[i] (pivot first, then u_len[i]-1
// entries right of it, columns increasing).
struct DevFactor {
    int64_t n = 0, nnz_l = 0, nnz_u = 0, repaired = 0;
    int64_t upd_entries = 0;   // U-row entries read by the eliminations
    DevBuf<int64_t> l_off, u_off;
    DevBuf<int32_t> l_len, u_len, l_col, u_col;
    DevBuf<double2> l_val, u_val;
};

// schedule_dev.hip: the L (kind 0) or U (kind 1) solve schedule of a device factor
om_status build_tri_device(const DevFactor& D, int kind, bool c64, TriSched& S, hipStream_t s);
// ilut_gpu.hip: device ILUT of batch item `item` of A into D; copy of D to the host
om_status ilut_factor_dev(const om_csr* A, int item, double drop_tol, double fill_factor, DevFactor* D,
                          std::string* err, hipStream_t s);
om_status devfactor_to_host(const DevFactor& D, HostFactor* F, hipStream_t s);

om_status ilu_factor_impl(const om_csr* A, double drop_tol, double fill_factor, uint32_t flags, om_ilu** M_out,
                          om_ilu_stats* st, hipStream_t s);
om_status host_ilut_impl(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val, double drop_tol,
                         double fill_factor, om_ilu** M_out, om_ilu_stats* st);
}  // namespace omss
