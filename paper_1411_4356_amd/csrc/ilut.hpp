// Host ILUT factor container and entry (internal).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace omss {

struct HostFactor {
    int64_t n = 0;
    std::vector<int64_t> l_ptr, u_ptr;
    std::vector<int32_t> l_col, u_col;
    std::vector<double> l_val, u_val;   // interleaved re, im
    std::vector<int32_t> perm;          // column permutation Q: perm[position] = column
    int64_t repaired = 0;
    int64_t pivots = 0;                 // column exchanges made by threshold pivoting
};

// Factor the n x n CSR matrix (values interleaved re,im; columns sorted per
// row), A Q ~ L U.  permtol = 0 disables pivoting.  Returns 0 on success.
int ilut_factor_host(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                     double drop_tol, double fill_factor, double permtol, HostFactor* out, std::string* err);

// Row-pipelined multi-threaded version (no pivoting): identical factor,
// `threads` host threads.  Returns 0 on success, 1 on breakdown (err set).
int ilut_factor_host_mt(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                        double drop_tol, double fill_factor, int threads, HostFactor* out, std::string* err);

}  // namespace omss
