// Host graph algorithms on CSR patterns: reverse Cuthill-McKee (Sec. III),
// symmetric permutation, transposition, bandwidth/profile (Sec. II).
#pragma once
#include <cstdint>
#include <vector>

namespace omss {

struct BandStats { int64_t ub, lb, B, up, lp, P; };

BandStats band_stats(int64_t n, const int64_t* row_ptr, const int32_t* col);

// perm[new] = old
void rcm_order(int64_t n, const int64_t* row_ptr, const int32_t* col, std::vector<int32_t>& perm);

// B = P A P^T: new pattern (sorted columns) and, per new entry, the index of
// its source entry in A.
void permute_pattern(int64_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* perm,
                     std::vector<int64_t>& new_ptr, std::vector<int32_t>& new_col, std::vector<int32_t>& src);

// A^T pattern (sorted columns) and source indices.
void transpose_pattern(int64_t n, const int64_t* row_ptr, const int32_t* col, std::vector<int64_t>& t_ptr,
                       std::vector<int32_t>& t_col, std::vector<int64_t>& src);

int host_threads();

}  // namespace omss
