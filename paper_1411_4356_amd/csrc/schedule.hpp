// Solve schedules for the ILU factors (internal).
#pragma once
#include <cstdint>
#include <vector>

#include "common.hpp"

namespace omss {

struct HostFactor;

// A strictly-lower CSR in solve coordinates (values interleaved re, im).
struct SolveCSR {
    int64_t n = 0;
    bool rev = false;
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    std::vector<double> val;
    std::vector<double> dinv;   // empty = none
};

// Entries of block g (rows 64g..64g+63) left of the block are split by the
// block of their column: near = block g-1, mid = block g-2, far = older.
constexpr int NEAR_BLOCKS = 2;

struct HostTri {
    int64_t n = 0, nblk = 0, depth = 0, nnz = 0;
    bool rev = false;
    std::vector<int64_t> far_off, mid_off, near_off;   // slot offsets per block (nblk + 1)
    std::vector<int32_t> far_col, mid_col, near_col, far_need;
    std::vector<double> far_val, mid_val, near_val, dg, dinv;
};

int64_t level_depth(int64_t n, const std::vector<int64_t>& ptr, const std::vector<int32_t>& col);
// kind: 0 = L, 1 = U (reversed, scaled), 2 = U^H (scaled), 3 = L^H (reversed)
void factor_to_solve(const HostFactor& F, int kind, SolveCSR& T);
void build_host_tri(const SolveCSR& T, HostTri& H);
om_status upload_tri(const HostTri& H, bool c64, TriSched& S);

}  // namespace omss
