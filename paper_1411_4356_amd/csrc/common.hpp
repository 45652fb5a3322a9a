// Internal definitions shared by the host and device sources of libomss.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/omss.h"

namespace omss {

// ---- error state (thread-local message, see om_last_error) -------------------
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
const char* last_error();

#define OM_HIP(expr)                                                                \
    do {                                                                            \
        hipError_t e__ = (expr);                                                    \
        if (e__ != hipSuccess) {                                                    \
            ::omss::set_error("%s:%d: %s failed: %s", __FILE__, __LINE__, #expr,     \
                              hipGetErrorString(e__));                              \
            return e__ == hipErrorOutOfMemory ? OM_ENOMEM : OM_EHIP;                \
        }                                                                           \
    } while (0)

#define OM_TRY(expr)                         \
    do {                                     \
        om_status s__ = (expr);              \
        if (s__ != OM_OK) return s__;        \
    } while (0)

// ---- device buffer ------------------------------------------------------------
template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    om_status alloc(size_t count) {
        release();
        if (count == 0) return OM_OK;
        hipError_t e = hipMalloc((void**)&p, count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            set_error("hipMalloc of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
            return OM_ENOMEM;
        }
        n = count;
        return OM_OK;
    }
    om_status upload(const T* host, size_t count, hipStream_t s) {
        OM_TRY(alloc(count));
        if (count) OM_HIP(hipMemcpyAsync(p, host, count * sizeof(T), hipMemcpyHostToDevice, s));
        return OM_OK;
    }
    size_t bytes() const { return n * sizeof(T); }
};

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Grid size helper.
inline unsigned blocks_for(int64_t work, int per_block) {
    int64_t b = (work + per_block - 1) / per_block;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace omss

// ---- handle types ---------------------------------------------------------------

struct om_csr {
    int64_t n = 0, nnz = 0;
    int32_t batch = 1;
    int32_t N = 0;                       // Hilbert dimension (0 if no model)
    omss::DevBuf<int32_t> row_ptr, col;  // pattern (shared by the batch)
    omss::DevBuf<double2> val;           // batch * nnz
    omss::DevBuf<float2> val32;          // optional complex64 copy
    // conjugate transpose, built on demand for A^H products
    bool has_t = false;
    omss::DevBuf<int32_t> t_row_ptr, t_col, t_src;
    omss::DevBuf<double2> t_val;
    omss::DevBuf<float2> t_val32;
    // host copy of the pattern (row_ptr as int64), built on demand
    std::vector<int64_t> h_row_ptr;
    std::vector<int32_t> h_col;
    // model description
    bool has_model = false;
    std::vector<om_params> params;
    int32_t trace_mode = OM_TRACE_REPLACE_ROW0;
    std::vector<double> w;
    // ordering: perm[new] = old relative to the natural model ordering
    bool permuted = false;
    std::vector<int32_t> perm;
    omss::DevBuf<int32_t> perm_d, iperm_d;
    // model parameters (8 doubles per item, in the stencil's order) and trace
    // weights on the device, uploaded by the first matrix-free product
    omss::DevBuf<double> lapply_params, lapply_w;
};

namespace omss {

struct HostFactor;

// One unit-lower triangular solve in "solve coordinates" (an upper factor is
// stored row- and column-reversed so that it is lower triangular too); see
// schedule.cpp for the layout.  dinv (optional): per-row factor applied to the
// right-hand side (the inverse pivots of U, whose rows are stored scaled).
struct TriSched {
    int64_t n = 0, nblk = 0, nslots_far = 0, nslots_near = 0, nnz = 0;
    bool rev = false, has_dinv = false;
    int64_t depth = 0;
    DevBuf<int64_t> far_off, mid_off, near_off;
    DevBuf<int32_t> far_col, mid_col, near_col, far_need;
    DevBuf<double2> far_val, mid_val, near_val, dg, dinv;
    DevBuf<float2> far_val32, mid_val32, near_val32, dg32, dinv32;
};

// POD view of a TriSched for kernels.
template <typename VT>
struct TriView {
    const int64_t* far_off;
    const int64_t* mid_off;
    const int64_t* near_off;
    const int32_t* far_col;
    const int32_t* mid_col;
    const int32_t* near_col;
    const int32_t* far_need;
    const VT* far_val;
    const VT* mid_val;
    const VT* near_val;
    const VT* dg;
    const VT* dinv;   // may be null
    int64_t n, nblk;
    int32_t rev;
};

// Device scratch shared by the cooperative triangular solves of one factor
// set: per item the far partial sums and ready flags of every block, a
// progress counter, and one abort flag.
struct TrsvScratch {
    DevBuf<double2> far_buf;    // batch * nblk * 64 (complex64 kernels use half of it)
    DevBuf<int32_t> fdone;      // batch * nblk, epoch tags
    DevBuf<int64_t> progress;   // batch, (epoch << 32) | blocks done
    DevBuf<int32_t> abort_flag; // 1 word
    uint32_t epoch = 0;
    // solves of several right-hand sides with one shared factor
    DevBuf<double2> m_far;      // nblk * batch * 64 partial sums
    DevBuf<double2> m_x;        // n * batch: the solution in solve order, interleaved
    DevBuf<int32_t> m_fdone;    // nblk, epoch tags
    DevBuf<int64_t> m_progress; // (epoch << 32) | blocks done
};

}  // namespace omss

struct om_ilu {
    int64_t n = 0;
    int32_t batch = 0;
    uint32_t flags = 0;
    bool host_only = false;
    bool shared = false;   // one factor (of item 0) serves every batch item
    std::vector<std::unique_ptr<omss::HostFactor>> host;   // per factor (1 if shared)
    // per factor: 0 = L, 1 = U (reversed, scaled), 2 = U^H (scaled), 3 = L^H (reversed)
    std::vector<omss::TriSched> sched;                     // factors * 4
    omss::DevBuf<omss::TriView<double2>> views64;          // batch * 4
    omss::DevBuf<omss::TriView<float2>> views32;           // batch * 4
    omss::TrsvScratch scratch;
    om_ilu_stats stats{};
};
