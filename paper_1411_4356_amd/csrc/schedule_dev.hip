// Solve schedules built on the device from the rows of a device ILU factor
// (the factor stays in HBM).  Same layout as the host build (schedule.cpp):
// per 64-row block the entries left of the block in three slot-major lists
// (far: column block <= g-3, mid: g-2, near: g-1; columns increasing with the
// slot, short rows padded with value 0 and a column of a finished block, far
// rows aligned to the last slot and the others to the first),
// need[slot] = newest column block a far slot reads, and the strictly-lower
// 64x64 diagonal block packed by column.
//   kind 0: L as stored (unit lower, no scaling);
//   kind 1: U reversed (row and column i -> n-1-i) with the pivots divided out
//           of the rows and returned as dinv = 1/u_ii.
// Division is written out as in the host build and contraction is off, so
// the schedules equal the host-built ones bit for bit.
#include <hipcub/hipcub.hpp>

#include "common.hpp"
#include "ilu.hpp"
#include "schedule.hpp"

#pragma clang fp contract(off)

namespace omss {

namespace {

constexpr int BLK = 64;
constexpr int TRI = BLK * (BLK - 1) / 2;

struct RowSrc {
    const int64_t* off;
    const int32_t* len;
    const int32_t* col;
    const double2* val;
};

__device__ inline int64_t tri_index(int c, int r) {  // r > c
    return (int64_t)c * (BLK - 1) - (int64_t)c * (c - 1) / 2 + (r - c - 1);
}

__device__ inline double2 cdiv(double ar, double ai, double br, double bi) {
    const double den = br * br + bi * bi;
    return make_double2((ar * br + ai * bi) / den, (ai * br - ar * bi) / den);
}

// number of entries of a sorted int32 run below v
__device__ inline int64_t count_below(const int32_t* c, int64_t len, int64_t v) {
    int64_t lo = 0, hi = len;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)c[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ inline int64_t wave_max(int64_t v) {
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Row ip of the solve matrix: its entries in increasing solve column.
//   kind 0: row ip of L;  kind 1: row n-1-ip of U without the pivot, reversed.
template <int KIND>
struct SolveRow {
    const int32_t* col;
    const double2* val;
    int64_t len;
    double2 piv;   // kind 1: u_ii
    __device__ SolveRow(const RowSrc& F, int64_t n, int64_t ip) {
        if (KIND == 0) {
            const int64_t b = F.off[ip];
            col = F.col + b;
            val = F.val + b;
            len = F.len[ip];
            piv = make_double2(1.0, 0.0);
        } else {
            const int64_t i = n - 1 - ip;
            const int64_t b = F.off[i];
            piv = F.val[b];
            col = F.col + b + 1;
            val = F.val + b + 1;
            len = F.len[i] - 1;
        }
    }
    // number of entries with solve column below t
    __device__ int64_t below(int64_t n, int64_t t) const {
        if (t <= 0) return 0;
        if (KIND == 0) return count_below(col, len, t);
        // solve column n-1-c < t  <=>  c > n-1-t  <=>  c >= n-t
        return len - count_below(col, len, n - t);
    }
    // q-th entry in increasing solve column
    __device__ void get(int64_t n, int64_t q, int64_t* c, double2* v) const {
        if (KIND == 0) {
            *c = col[q];
            *v = val[q];
        } else {
            const int64_t t = len - 1 - q;
            *c = n - 1 - (int64_t)col[t];
            const double2 u = val[t];
            *v = cdiv(u.x, u.y, piv.x, piv.y);
        }
    }
};

template <int KIND>
__global__ __launch_bounds__(BLK) void tri_count_kernel(RowSrc F, int64_t n, int64_t nblk, int64_t* cnt) {
    const int64_t g = blockIdx.x;
    const int r = threadIdx.x;
    const int64_t ip = g * BLK + r;
    int64_t c0 = 0, c1 = 0, c2 = 0;
    if (ip < n) {
        const SolveRow<KIND> R(F, n, ip);
        const int64_t b0 = R.below(n, (g - 2) * BLK), b1 = R.below(n, (g - 1) * BLK), b2 = R.below(n, g * BLK);
        c0 = b0;
        c1 = b1 - b0;
        c2 = b2 - b1;
    }
    c0 = wave_max(c0);
    c1 = wave_max(c1);
    c2 = wave_max(c2);
    if (r == 0) {
        cnt[g] = c0;
        cnt[(nblk + 1) + g] = c1;
        cnt[2 * (nblk + 1) + g] = c2;
    }
}

struct TriOut {
    const int64_t* off[3];   // far, mid, near slot offsets (nblk + 1)
    int32_t* col[3];
    double2* val[3];
    float2* val32[3];        // null without the complex64 copy
    int32_t* far_need;
    double2* dg;
    float2* dg32;
    double2* dinv;
    float2* dinv32;
};

template <int KIND>
__global__ __launch_bounds__(BLK) void tri_fill_kernel(RowSrc F, int64_t n, TriOut o) {
    const int64_t g = blockIdx.x;
    const int r = threadIdx.x;
    const int64_t ip = g * BLK + r;
    const int64_t nf = o.off[0][g + 1] - o.off[0][g];
    int64_t idx[3] = {0, 0, 0};   // next slot per list; far: starts past the padding
    int64_t fpad = nf;            // far slots of padding (all when the row is past n)
    if (ip < n) {
        const SolveRow<KIND> R(F, n, ip);
        fpad = nf - R.below(n, (g - 2) * BLK);
        idx[0] = fpad;
        for (int64_t q = 0; q < R.len; ++q) {
            int64_t c;
            double2 v;
            R.get(n, q, &c, &v);
            const int64_t cb = c / BLK;
            if (cb == g) {
                const int64_t at = g * TRI + tri_index((int)(c - g * BLK), r);
                o.dg[at] = v;
                if (o.dg32) o.dg32[at] = make_float2((float)v.x, (float)v.y);
                continue;
            }
            const int k = cb == g - 1 ? 2 : cb == g - 2 ? 1 : 0;
            const int64_t at = (o.off[k][g] + idx[k]++) * BLK + r;
            o.col[k][at] = (int32_t)c;
            o.val[k][at] = v;
            if (o.val32[k]) o.val32[k][at] = make_float2((float)v.x, (float)v.y);
        }
        if (KIND == 1) {
            const double2 d = cdiv(1.0, 0.0, R.piv.x, R.piv.y);
            o.dinv[ip] = d;
            if (o.dinv32) o.dinv32[ip] = make_float2((float)d.x, (float)d.y);
        }
    }
    // padding: value 0, a column of a finished block (far: column 0, before
    // the row's entries; mid and near: after them)
    for (int k = 0; k < 3; ++k) {
        const int64_t s0 = k == 0 ? 0 : idx[k];
        const int64_t s1 = k == 0 ? fpad : o.off[k][g + 1] - o.off[k][g];
        const int32_t pad = k == 0 ? 0 : (int32_t)((g - 3 + k) * BLK > 0 ? (g - 3 + k) * BLK : 0);
        for (int64_t s = s0; s < s1; ++s) {
            const int64_t at = (o.off[k][g] + s) * BLK + r;
            o.col[k][at] = pad;
            o.val[k][at] = make_double2(0.0, 0.0);
            if (o.val32[k]) o.val32[k][at] = make_float2(0.0f, 0.0f);
        }
    }
    // far_need: the newest column block any lane reads in the slot
    const int64_t f0 = o.off[0][g];
    for (int64_t s = 0; s < nf; ++s) {
        int64_t need = s >= fpad ? (int64_t)o.col[0][(f0 + s) * BLK + r] / BLK : 0;
        need = wave_max(need);
        if (r == 0) o.far_need[f0 + s] = (int32_t)need;
    }
}

template <int KIND>
om_status build_kind(const DevFactor& D, bool c64, TriSched& S, hipStream_t s) {
    const int64_t n = D.n;
    const int64_t nblk = (n + BLK - 1) / BLK;
    RowSrc F;
    if (KIND == 0) { F.off = D.l_off.p; F.len = D.l_len.p; F.col = D.l_col.p; F.val = D.l_val.p; }
    else { F.off = D.u_off.p; F.len = D.u_len.p; F.col = D.u_col.p; F.val = D.u_val.p; }
    // slot counts per block and class, then offsets by exclusive scans
    DevBuf<int64_t> cnt;
    OM_TRY(cnt.alloc((size_t)3 * (nblk + 1)));
    OM_HIP(hipMemsetAsync(cnt.p, 0, cnt.bytes(), s));
    hipLaunchKernelGGL(tri_count_kernel<KIND>, dim3((unsigned)nblk), dim3(BLK), 0, s, F, n, nblk, cnt.p);
    OM_HIP(hipGetLastError());
    DevBuf<int64_t>* offs[3] = {&S.far_off, &S.mid_off, &S.near_off};
    size_t tmp_bytes = 0;
    OM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, cnt.p, S.far_off.p, (int)(nblk + 1), s));
    DevBuf<unsigned char> tmp;
    OM_TRY(tmp.alloc(tmp_bytes + 1));
    int64_t tot[3];
    for (int k = 0; k < 3; ++k) {
        OM_TRY(offs[k]->alloc(nblk + 1));
        OM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, tmp_bytes, cnt.p + k * (nblk + 1), offs[k]->p, (int)(nblk + 1), s));
        OM_HIP(hipMemcpyAsync(&tot[k], offs[k]->p + nblk, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    }
    OM_HIP(hipStreamSynchronize(s));
    DevBuf<int32_t>* cols[3] = {&S.far_col, &S.mid_col, &S.near_col};
    DevBuf<double2>* vals[3] = {&S.far_val, &S.mid_val, &S.near_val};
    DevBuf<float2>* vals32[3] = {&S.far_val32, &S.mid_val32, &S.near_val32};
    TriOut o{};
    for (int k = 0; k < 3; ++k) {
        const size_t m = (size_t)std::max<int64_t>(1, tot[k]) * BLK;
        OM_TRY(cols[k]->alloc(m));
        OM_TRY(vals[k]->alloc(m));
        if (c64) OM_TRY(vals32[k]->alloc(m));
        else vals32[k]->release();
        o.off[k] = offs[k]->p;
        o.col[k] = cols[k]->p;
        o.val[k] = vals[k]->p;
        o.val32[k] = c64 ? vals32[k]->p : nullptr;
    }
    OM_TRY(S.far_need.alloc((size_t)std::max<int64_t>(1, tot[0])));
    OM_TRY(S.dg.alloc((size_t)nblk * TRI));
    OM_HIP(hipMemsetAsync(S.dg.p, 0, S.dg.bytes(), s));
    if (c64) {
        OM_TRY(S.dg32.alloc((size_t)nblk * TRI));
        OM_HIP(hipMemsetAsync(S.dg32.p, 0, S.dg32.bytes(), s));
    } else {
        S.dg32.release();
    }
    if (KIND == 1) {
        OM_TRY(S.dinv.alloc(n));
        if (c64) OM_TRY(S.dinv32.alloc(n));
        else S.dinv32.release();
    } else {
        S.dinv.release();
        S.dinv32.release();
    }
    o.far_need = S.far_need.p;
    o.dg = S.dg.p;
    o.dg32 = c64 ? S.dg32.p : nullptr;
    o.dinv = KIND == 1 ? S.dinv.p : nullptr;
    o.dinv32 = (KIND == 1 && c64) ? S.dinv32.p : nullptr;
    hipLaunchKernelGGL(tri_fill_kernel<KIND>, dim3((unsigned)nblk), dim3(BLK), 0, s, F, n, o);
    OM_HIP(hipGetLastError());
    OM_HIP(hipStreamSynchronize(s));
    S.n = n;
    S.nblk = nblk;
    S.rev = KIND == 1;
    S.depth = -1;   // not computed for device-built schedules
    S.nnz = KIND == 0 ? D.nnz_l : D.nnz_u - n;
    S.has_dinv = KIND == 1;
    S.nslots_far = tot[0];
    S.nslots_near = tot[1] + tot[2];
    return OM_OK;
}

}  // namespace

om_status build_tri_device(const DevFactor& D, int kind, bool c64, TriSched& S, hipStream_t s) {
    if (kind == 0) return build_kind<0>(D, c64, S, s);
    if (kind == 1) return build_kind<1>(D, c64, S, s);
    set_error("device schedule build supports the L and U solves only");
    return OM_EINVAL;
}

}  // namespace omss
