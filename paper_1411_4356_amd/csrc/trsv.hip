// Preconditioner application: blocked sparse triangular solves on the device.
//
// The factors of an RCM-ordered ILUT are banded and their rows depend on the
// rows just before them, so the solve walks 64-row blocks (one wavefront of
// rows, lane = row) in order.  For block g the unknowns are
//     x_g = T_gg^{-1} (dinv .* y_g - sum_{h < g} T_gh x_h),
// T_gg unit lower triangular.  The entries left of the block are in three
// slot-major lists by the block of their column (near = g-1, mid = g-2, far =
// older); T_gg is swept column by column: at step c the finished unknown of
// lane c is broadcast with readlane and subtracted from the rows below it.
//
// trsv_chain_kernel  one workgroup per batch item, everything in order.
// trsv_coop_kernel   per batch item one critical workgroup and H helpers.
//   Helpers stream the far list of later blocks at memory bandwidth and
//   publish each block's partial sum.  The critical workgroup keeps the last
//   two blocks of unknowns in an LDS ring: wave 0 sweeps block g while waves
//   1-3 prefetch the triangle and the near list of block g+1 into LDS and
//   compute its mid part; then all waves finish the near part of g+1.
//   Communication: data that crosses workgroups is stored write-through
//   (agent-coherent stores), followed by s_waitcnt and a flag store; readers
//   poll flags with coherent loads and read published data with coherent
//   loads, except unknowns two or more blocks behind the progress counter,
//   whose cache lines can no longer hold unfinished rows.  Flags carry the
//   launch's epoch, so nothing is reset between launches.  The launch is
//   cooperative (all workgroups co-resident) and every wait is bounded: a
//   timeout raises an abort flag that ends all waits.  All workgroups of a
//   batch item are placed on one XCD (workgroup id mod 8) so that they share
//   its L2.
#include <cstdio>

#include "common.hpp"
#include "cplx.hpp"
#include "kernels.hpp"
#include "profile.hpp"
#include "schedule.hpp"

namespace omss {

__device__ inline double bcast(double v, int l) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ inline float bcast(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

constexpr int TW = 4;              // waves per workgroup
constexpr int TRI_N = 2016;        // packed strictly-lower 64x64
constexpr int TRI_LD = TRI_N + 1;  // a triangle in LDS: the packed entries, then a zero
constexpr int RING = NEAR_BLOCKS * 64;
constexpr int NEAR_PF = 64;        // near slots of the next block staged in LDS (all: a row has at most 64 entries in the previous block)
constexpr int NXCD = 8;
constexpr int FU = 8;               // slots per wave per chunk in the streamed loops
constexpr int FH = 16;              // the same for the far lists streamed by the helpers
constexpr long long SPIN_LIMIT = 1ll << 22;

// Column sweep of the unit-lower diagonal block (wave 0): r holds the right-
// hand side of lane = row on entry and the unknown on exit.  Columns are
// taken in chunks of SWC: the LDS entries of chunk k+1 are requested before
// the steps of chunk k (scheduling barriers keep that order), so that the
// chain of dependent steps does not wait for LDS.  Lanes at or above the
// diagonal of a column read the zero after the packed entries (tri[TRI_N]):
// their update subtracts zero, so every step runs on all lanes, without a
// lane mask on the chain.
constexpr int SWC = 8;
template <typename VT>
__device__ __forceinline__ void sweep_load(VT (&t)[SWC], const VT* tri, int c0, int lane) {
#pragma unroll
    for (int j = 0; j < SWC; ++j) {
        const int c = c0 + j;
        if (c < 63) t[j] = tri[lane > c ? c * 63 - (c * (c - 1)) / 2 + lane - c - 1 : TRI_N];
    }
}
template <int K, typename VT>
__device__ __forceinline__ void sweep_chunk(VT& r, const VT (&cur)[SWC], VT (&nxt)[SWC], const VT* tri, int lane) {
    using ST = typename Scalar<VT>::type;
    if (K + 1 < 8) sweep_load(nxt, tri, (K + 1) * SWC, lane);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < SWC; ++j) {
        const int c = K * SWC + j;
        if (c < 63) {
            const VT t = cur[j];
            const ST xr = bcast(r.x, c);
            const ST xi = bcast(r.y, c);
            r.x -= t.x * xr;
            r.x += t.y * xi;
            r.y -= t.x * xi;
            r.y -= t.y * xr;
        }
    }
    __builtin_amdgcn_sched_barrier(0);
}
template <typename VT>
__device__ __forceinline__ VT sweep(VT r, const VT* tri, int lane) {
    VT ta[SWC], tb[SWC];
    sweep_load(ta, tri, 0, lane);
    sweep_chunk<0>(r, ta, tb, tri, lane);
    sweep_chunk<1>(r, tb, ta, tri, lane);
    sweep_chunk<2>(r, ta, tb, tri, lane);
    sweep_chunk<3>(r, tb, ta, tri, lane);
    sweep_chunk<4>(r, ta, tb, tri, lane);
    sweep_chunk<5>(r, tb, ta, tri, lane);
    sweep_chunk<6>(r, ta, tb, tri, lane);
    sweep_chunk<7>(r, tb, ta, tri, lane);
    return r;
}

// An unwritten far sum has every bit set.  A far sum counts as written only
// when none of its 32-bit words is all ones: a store seen in part then reads
// as unwritten, and a written value that happens to hold such a word costs a
// wait for the flag, never a wrong result.
template <typename VT> __device__ inline bool is_unwritten(VT v);
template <> __device__ inline bool is_unwritten<double2>(double2 v) {
    const unsigned long long a = (unsigned long long)__double_as_longlong(v.x);
    const unsigned long long b = (unsigned long long)__double_as_longlong(v.y);
    return (unsigned)a == ~0u || (unsigned)(a >> 32) == ~0u || (unsigned)b == ~0u || (unsigned)(b >> 32) == ~0u;
}
template <> __device__ inline bool is_unwritten<float2>(float2 v) {
    return __float_as_int(v.x) == -1 || __float_as_int(v.y) == -1;
}
template <typename VT> __device__ inline VT unwritten();
template <> __device__ inline double2 unwritten<double2>() {
    return make_double2(__longlong_as_double(-1ll), __longlong_as_double(-1ll));
}
template <> __device__ inline float2 unwritten<float2>() {
    return make_float2(__int_as_float(-1), __int_as_float(-1));
}

// coherent (agent-scope) loads and write-through stores of complex values
template <typename VT> __device__ inline VT ld_coh(const VT* p);
template <> __device__ inline double2 ld_coh<double2>(const double2* p) {
    const double* q = reinterpret_cast<const double*>(p);
    return make_double2(__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                        __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
template <> __device__ inline float2 ld_coh<float2>(const float2* p) {
    const float* q = reinterpret_cast<const float*>(p);
    return make_float2(__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                       __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
template <typename VT> __device__ inline void st_wt(VT* p, VT v);
template <> __device__ inline void st_wt<double2>(double2* p, double2 v) {
    double* q = reinterpret_cast<double*>(p);
    __hip_atomic_store(q, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(q + 1, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <> __device__ inline void st_wt<float2>(float2* p, float2 v) {
    float* q = reinterpret_cast<float*>(p);
    __hip_atomic_store(q, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(q + 1, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- single-workgroup chain
template <typename VT>
__global__ __launch_bounds__(64 * TW) void trsv_chain_kernel(const TriView<VT>* __restrict__ views, int kind,
                                                              const VT* rhs, VT* out, int64_t n,
                                                              const int32_t* __restrict__ active) {
    const int b = blockIdx.x;
    if (active && !active[b]) return;
    const TriView<VT> S = views[b * 4 + kind];
    const VT* y = rhs + (int64_t)b * n;
    VT* x = out + (int64_t)b * n;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    __shared__ VT part[TW][64];
    __shared__ VT tri[TRI_LD];
    if (threadIdx.x == 0) tri[TRI_N] = czero<VT>();   // (ordered by the first barrier below)

    for (int64_t g = 0; g < S.nblk; ++g) {
        {
            constexpr int TPER = (TRI_N + 64 * TW - 1) / (64 * TW);
            VT tv[TPER];
#pragma unroll
            for (int j = 0; j < TPER; ++j)
                if (threadIdx.x + j * 64 * TW < TRI_N) tv[j] = S.dg[g * TRI_N + threadIdx.x + j * 64 * TW];
#pragma unroll
            for (int j = 0; j < TPER; ++j)
                if (threadIdx.x + j * 64 * TW < TRI_N) tri[threadIdx.x + j * 64 * TW] = tv[j];
        }
        VT acc = czero<VT>();
        for (int list = 0; list < 3; ++list) {
            const int64_t* off = list == 0 ? S.far_off : list == 1 ? S.mid_off : S.near_off;
            const int32_t* cl = list == 0 ? S.far_col : list == 1 ? S.mid_col : S.near_col;
            const VT* vl = list == 0 ? S.far_val : list == 1 ? S.mid_val : S.near_val;
            const int64_t e1 = off[g + 1];
            for (int64_t c0 = off[g] + (int64_t)wave * FU; c0 < e1; c0 += (int64_t)TW * FU) {
                const int cnt = (int)(e1 - c0 < FU ? e1 - c0 : FU);
                int32_t cc[FU];
                VT vv[FU];
#pragma unroll
                for (int j = 0; j < FU; ++j)
                    if (j < cnt) { cc[j] = cl[(c0 + j) * 64 + lane]; vv[j] = vl[(c0 + j) * 64 + lane]; }
                VT xv[FU];
#pragma unroll
                for (int j = 0; j < FU; ++j)
                    if (j < cnt) xv[j] = x[S.rev ? (n - 1 - cc[j]) : cc[j]];
#pragma unroll
                for (int j = 0; j < FU; ++j)
                    if (j < cnt) cfma(acc, vv[j], xv[j]);
            }
        }
        part[wave][lane] = acc;
        __syncthreads();
        if (wave == 0) {
            const int64_t row = g * 64 + lane;
            const bool valid = row < n;
            const int64_t mi = S.rev ? (n - 1 - row) : row;
            VT r = czero<VT>();
            if (valid) {
                r = y[mi];
                if (S.dinv) r = cmul(r, S.dinv[row]);
            }
#pragma unroll
            for (int w = 0; w < TW; ++w) r = csub(r, part[w][lane]);
            r = sweep(r, tri, lane);
            if (valid) x[mi] = r;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- cooperative version
struct CoopArgs {
    double2* far_buf;     // batch * nblk * 64 values of VT (reinterpreted)
    int32_t* fdone;       // batch * nblk
    int64_t* progress;    // batch
    int32_t* abort_flag;
    uint32_t epoch;
    int helpers;          // helper workgroups per item
    int batch;
    int per_xcd;          // workgroups of one item on one XCD
    int xcd_per_item;     // XCDs an item spans (8 / batch when batch divides 8, else 1)
    unsigned long long* tstat;   // diagnostics (nullable)
};

__device__ inline bool aborted(const int32_t* f) {
    return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

__device__ inline void raise_abort(int32_t* f) {
    __hip_atomic_store(f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Control flow around barriers depends only on wave-uniform values
// (readfirstlane), so that every wave executes the same barriers.
__device__ inline int64_t rfl64(int64_t v) {
    const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return ((int64_t)hi << 32) | (uint32_t)lo;
}

__device__ inline int block_or(bool v, int* buf) {
    const unsigned long long b = __ballot(v);
    if ((threadIdx.x & 63) == 0) buf[threadIdx.x >> 6] = b != 0ull;
    __syncthreads();
    int r = 0;
    for (int w = 0; w < TW; ++w) r |= buf[w];
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(r);
}

// Wait until *p >= target; returns the observed value or -1 on timeout/abort.
__device__ inline int64_t wait_ge64(const int64_t* p, int64_t target, int32_t* abort_flag) {
    long long spins = 0;
    int64_t v;
    while ((v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < target) {
        if (aborted(abort_flag)) return -1;
        if (++spins > SPIN_LIMIT) { raise_abort(abort_flag); return -1; }
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    return v;
}

__device__ inline bool wait_eq32(const int32_t* p, int32_t v, int32_t* abort_flag) {
    long long spins = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != v) {
        if (aborted(abort_flag)) return false;
        if (++spins > SPIN_LIMIT) { raise_abort(abort_flag); return false; }
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    return true;
}

// Loads through explicit address spaces: read-only schedule metadata with a
// wave-uniform index through the scalar cache (its wait does not include the
// vector loads in flight), everything else as global (not flat) loads.
template <typename T>
__device__ __forceinline__ T ldc(const T* p) { return *(const __attribute__((address_space(4))) T*)p; }
template <typename T>
__device__ __forceinline__ T ldg(const T* p) { return *(const __attribute__((address_space(1))) T*)p; }
// complex values through the compiler's own vector types (a load of the HIP
// vector class would go through its generic-pointer copy constructor)
template <>
__device__ __forceinline__ double2 ldg<double2>(const double2* p) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    const v2 v = *(const __attribute__((address_space(1))) v2*)p;
    return make_double2(v.x, v.y);
}
template <>
__device__ __forceinline__ float2 ldg<float2>(const float2* p) {
    typedef float v2 __attribute__((ext_vector_type(2)));
    const v2 v = *(const __attribute__((address_space(1))) v2*)p;
    return make_float2(v.x, v.y);
}

// Copy `bytes` (a multiple of 16) from global memory to LDS without passing
// through registers: 1 KiB per wave instruction (16 bytes per lane), chunks
// dealt to the `nw` waves numbered from `w`.  The copy completes
// asynchronously; the caller waits (s_waitcnt) before its next barrier.
__device__ inline void copy_to_lds(void* dst, const void* src, int64_t bytes, int w, int nw, int lane) {
    const char* sp = static_cast<const char*>(src);
    char* dp = static_cast<char*>(dst);
    for (int64_t c = (int64_t)w * 1024; c < bytes; c += (int64_t)nw * 1024) {
        const int64_t off = c + (int64_t)lane * 16;
        if (off < bytes)
            __builtin_amdgcn_global_load_lds(sp + off, (__attribute__((address_space(3))) void*)(dp + c), 16, 0, 0);
    }
}


template <typename VT>
__global__ __launch_bounds__(64 * TW) void trsv_coop_kernel(const TriView<VT>* __restrict__ views, int kind,
                                                             const VT* rhs, VT* out, int64_t n,
                                                             const int32_t* __restrict__ active, CoopArgs a) {
    // placement: workgroup w sits on XCD w % 8.  When batch divides 8, item b spans
    // the XCDs congruent to b modulo batch; otherwise item b uses XCD b % 8.
    const int xcd = blockIdx.x % NXCD;
    const int q = blockIdx.x / NXCD;
    int b, role;
    if (a.xcd_per_item > 1) {
        b = xcd % a.batch;
        role = q * a.xcd_per_item + xcd / a.batch;   // 0 = critical workgroup (on XCD b)
    } else {
        b = xcd + NXCD * (q / a.per_xcd);
        role = q % a.per_xcd;
    }
    if (b >= a.batch || role > a.helpers) return;
    if (active && !active[b]) return;
    const TriView<VT> S = views[b * 4 + kind];
    VT* x = out + (int64_t)b * n;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    VT* far_buf = reinterpret_cast<VT*>(a.far_buf) + (int64_t)b * S.nblk * 64;
    int32_t* fdone = a.fdone + (int64_t)b * S.nblk;
    int64_t* progress = a.progress + b;
    const int64_t ep = (int64_t)a.epoch << 32;
    // LDS of the critical workgroup, as separate objects: the compiler then
    // knows that reads of one do not depend on copies still landing in another
    __shared__ __attribute__((aligned(16))) VT s_tri[2][TRI_LD];
    __shared__ __attribute__((aligned(16))) VT s_near_v[NEAR_PF][64];
    __shared__ __attribute__((aligned(16))) int32_t s_near_c[NEAR_PF][64];
    __shared__ VT s_part[TW][64];
    __shared__ VT s_mid[2][TW - 1][64];
    __shared__ VT s_ring[RING];
    __shared__ int s_fail;
    __shared__ int s_orbuf[TW];

    if (role > 0) {
        // ---- helper: far parts of blocks role-1, role-1+H, ...
        int64_t known = 0;   // blocks finished in this epoch, as last observed
        for (int64_t g = role - 1; g < S.nblk; g += a.helpers) {
            {
                const int64_t v = rfl64(__hip_atomic_load(progress, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) - ep;
                if (v > known && v <= S.nblk) known = v;
            }
            VT acc = czero<VT>();
            bool ok = true;
            const int64_t s1 = ldc(S.far_off + g + 1);
            // chunks of FH consecutive slots per wave: the columns and values of a
            // chunk are loaded first (they do not depend on the solve), then the
            // progress is checked once for the chunk, then the unknowns are gathered
            for (int64_t c0 = ldc(S.far_off + g) + (int64_t)wave * FH; c0 < s1; c0 += (int64_t)TW * FH) {
                const int cnt = (int)(s1 - c0 < FH ? s1 - c0 : FH);
                // slots past the end of the block repeat its last slot (no
                // branches between the loads) and are not accumulated
                int32_t cc[FH];
                VT vv[FH];
#pragma unroll
                for (int j = 0; j < FH; ++j) {
                    const int64_t sl = c0 + (j < cnt ? j : cnt - 1);
                    cc[j] = ldg(S.far_col + sl * 64 + lane);
                    vv[j] = ldg(S.far_val + sl * 64 + lane);
                }
                // far slots need non-decreasing blocks (rows end at the last slot)
                const int64_t needmax = ldc(S.far_need + c0 + cnt - 1);
                if (needmax + 2 > known) {
                    // every lane waits for the same target; the result is made
                    // wave-uniform so that the loop exits uniformly
                    const int64_t v = rfl64(wait_ge64(progress, ep + needmax + 1, a.abort_flag));
                    if (v < 0) { ok = false; break; }
                    known = v - ep;
                }
                VT xv[FH];
#pragma unroll
                for (int j = 0; j < FH; ++j) {
                    const int64_t c = cc[j];
                    const VT* px = x + (S.rev ? (n - 1 - c) : c);
                    // unknowns of the newest finished block may share a cache line
                    // with unfinished rows: read them coherently
                    xv[j] = (c >> 6) + 1 >= known ? ld_coh(px) : ldg(px);
                }
#pragma unroll
                for (int j = 0; j < FH; ++j)
                    if (j < cnt) cfma(acc, vv[j], xv[j]);
            }
            s_part[wave][lane] = acc;
            if (block_or(!ok, s_orbuf)) return;
            if (wave == 0) {
                VT t = s_part[0][lane];
#pragma unroll
                for (int w = 1; w < TW; ++w) t = cadd(t, s_part[w][lane]);
                st_wt(far_buf + g * 64 + lane, t);
                __builtin_amdgcn_s_waitcnt(0);
                if (lane == 0) __hip_atomic_store(fdone + g, (int32_t)a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            __syncthreads();
        }
        return;
    }

    // ---- critical workgroup
    const VT* y = rhs + (int64_t)b * n;
    unsigned long long t_near = 0, t_wait = 0, t_sweep = 0, t_tail = 0, t_pub = 0, t_bar = 0, tA = 0;
    // prologue: triangle and near list of block 0, mid(0) = 0
    {
        const int64_t n0 = ldc(S.near_off), n1 = ldc(S.near_off + 1);
        const int64_t nl = n1 - n0 < NEAR_PF ? n1 - n0 : NEAR_PF;
        copy_to_lds(s_tri[0], S.dg, (int64_t)TRI_N * sizeof(VT), wave, TW, lane);
        copy_to_lds(s_near_c, S.near_col + n0 * 64, nl * 64 * 4, wave, TW, lane);
        copy_to_lds(s_near_v, S.near_val + n0 * 64, nl * 64 * (int64_t)sizeof(VT), wave, TW, lane);
        __builtin_amdgcn_s_waitcnt(0);
    }
    if (wave > 0) s_mid[0][wave - 1][lane] = czero<VT>();
    if (threadIdx.x == 0) {
        s_fail = 0;
        s_tri[0][TRI_N] = czero<VT>();
        s_tri[1][TRI_N] = czero<VT>();
        __hip_atomic_store(progress, ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    constexpr int MPW = (64 + TW - 2) / (TW - 1);   // mid slots per wave (a row has at most 64)
    for (int64_t g = 0; g < S.nblk; ++g) {
        if (a.tstat && threadIdx.x == 0) tA = wall_clock64();
        const int buf = (int)(g & 1);
        const int64_t g1 = g + 1;
        // loads that depend on nothing computed: wave 0 the right-hand side of
        // block g, waves 1-3 the mid list of block g+1 (columns in block g-1)
        VT r0 = czero<VT>(), dv = czero<VT>();
        // (defined on every path, so that they are not live across the sweep)
        int32_t mc[MPW];
        VT mv[MPW];
#pragma unroll
        for (int j = 0; j < MPW; ++j) { mc[j] = 0; mv[j] = czero<VT>(); }
        const int64_t m0 = g1 < S.nblk ? ldc(S.mid_off + g1) : 0, m1 = g1 < S.nblk ? ldc(S.mid_off + g1 + 1) : 0;
        VT fb = czero<VT>();
        if (wave == 0) {
            const int64_t row = g * 64 + lane;
            if (row < n) {
                r0 = ldg(y + (S.rev ? (n - 1 - row) : row));
                if (S.dinv) dv = ldg(S.dinv + row);
            }
            // the helpers' far sum of block g, read now: if it is already
            // written, neither the flag nor a second read is on the chain
            fb = ld_coh(far_buf + g * 64 + lane);
        } else {
            if (m1 > m0) {
                // slots past the end repeat the last one (not accumulated)
#pragma unroll
                for (int j = 0; j < MPW; ++j) {
                    int64_t sl = m0 + (wave - 1) + (int64_t)j * (TW - 1);
                    sl = sl < m1 ? sl : m1 - 1;
                    mc[j] = ldg(S.mid_col + sl * 64 + lane);
                    mv[j] = ldg(S.mid_val + sl * 64 + lane);
                }
            }
            // the triangle of block g+1 goes to the idle buffer now
            if (g1 < S.nblk)
                copy_to_lds(s_tri[buf ^ 1], S.dg + g1 * TRI_N, (int64_t)TRI_N * sizeof(VT), wave - 1, TW - 1, lane);
        }
        // near part of block g (columns in block g-1), x from the ring
        VT acc = czero<VT>();
        {
            const int64_t n0 = ldc(S.near_off + g), n1 = ldc(S.near_off + g + 1);
            const int64_t nl = n1 - n0 < NEAR_PF ? n1 - n0 : NEAR_PF;
            // rounds of NR slots per wave: columns, then values and unknowns, then products
            constexpr int NR = 8;
            for (int64_t k0 = wave; k0 < nl; k0 += (int64_t)TW * NR) {
                int32_t cc[NR];
                VT vv[NR], xv[NR];
#pragma unroll
                for (int j = 0; j < NR; ++j)
                    if (k0 + j * TW < nl) cc[j] = s_near_c[k0 + j * TW][lane];
#pragma unroll
                for (int j = 0; j < NR; ++j)
                    if (k0 + j * TW < nl) { vv[j] = s_near_v[k0 + j * TW][lane]; xv[j] = s_ring[cc[j] & (RING - 1)]; }
#pragma unroll
                for (int j = 0; j < NR; ++j)
                    if (k0 + j * TW < nl) cfma(acc, vv[j], xv[j]);
            }
            for (int64_t c0 = n0 + NEAR_PF + (int64_t)wave * FU; c0 < n1; c0 += (int64_t)TW * FU) {
                const int cnt = (int)(n1 - c0 < FU ? n1 - c0 : FU);
                int32_t cc[FU];
                VT vv[FU];
#pragma unroll
                for (int j = 0; j < FU; ++j)
                    if (j < cnt) { cc[j] = ldg(S.near_col + (c0 + j) * 64 + lane); vv[j] = ldg(S.near_val + (c0 + j) * 64 + lane); }
#pragma unroll
                for (int j = 0; j < FU; ++j)
                    if (j < cnt) cfma(acc, vv[j], s_ring[cc[j] & (RING - 1)]);
            }
        }
        s_part[wave][lane] = acc;
        if (wave == 0) {
            // publish block g-1: its unknowns were stored at the end of the
            // previous iteration, and waiting for them here rather than there
            // keeps the store latency off the chain of blocks
            if (g > 0) {
                const unsigned long long tP = a.tstat ? wall_clock64() : 0;
                __builtin_amdgcn_s_waitcnt(0);
                if (lane == 0) __hip_atomic_store(progress, ep + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (a.tstat && lane == 0) t_pub += wall_clock64() - tP;
            }
            const unsigned long long tB = a.tstat ? wall_clock64() : 0;
            if (__ballot(is_unwritten(fb)) != 0ull) {
                // not yet (or only partly) written: wait for the flag, then read again
                if (lane == 0 && !wait_eq32(fdone + g, (int32_t)a.epoch, a.abort_flag)) s_fail = 1;
                fb = ld_coh(far_buf + g * 64 + lane);
            }
            if (a.tstat && lane == 0) { const unsigned long long tC = wall_clock64(); t_near += tB - tA; t_wait += tC - tB; tA = tC; }
        }
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(s_fail)) return;
        if (a.tstat && threadIdx.x == 0) { const unsigned long long tE = wall_clock64(); t_bar += tE - tA; tA = tE; }
        if (wave == 0) {
            const int64_t row = g * 64 + lane;
            const bool valid = row < n;
            VT r = S.dinv ? cmul(r0, dv) : r0;
            r = csub(r, fb);
#pragma unroll
            for (int w = 0; w < TW; ++w) r = csub(r, s_part[w][lane]);
#pragma unroll
            for (int w = 0; w < TW - 1; ++w) r = csub(r, s_mid[buf][w][lane]);
            r = sweep(r, s_tri[buf], lane);
            s_ring[(g * 64 + lane) & (RING - 1)] = r;
            if (valid) st_wt(x + (S.rev ? (n - 1 - row) : row), r);
            // consumed: marked unwritten for the next solve
            st_wt(far_buf + g * 64 + lane, unwritten<VT>());
            if (a.tstat && lane == 0) { const unsigned long long tD = wall_clock64(); t_sweep += tD - tA; tA = tD; }
        } else if (g1 < S.nblk) {
            // waves 1-3: stage the near list of block g+1 (copies straight to
            // LDS, completed before the barrier) and finish its mid part from
            // the prefetched list and block g-1 in the ring
            {
                const int64_t n0 = ldc(S.near_off + g1), n1 = ldc(S.near_off + g1 + 1);
                const int64_t nl = n1 - n0 < NEAR_PF ? n1 - n0 : NEAR_PF;
                copy_to_lds(s_near_c, S.near_col + n0 * 64, nl * 64 * 4, wave - 1, TW - 1, lane);
                copy_to_lds(s_near_v, S.near_val + n0 * 64, nl * 64 * (int64_t)sizeof(VT), wave - 1, TW - 1, lane);
            }
            VT m = czero<VT>();
#pragma unroll
            for (int j = 0; j < MPW; ++j) {
                const int64_t sl = m0 + (wave - 1) + (int64_t)j * (TW - 1);
                if (sl < m1) cfma(m, mv[j], s_ring[mc[j] & (RING - 1)]);
            }
            s_mid[buf ^ 1][wave - 1][lane] = m;
            __builtin_amdgcn_s_waitcnt(0);
        }
        __syncthreads();
        if (a.tstat && threadIdx.x == 0) t_tail += wall_clock64() - tA;
    }
    if (wave == 0) {
        __builtin_amdgcn_s_waitcnt(0);
        if (lane == 0) __hip_atomic_store(progress, ep + S.nblk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (a.tstat && threadIdx.x == 0) {
        atomicAdd(a.tstat + 0, t_near - t_pub);
        atomicAdd(a.tstat + 1, t_wait);
        atomicAdd(a.tstat + 2, t_sweep);
        atomicAdd(a.tstat + 3, t_tail);
        atomicAdd(a.tstat + 4, t_pub);
        atomicAdd(a.tstat + 5, t_bar);
    }
}

// ---------------------------------------------------------------- several right-hand sides, one factor
// With one factor shared by the batch, all right-hand sides are solved in one
// pass over the factor.  The critical workgroup has one wave per right-hand
// side: per 64-row block every wave takes its side's far+mid partial sums
// from the helpers, subtracts the near part (block g-1, its side's unknowns
// in an LDS ring, the near list staged in LDS) and sweeps the diagonal block.
// The helpers stream the far and mid lists for all sides at once: the
// unknowns are kept in solve order and interleaved by side (X[c * nb + b]),
// so that one gathered column is one contiguous run.  Flags and placement of
// the protocol are those of the single-side kernel above.
constexpr int MAXB = 8;
constexpr int MT = 64 * MAXB;

struct MrhsArgs {
    void* X;               // n * nb of VT
    void* far_buf;         // nblk * nb * 64 of VT
    int32_t* fdone;
    int64_t* progress;
    int32_t* abort_flag;
    uint32_t epoch;
    int helpers;
    int nb;
    unsigned long long* tstat;   // diagnostics (nullable): wall-clock ticks waiting / total
};

template <typename VT>
struct MrhsShared {
    union {
        struct {
            VT tri[2][TRI_LD];
            VT near_v[NEAR_PF][64];
            uint8_t near_c[NEAR_PF][64];   // column within the previous block
            VT ring[RING][MAXB];
        } cw;
        struct {
            VT part[MAXB][MAXB][64];       // [wave][side][lane]
        } hp;
    };
    int fail;
    int orbuf[MAXB];
};

template <typename VT>
__device__ inline int mrhs_block_or(bool v, int* buf) {
    const unsigned long long b = __ballot(v);
    if ((threadIdx.x & 63) == 0) buf[threadIdx.x >> 6] = b != 0ull;
    __syncthreads();
    int r = 0;
    for (int w = 0; w < MAXB; ++w) r |= buf[w];
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(r);
}

template <typename VT>
__global__ __launch_bounds__(MT) void trsv_mrhs_kernel(const TriView<VT>* __restrict__ views, int kind,
                                                        const VT* rhs, VT* out, int64_t n,
                                                        const int32_t* __restrict__ active, MrhsArgs a) {
    const TriView<VT> S = views[kind];
    const int role = blockIdx.x;
    if (role > a.helpers) return;
    const int nb = a.nb;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    VT* X = reinterpret_cast<VT*>(a.X);
    VT* far_buf = reinterpret_cast<VT*>(a.far_buf);
    const int64_t ep = (int64_t)a.epoch << 32;
    __shared__ MrhsShared<VT> sh;

    if (role > 0) {
        // ---- helper: far and mid parts of blocks role-1, role-1+H, ... for all sides
        int64_t known = 0;
        for (int64_t g = role - 1; g < S.nblk; g += a.helpers) {
            // blocks finished so far.  Every time more are seen finished, an acquire
            // fence drops cached lines, so that the unknowns of finished blocks can
            // be read with plain (wide) loads
            {
                const int64_t v = rfl64(__hip_atomic_load(a.progress, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) - ep;
                if (v > known && v <= S.nblk) {
                    known = v;
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
            }
            VT acc[MAXB];
#pragma unroll
            for (int b = 0; b < MAXB; ++b) acc[b] = czero<VT>();
            bool ok = true;
            for (int list = 0; list < 2 && ok; ++list) {
                const int64_t* off = list == 0 ? S.far_off : S.mid_off;
                const int32_t* cl = list == 0 ? S.far_col : S.mid_col;
                const VT* vl = list == 0 ? S.far_val : S.mid_val;
                const int64_t s1 = off[g + 1];
                for (int64_t c0 = off[g] + (int64_t)wave * 2; c0 < s1; c0 += (int64_t)MAXB * 2) {
                    const int cnt = (int)(s1 - c0 < 2 ? s1 - c0 : 2);
                    // newest block read by the chunk: far slots carry it, mid slots read block g-2
                    int64_t needmax = 0;
                    if (list == 0) {
                        for (int j = 0; j < cnt; ++j)
                            needmax = needmax > S.far_need[c0 + j] ? needmax : (int64_t)S.far_need[c0 + j];
                    } else {
                        needmax = g - 2;
                    }
                    if (needmax + 1 > known) {
                        const int64_t v = rfl64(wait_ge64(a.progress, ep + needmax + 1, a.abort_flag));
                        if (v < 0) { ok = false; break; }
                        known = v - ep;
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    }
                    int32_t cc[2];
                    VT vv[2];
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        if (j < cnt) {
                            cc[j] = cl[(c0 + j) * 64 + lane];
                            vv[j] = vl[(c0 + j) * 64 + lane];
                        }
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        if (j >= cnt) continue;
                        const int64_t c = cc[j];
                        const VT* px = X + c * nb;
                        VT xv[MAXB];
#pragma unroll
                        for (int b = 0; b < MAXB; ++b)
                            if (b < nb) xv[b] = px[b];
#pragma unroll
                        for (int b = 0; b < MAXB; ++b)
                            if (b < nb) cfma(acc[b], vv[j], xv[b]);
                    }
                }
            }
#pragma unroll
            for (int b = 0; b < MAXB; ++b) sh.hp.part[wave][b][lane] = acc[b];
            if (mrhs_block_or<VT>(!ok, sh.orbuf)) return;
            // wave w < nb sums side w over the waves
            if (wave < nb) {
                VT t = sh.hp.part[0][wave][lane];
#pragma unroll
                for (int w = 1; w < MAXB; ++w) t = cadd(t, sh.hp.part[w][wave][lane]);
                st_wt(far_buf + (g * nb + wave) * 64 + lane, t);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (threadIdx.x == 0) __hip_atomic_store(a.fdone + g, (int32_t)a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }

    // ---- critical workgroup: wave w solves side w
    const bool mine = wave < nb;
    const bool act = mine && (!active || active[wave]);
    const VT* y = rhs + (int64_t)(mine ? wave : 0) * n;
    VT* x = out + (int64_t)(mine ? wave : 0) * n;
    constexpr int TPER = (TRI_N + MT - 1) / MT;
    constexpr int NPER = (NEAR_PF * 64 + MT - 1) / MT;
    static_assert(TPER == 4 && NPER == 8, "register staging is written out for 4 + 8 entries per thread");
    // registers: the next block's triangle and near list (named, so that they
    // stay in registers across the loop)
    VT tv0, tv1, tv2, tv3;
    VT nv0, nv1, nv2, nv3, nv4, nv5, nv6, nv7;
    int32_t nc0 = 0, nc1 = 0, nc2 = 0, nc3 = 0, nc4 = 0, nc5 = 0, nc6 = 0, nc7 = 0;
#define MRHS_FT(j) { const int t = threadIdx.x + (j) * MT; if (t < TRI_N) tv##j = S.dg[gb * TRI_N + t]; }
#define MRHS_FN(j) { const int t = threadIdx.x + (j) * MT; const int64_t sl = n0 + t / 64; \
                     if (sl < n1) { nc##j = S.near_col[sl * 64 + (t & 63)]; nv##j = S.near_val[sl * 64 + (t & 63)]; } }
#define MRHS_ST(j) { const int t = threadIdx.x + (j) * MT; if (t < TRI_N) sh.cw.tri[buf][t] = tv##j; }
#define MRHS_SN(j) { const int t = threadIdx.x + (j) * MT; if (n0 + t / 64 < n1) { \
                     sh.cw.near_c[t / 64][t & 63] = (uint8_t)(nc##j & 63); sh.cw.near_v[t / 64][t & 63] = nv##j; } }
#define MRHS_FETCH(GB) { const int64_t gb = (GB); \
        MRHS_FT(0) MRHS_FT(1) MRHS_FT(2) MRHS_FT(3) \
        const int64_t n0 = S.near_off[gb], n1 = S.near_off[gb + 1]; \
        MRHS_FN(0) MRHS_FN(1) MRHS_FN(2) MRHS_FN(3) MRHS_FN(4) MRHS_FN(5) MRHS_FN(6) MRHS_FN(7) }
    tv0 = tv1 = tv2 = tv3 = czero<VT>();
    nv0 = nv1 = nv2 = nv3 = nv4 = nv5 = nv6 = nv7 = czero<VT>();
    if (threadIdx.x == 0) {
        sh.fail = 0;
        sh.cw.tri[0][TRI_N] = czero<VT>();
        sh.cw.tri[1][TRI_N] = czero<VT>();
        __hip_atomic_store(a.progress, ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    unsigned long long t_wait = 0, t_all = 0;
    if (a.tstat && threadIdx.x == 0) t_all = wall_clock64();
    // right-hand side (with the pivot scaling) of the next block, prefetched
    VT yn = czero<VT>(), dn = czero<VT>();
#define MRHS_FETCH_Y(GB) if (mine) { const int64_t rw = (GB) * 64 + lane; \
        if (rw < n) { yn = y[S.rev ? (n - 1 - rw) : rw]; if (S.dinv) dn = S.dinv[rw]; } }
    MRHS_FETCH(0)
    MRHS_FETCH_Y(0)
    for (int64_t g = 0; g < S.nblk; ++g) {
        const int buf = (int)(g & 1);
        {   // stage block g from the registers into LDS
            MRHS_ST(0) MRHS_ST(1) MRHS_ST(2) MRHS_ST(3)
            const int64_t n0 = S.near_off[g], n1 = S.near_off[g + 1];
            MRHS_SN(0) MRHS_SN(1) MRHS_SN(2) MRHS_SN(3) MRHS_SN(4) MRHS_SN(5) MRHS_SN(6) MRHS_SN(7)
        }
        __syncthreads();
        // this block's right-hand side, then the next block's loads in flight
        const int64_t row = g * 64 + lane;
        const bool valid = row < n;
        const int64_t mi = S.rev ? (n - 1 - row) : row;
        VT r = czero<VT>();
        if (mine && valid) r = S.dinv ? cmul(yn, dn) : yn;
        if (g + 1 < S.nblk) {
            MRHS_FETCH(g + 1)
            MRHS_FETCH_Y(g + 1)
        }
        // near part (block g-1, from the ring) while the helpers finish block g
        if (mine) {
            const int64_t n0 = S.near_off[g], n1 = S.near_off[g + 1];
            const int64_t nl = n1 - n0 < NEAR_PF ? n1 - n0 : NEAR_PF;
            const int base = (int)(((g - 1) * 64) & (RING - 1));
            VT acc = czero<VT>();
            for (int64_t k = 0; k < nl; ++k)
                cfma(acc, sh.cw.near_v[k][lane], sh.cw.ring[(base + sh.cw.near_c[k][lane]) & (RING - 1)][wave]);
            // rows with more near entries than staged: the rest from memory
            for (int64_t k = n0 + NEAR_PF; k < n1; ++k) {
                const int32_t c = S.near_col[k * 64 + lane];
                cfma(acc, S.near_val[k * 64 + lane], sh.cw.ring[c & (RING - 1)][wave]);
            }
            r = csub(r, acc);
        }
        unsigned long long tw0 = 0;
        if (a.tstat && threadIdx.x == 0) tw0 = wall_clock64();
        if (threadIdx.x == 0 && !wait_eq32(a.fdone + g, (int32_t)a.epoch, a.abort_flag)) sh.fail = 1;
        if (a.tstat && threadIdx.x == 0) t_wait += wall_clock64() - tw0;
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(sh.fail)) return;
        if (mine) {
            r = csub(r, ld_coh(far_buf + (g * nb + wave) * 64 + lane));
            r = sweep(r, sh.cw.tri[buf], lane);
            sh.cw.ring[(g * 64 + lane) & (RING - 1)][wave] = r;
            if (valid) {
                st_wt(X + row * nb + wave, r);
                if (act) x[mi] = r;
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_store(a.progress, ep + g + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (a.tstat && threadIdx.x == 0) {
        a.tstat[0] = t_wait;
        a.tstat[1] = wall_clock64() - t_all;
    }
}
#undef MRHS_FT
#undef MRHS_FN
#undef MRHS_ST
#undef MRHS_SN
#undef MRHS_FETCH
#undef MRHS_FETCH_Y

// ---------------------------------------------------------------- launch

// Algorithmic bytes of one triangular solve over the active items: values and
// column indices of the factor, right-hand side read, solution written, and
// the pivot scaling where present.
static double trsv_bytes(const om_ilu* M, int kind, size_t s, const int32_t* act_host) {
    double b = 0.0;
    for (int i = 0; i < M->batch; ++i) {
        if (act_host && !act_host[i]) continue;
        const TriSched& S = M->sched[(size_t)(M->shared ? 0 : i) * 4 + kind];
        b += (double)S.nnz * (double)(s + 4) + 2.0 * (double)S.n * (double)s + (S.has_dinv ? (double)S.n * s : 0.0);
    }
    return b;
}

static bool use_chain() {
    const char* e = getenv("OMSS_TRSV");
    return e && e[0] == 'c' && e[1] == 'h';   // "chain" forces the single-workgroup kernel
}

// Several right-hand sides with the shared factor of M: the factor is read
// once per solve.  Returns OM_EINVAL (nothing launched) when it does not apply.
template <typename VT>
static om_status launch_mrhs(om_ilu* M, const TriView<VT>* views, int kind, const VT* rhs, VT* out,
                             const int32_t* active, const int32_t* act_host, hipStream_t s) {
    const int B = M->batch;
    if (!M->shared || B < 2 || B > MAXB || use_chain()) return OM_EINVAL;
    // opt-in (OMSS_TRSV_MRHS=1): one critical path for all sides is slower than
    // one per side on separate CUs while the solve is latency-bound
    const char* me = getenv("OMSS_TRSV_MRHS");
    if (!me || me[0] != '1') return OM_EINVAL;
    static int maxgrid[2] = {0, 0};
    int& mg = maxgrid[sizeof(VT) == sizeof(double2)];
    if (mg == 0) {
        int dev = 0, cus = 0, per = 0, coop = 0;
        OM_HIP(hipGetDevice(&dev));
        OM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        OM_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
        OM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, trsv_mrhs_kernel<VT>, MT, 0));
        mg = coop && per > 0 ? cus * per : -1;
    }
    if (mg < 2) return OM_EINVAL;
    const TriSched& T = M->sched[kind];
    const int64_t n = M->n, nblk = T.nblk;
    TrsvScratch& X = M->scratch;
    if (X.m_x.n < (size_t)n * B || X.m_far.n < (size_t)nblk * B * 64 || X.m_fdone.n < (size_t)nblk) {
        OM_TRY(X.m_x.alloc((size_t)n * B));
        OM_TRY(X.m_far.alloc((size_t)nblk * B * 64));
        OM_TRY(X.m_fdone.alloc((size_t)nblk));
        OM_TRY(X.m_progress.alloc(1));
        OM_HIP(hipMemsetAsync(X.m_fdone.p, 0, X.m_fdone.bytes(), s));
        OM_HIP(hipMemsetAsync(X.m_progress.p, 0, X.m_progress.bytes(), s));
        OM_HIP(hipStreamSynchronize(s));
    }
    int H = (int)std::min<int64_t>(mg - 1, nblk);
    if (const char* e = getenv("OMSS_TRSV_HELPERS")) H = std::max(1, std::min(H, atoi(e)));
    MrhsArgs a;
    a.X = X.m_x.p;
    a.far_buf = X.m_far.p;
    a.fdone = X.m_fdone.p;
    a.progress = X.m_progress.p;
    a.abort_flag = X.abort_flag.p;
    a.epoch = ++X.epoch;
    if (a.epoch == 0) a.epoch = ++X.epoch;
    a.helpers = H;
    a.nb = B;
    static unsigned long long* tst = nullptr;
    a.tstat = nullptr;
    if (getenv("OMSS_TRSV_STATS")) {
        if (!tst) OM_HIP(hipMalloc((void**)&tst, 2 * sizeof(unsigned long long)));
        a.tstat = tst;
    }
    int nact = B;
    if (act_host) {
        nact = 0;
        for (int i = 0; i < B; ++i) nact += act_host[i] != 0;
    }
    const double bytes = (double)T.nnz * (double)(sizeof(VT) + 4) +
                         (double)nact * (2.0 * (double)n * sizeof(VT) + (T.has_dinv ? (double)n * sizeof(VT) : 0.0));
    ProfScope prof("trsv", s, profile_enabled() ? bytes : 0.0);
    void* args[] = {(void*)&views, (void*)&kind, (void*)&rhs, (void*)&out, (void*)&n, (void*)&active, (void*)&a};
    OM_HIP(hipLaunchCooperativeKernel((const void*)trsv_mrhs_kernel<VT>, dim3(1 + H), dim3(MT), args, 0, s));
    if (a.tstat) {
        unsigned long long h[2];
        OM_HIP(hipMemcpyAsync(h, a.tstat, sizeof h, hipMemcpyDeviceToHost, s));
        OM_HIP(hipStreamSynchronize(s));
        fprintf(stderr, "[trsv stats] multi-side kind %d, %d sides, H=%d: %lld blocks, critical workgroup %.3f ms, "
                "of which waiting for helpers %.3f ms\n", kind, B, H, (long long)nblk, h[1] / 1e5, h[0] / 1e5);
    }
    return OM_OK;
}

template <typename VT>
static om_status launch_trsv(om_ilu* M, const TriView<VT>* views, int kind, const VT* rhs, VT* out,
                             const int32_t* active, const int32_t* act_host, hipStream_t s) {
    {
        const om_status r = launch_mrhs<VT>(M, views, kind, rhs, out, active, act_host, s);
        if (r != OM_EINVAL) return r;
    }
    ProfScope prof("trsv", s, profile_enabled() ? trsv_bytes(M, kind, sizeof(VT), act_host) : 0.0);
    const int B = M->batch;
    if (!use_chain()) {
        static int maxgrid[2] = {0, 0};
        int& mg = maxgrid[sizeof(VT) == sizeof(double2)];
        if (mg == 0) {
            int dev = 0, cus = 0, per = 0, coop = 0;
            OM_HIP(hipGetDevice(&dev));
            OM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            OM_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
            OM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, trsv_coop_kernel<VT>, 64 * TW, 0));
            mg = coop ? cus * per : -1;
        }
        const int64_t nblk = (M->n + 63) / 64;
        const int slots = (B + NXCD - 1) / NXCD;             // items per XCD
        const int span = (B <= NXCD && NXCD % B == 0) ? NXCD / B : 1;   // XCDs per item
        int H = 0, per_xcd = 0;
        if (mg > 0) {
            // default: every workgroup slot of the device (the helpers are bound
            // by the latency of their loads, so more of them stream more)
            const char* e = getenv("OMSS_TRSV_HELPERS");
            H = e ? atoi(e) : (mg / (NXCD * slots)) * span - 1;
            H = (int)std::min<int64_t>(H, nblk);
            // workgroups of an item: 1 + H over `span` XCDs; grid = 8 * per_xcd * slots
            per_xcd = (1 + H + span - 1) / span;
            const int cap = mg / (NXCD * slots);
            if (per_xcd > cap) { per_xcd = cap; H = per_xcd * span - 1; }
        }
        if (H >= 1) {
            CoopArgs a;
            a.far_buf = M->scratch.far_buf.p;
            a.fdone = M->scratch.fdone.p;
            a.progress = M->scratch.progress.p;
            a.abort_flag = M->scratch.abort_flag.p;
            a.epoch = ++M->scratch.epoch;
            if (a.epoch == 0) a.epoch = ++M->scratch.epoch;
            a.helpers = H;
            a.batch = B;
            a.per_xcd = span > 1 ? per_xcd : 1 + H;
            a.xcd_per_item = span;
            static unsigned long long* tst = nullptr;
            a.tstat = nullptr;
            if (getenv("OMSS_TRSV_STATS")) {
                if (!tst) OM_HIP(hipMalloc((void**)&tst, 6 * sizeof(unsigned long long)));
                OM_HIP(hipMemsetAsync(tst, 0, 6 * sizeof(unsigned long long), s));
                a.tstat = tst;
            }
            int64_t n = M->n;
            void* args[] = {(void*)&views, (void*)&kind, (void*)&rhs, (void*)&out, (void*)&n, (void*)&active, (void*)&a};
            const unsigned grid = span > 1 ? (unsigned)(NXCD * per_xcd) : (unsigned)(NXCD * slots * (1 + H));
            OM_HIP(hipLaunchCooperativeKernel((const void*)trsv_coop_kernel<VT>, dim3(grid), dim3(64 * TW), args, 0, s));
            if (a.tstat) {
                unsigned long long h[6];
                OM_HIP(hipMemcpyAsync(h, a.tstat, sizeof h, hipMemcpyDeviceToHost, s));
                OM_HIP(hipStreamSynchronize(s));
                fprintf(stderr, "[trsv stats] H=%d kind=%d per item (critical workgroup): near %.3f ms, publish %.3f ms, "
                        "wait for helpers %.3f ms, barrier %.3f ms, sweep %.3f ms, end barrier %.3f ms\n", H, kind,
                        h[0] / 1e5 / B, h[4] / 1e5 / B, h[1] / 1e5 / B, h[5] / 1e5 / B, h[2] / 1e5 / B, h[3] / 1e5 / B);
            }
            return OM_OK;
        }
    }
    hipLaunchKernelGGL(trsv_chain_kernel<VT>, dim3(B), dim3(64 * TW), 0, s, views, kind, rhs, out, M->n, active);
    OM_HIP(hipGetLastError());
    return OM_OK;
}

// y = (L U)^{-1} x or (L U)^{-H} x for every active batch item; x, y may alias.
om_status ilu_apply_dev(const om_ilu* Mc, int adjoint, int dtype, const void* x, void* y, const int32_t* active,
                        hipStream_t s, const int32_t* act_host) {
    om_ilu* M = const_cast<om_ilu*>(Mc);
    const int k0 = adjoint ? 2 : 0, k1 = adjoint ? 3 : 1;
    if (dtype == OM_C128) {
        OM_TRY(launch_trsv<double2>(M, M->views64.p, k0, (const double2*)x, (double2*)y, active, act_host, s));
        OM_TRY(launch_trsv<double2>(M, M->views64.p, k1, (const double2*)y, (double2*)y, active, act_host, s));
    } else {
        OM_TRY(launch_trsv<float2>(M, M->views32.p, k0, (const float2*)x, (float2*)y, active, act_host, s));
        OM_TRY(launch_trsv<float2>(M, M->views32.p, k1, (const float2*)y, (float2*)y, active, act_host, s));
    }
    return OM_OK;
}

// OM_ETIMEOUT if a bounded wait of a cooperative solve expired since the last
// check (the flag is cleared).
om_status trsv_check(const om_ilu* Mc, hipStream_t s) {
    om_ilu* M = const_cast<om_ilu*>(Mc);
    if (!M->scratch.abort_flag.p) return OM_OK;
    int32_t f = 0;
    OM_HIP(hipMemcpyAsync(&f, M->scratch.abort_flag.p, sizeof f, hipMemcpyDeviceToHost, s));
    OM_HIP(hipStreamSynchronize(s));
    if (f) {
        OM_HIP(hipMemsetAsync(M->scratch.abort_flag.p, 0, sizeof f, s));
        // an abandoned solve may leave far sums written but not consumed
        OM_HIP(hipMemsetAsync(M->scratch.far_buf.p, 0xff, M->scratch.far_buf.bytes(), s));
        OM_HIP(hipStreamSynchronize(s));
        set_error("a triangular solve timed out waiting for its helpers (abort flag set)");
        return OM_ETIMEOUT;
    }
    return OM_OK;
}

}  // namespace omss
