// Dual-threshold incomplete LU on the device, row-pipelined: the same factor
// as the host ILUT (ilut.cpp, no pivoting), bit for bit.
//
// A persistent grid of workgroups takes rows in increasing order from an
// atomic counter.  For row i the workgroup keeps a dense accumulator over the
// band window [i - lb, i + ub] (which contains every fill entry of the row)
// in global memory and a presence bitmap of the window in LDS, and:
//   1. loads row i of A, tau_i = d * ||a_i||_inf;
//   2. eliminates against U rows in increasing column: wave 0 finds the next
//      present column k left of the diagonal in the bitmap, makes sure row k
//      is finished (ready flags of 64 rows are polled at once, after an L2
//      invalidation, and remembered; waits poll with acquire loads)
//      and forms the multiplier w_k / u_kk, dropping it if |w_k| < tau_i; all
//      threads then subtract w_k * u_k from the window;
//   3. drops entries below tau_i and keeps the lfil_i largest of each
//      triangle (exact radix select on the squared moduli, ties to the lower
//      column), writes the L and U rows in column order and raises row i's
//      ready flag.
// Rows are handed out in increasing order and wait only for smaller rows,
// which are held by running workgroups, so the grid always makes progress;
// every wait is bounded in time.  Published rows are written through to
// memory before the flag (s_waitcnt); row storage is 128-byte aligned so a
// cache line never mixes rows and readers of a flagged row may use ordinary
// loads; the pivots, kept in a dense array, are read with coherent loads.
// The first row that breaks down (non-finite pivot or kept entry) is recorded
// and ends the launch.  Floating-point contraction is disabled so that every
// operation matches the host code.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "common.hpp"
#include "ilu.hpp"
#include "ilut.hpp"
#include "kernels.hpp"
#include "profile.hpp"

#pragma clang fp contract(off)

namespace omss {

constexpr int IT = 256;             // threads per workgroup
constexpr int IWAVES = IT / 64;
constexpr int WBITS_MAX = 1 << 16;  // largest band window (lb + ub + 1)
constexpr int RADIX_BITS = 11;
constexpr int FLAG_STRIDE = 32;
constexpr int UF = 4;               // U-row entries per thread in flight in an update
constexpr int WB = 16;              // window positions per thread in flight in the unstaged dropping
constexpr int RADIX = 1 << RADIX_BITS;

struct IlutDevArgs {
    int64_t n;
    int32_t lb, ub, W;
    int64_t wstride;        // work window stride (entries, a whole number of 128-byte lines)
    const int32_t* row_ptr;
    const int32_t* col;
    const double2* val;
    double drop_tol, fill_factor;
    int32_t capped;
    const int64_t* l_off;   // n + 1 capacity offsets (entries)
    const int64_t* u_off;
    int32_t* l_len;
    int32_t* u_len;
    int32_t* l_col;
    double2* l_val;
    int32_t* u_col;
    double2* u_val;
    double2* udiag;         // pivot u_ii per row
    int32_t* ready;         // per row, epoch tags
    uint32_t epoch;
    long long wait_ticks;   // bound of one wait, in wall-clock ticks
    int32_t* host_progress; // host-mapped: a recently published row (progress report)
    double2* work;          // gridDim * W
    int32_t* next_row;
    int32_t* abort_flag;
    unsigned long long* tstat;  // diagnostics (nullable): wall-clock ticks and counts per phase
    int32_t acq_fence;      // agent-scope acquire fence after observing finished rows
    int32_t max_pause;      // longest back-off of a wait, in units of s_sleep(1)
    int32_t cand_lim;       // largest LDS staging used (<= CAND_MAX; smaller only to exercise the other path)
    int32_t* status;        // [0] first breakdown row + 1 (0 = none), [1] repaired pivots, [38..39] U-row entries read,
                            // [2], [3] row + 1 of the waiter and of the awaited row on a timeout,
                            // [4] row + 1 that found inconsistent row data
};

__device__ inline void wt_store(double2* p, double2 v) {
    double* q = reinterpret_cast<double*>(p);
    __hip_atomic_store(q, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(q + 1, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void wt_store(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline double2 ld_coh(const double2* p) {
    const double* q = reinterpret_cast<const double*>(p);
    return make_double2(__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                        __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

__device__ inline int32_t ld_flag(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Flags that cross workgroups.  Each row's flag has a cache line of its own,
// so that waiters on different rows poll different lines and no flag shares
// a line with another row's; waits back off exponentially and look at the
// abort flag rarely: hundreds of waves polling a few lines without pause
// saturate the memory channel behind them and stall every access routed
// there, including the stores of the rows being waited for.
__device__ inline void publish_flag(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until *f == v; false on abort or when the time bound passes (which
// raises the abort flag and records the waiting and the awaited row).  The
// abort flag, read by every waiter, is polled only every 16th round, with a
// growing pause between polls, to keep the flag lines from becoming hot spots.
__device__ bool wait_flag(int32_t* f, int32_t v, int32_t* abort_flag, long long ticks, int32_t* diag,
                          int64_t waiter, int64_t awaited, unsigned int max_pause) {
    const long long t0 = wall_clock64();
    unsigned int pause = 1;
    for (unsigned int it = 0; ld_flag(f) != v; ++it) {
        if ((it & 63u) == 63u) {
            if (ld_flag(abort_flag)) return false;
            if (wall_clock64() - t0 > ticks) {
                if (atomicCAS(diag, 0, (int32_t)(waiter + 1)) == 0)
                    __hip_atomic_store(diag + 1, (int32_t)(awaited + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                publish_flag(abort_flag, 1);
                return false;
            }
        }
        // exponential back-off from 64 cycles up to 64 * max_pause
        for (unsigned int q = 0; q < pause; ++q) __builtin_amdgcn_s_sleep(1);
        if (pause < max_pause) pause <<= 1;
    }
    return true;
}

__device__ inline unsigned long long key_of(double m2) { return (unsigned long long)__double_as_longlong(m2); }

// Block-wide inclusive prefix sum of one int per thread; returns the exclusive
// prefix, *total receives the sum.
__device__ inline int block_scan(int v, int* total, int* sbuf) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) sbuf[wave] = x;
    __syncthreads();
    int base = 0, tot = 0;
    for (int w = 0; w < IWAVES; ++w) {
        if (w < wave) base += sbuf[w];
        tot += sbuf[w];
    }
    __syncthreads();
    *total = __builtin_amdgcn_readfirstlane(tot);
    return base + x - v;
}

// Block-wide OR of one predicate per thread; the result is wave-uniform.
__device__ inline int block_or(bool v, int* sor) {
    const unsigned long long b = __ballot(v);
    if ((threadIdx.x & 63) == 0) sor[threadIdx.x >> 6] = b != 0ull;
    __syncthreads();
    int r = 0;
    for (int w = 0; w < IWAVES; ++w) r |= sor[w];
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(r);
}

// Radix select over the candidate keys of one triangle: returns the key K of
// the lfil-th largest and, in *n_gt, how many keys exceed K, with *capped
// true; with at most lfil candidates (counted by the first pass) it returns
// at once with *capped false.  Requires lfil >= 1.  sbuf: 8 ints.
__device__ unsigned long long select_kth(const double2* w, const uint32_t* bits, int p0, int p1, double tau2, int lfil,
                                         int* n_gt, unsigned int* hist, int* sbuf, bool* capped) {
    unsigned long long prefix = 0, pmask = 0;
    int need = lfil;   // rank (1-based) of the wanted key among those matching the prefix, from the top
    int above = 0;     // keys strictly greater than the prefix range, counted so far
    for (int shift = 64 - RADIX_BITS; shift > -RADIX_BITS; shift -= RADIX_BITS) {
        const int sh = shift < 0 ? 0 : shift;
        const int nb = shift < 0 ? RADIX_BITS + shift : RADIX_BITS;
        const unsigned int dmask = (1u << nb) - 1u;
        for (int t = threadIdx.x; t < RADIX; t += IT) hist[t] = 0;
        __syncthreads();
        // WB positions per thread at a time, their loads issued together
        for (int pb = p0 + threadIdx.x; pb < p1; pb += WB * IT) {
            double2 vb[WB];
#pragma unroll
            for (int u = 0; u < WB; ++u) vb[u] = w[min(pb + u * IT, p1 - 1)];
#pragma unroll
            for (int u = 0; u < WB; ++u) {
                const int p = pb + u * IT;
                if (p >= p1 || !((bits[p >> 5] >> (p & 31)) & 1u)) continue;
                const double m2 = vb[u].x * vb[u].x + vb[u].y * vb[u].y;
                if (m2 == 0.0 || m2 < tau2) continue;
                const unsigned long long k = key_of(m2);
                if ((k & pmask) != prefix) continue;
                atomicAdd(&hist[(unsigned int)(k >> sh) & dmask], 1u);
            }
        }
        __syncthreads();
        // thread t owns the digits dmask - 8t - j, j = 0..7 (descending); the
        // counts above its range come from a block-wide scan
        int own = 0;
        int cnt[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int d = (int)dmask - 8 * threadIdx.x - j;
            cnt[j] = d >= 0 ? (int)hist[d] : 0;
            own += cnt[j];
        }
        int tot;
        const int before = block_scan(own, &tot, sbuf + 2);
        // the first pass counts every candidate: at most lfil means no cap
        if (shift == 64 - RADIX_BITS) {
            *capped = tot > lfil;
            if (!*capped) return 0ull;
        }
        if (before < need && need <= before + own) {
            int acc = before;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (acc + cnt[j] >= need) {
                    sbuf[0] = (int)dmask - 8 * threadIdx.x - j;
                    sbuf[1] = acc;
                    break;
                }
                acc += cnt[j];
            }
        }
        __syncthreads();
        const int d = __builtin_amdgcn_readfirstlane(sbuf[0]);
        const int acc = __builtin_amdgcn_readfirstlane(sbuf[1]);
        const int in_d = __builtin_amdgcn_readfirstlane((int)hist[d]);
        __syncthreads();
        above += acc;
        need -= acc;
        prefix |= ((unsigned long long)d) << sh;
        pmask |= ((unsigned long long)dmask) << sh;
        if (need == in_d && prefix != 0ull) {
            // every key of the chosen digit range is kept (as in select_kth_lds)
            *n_gt = lfil;
            return prefix - 1ull;
        }
    }
    *n_gt = above;
    return prefix;
}

// Sum over the block of one int per thread (wave-uniform result).
__device__ inline int block_sum(int v, int* sbuf) {
    int tot;
    (void)block_scan(v, &tot, sbuf);
    return tot;
}

// Radix select over keys held in LDS (0 = not a candidate): the key K of the
// lfil-th largest and, in *n_gt, how many keys exceed K.  Same digits and
// tie rule as select_kth.  Requires 1 <= lfil < number of candidates.
__device__ unsigned long long select_kth_lds(const unsigned long long* key, int cnt, int lfil, int* n_gt,
                                             unsigned int* hist, int* sbuf) {
    unsigned long long prefix = 0, pmask = 0;
    int need = lfil, above = 0;
    for (int shift = 64 - RADIX_BITS; shift > -RADIX_BITS; shift -= RADIX_BITS) {
        const int sh = shift < 0 ? 0 : shift;
        const int nb = shift < 0 ? RADIX_BITS + shift : RADIX_BITS;
        const unsigned int dmask = (1u << nb) - 1u;
        for (int t = threadIdx.x; t < RADIX; t += IT) hist[t] = 0;
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += IT) {
            const unsigned long long k = key[t];
            if (k == 0ull || (k & pmask) != prefix) continue;
            atomicAdd(&hist[(unsigned int)(k >> sh) & dmask], 1u);
        }
        __syncthreads();
        int own = 0;
        int c8[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int d = (int)dmask - 8 * threadIdx.x - j;
            c8[j] = d >= 0 ? (int)hist[d] : 0;
            own += c8[j];
        }
        int tot;
        const int before = block_scan(own, &tot, sbuf + 2);
        if (before < need && need <= before + own) {
            int acc = before;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (acc + c8[j] >= need) {
                    sbuf[0] = (int)dmask - 8 * threadIdx.x - j;
                    sbuf[1] = acc;
                    break;
                }
                acc += c8[j];
            }
        }
        __syncthreads();
        const int d = __builtin_amdgcn_readfirstlane(sbuf[0]);
        const int acc = __builtin_amdgcn_readfirstlane(sbuf[1]);
        const int in_d = __builtin_amdgcn_readfirstlane((int)hist[d]);
        __syncthreads();
        above += acc;
        need -= acc;
        prefix |= ((unsigned long long)d) << sh;
        pmask |= ((unsigned long long)dmask) << sh;
        if (need == in_d && prefix != 0ull) {
            // every key of the chosen digit range is kept: the lfil largest are
            // exactly the keys >= prefix, so K = prefix - 1 with lfil keys above
            // it selects them and leaves no tie to take
            *n_gt = lfil;
            return prefix - 1ull;
        }
    }
    *n_gt = above;
    return prefix;
}

constexpr int CAND_MAX = 6144;   // entries of one triangle staged in LDS for the cap

constexpr int RPT = 8;          // candidate rounds per group (strided by the block size): all of CAND_MAX

// While a row is eliminated, the staging arrays hold the part of the dense
// working row around the diagonal (WIN_N positions, the most updated ones):
// its read-modify-writes stay in LDS instead of going to memory.
constexpr int WIN_N = 3840;

struct SideShared {
    alignas(16) unsigned long long key[CAND_MAX];
    uint16_t pos[CAND_MAX];
    int cnt[RPT][IWAVES];        // per round and wave: flags set (scans in candidate order)
    unsigned long long tph[12];  // diagnostics (thread 0): [0..3] ticks in positions, keys, select, output;
                                 // [4] staged calls, [6] calls reading the window, [11] capped staged calls
    int on;                      // diagnostics enabled
};

// Rank of each thread's flagged candidates in candidate order, candidate
// u * IT + tid being flag f[u]: returns in r[u] the number of flagged
// candidates before it and the total in *total.  Wave ballots, one barrier.
__device__ inline void strided_rank(const bool (&f)[RPT], int (&r)[RPT], int* total, SideShared& ss) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long m[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        m[u] = __ballot(f[u]);
        if (lane == 0) ss.cnt[u][wave] = __popcll(m[u]);
    }
    __syncthreads();
    int base = 0;
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        int before_w = 0, row = 0;
#pragma unroll
        for (int q = 0; q < IWAVES; ++q) {
            const int c = ss.cnt[u][q];
            before_w += q < wave ? c : 0;
            row += c;
        }
        const unsigned long long below = lane ? (m[u] & (~0ull >> (64 - lane))) : 0ull;
        r[u] = base + before_w + __popcll(below);
        base += row;
    }
    *total = __builtin_amdgcn_readfirstlane(base);
    __syncthreads();   // cnt is reused by the next call
}

// Dropping and cap of one triangle of row i, window positions [p0, p1), and
// output of the kept entries in column order to (ocol, oval); returns how
// many were kept, and sets *bad when check_finite and a kept entry is not
// finite.  The present positions and the keys (squared moduli; 0 = dropped)
// are staged in LDS once, so the window is read twice (keys, output) however
// many digit passes the cap takes; a triangle with more than CAND_MAX present
// entries reads its keys from the window in every pass instead.
__device__ int output_side(const double2* w, const uint32_t* bits, int p0, int p1, int64_t lo, double tau2, int lfil,
                           int32_t* ocol, double2* oval, bool check_finite, bool* bad, SideShared& ss,
                           unsigned int* hist, int* sbuf, int cand_lim) {
    const int tid = threadIdx.x;
    // present positions per thread over a contiguous range of bitmap words
    const int wlo = p0 >> 5, whi = p1 > p0 ? ((p1 - 1) >> 5) + 1 : wlo;
    const int nw = whi - wlo, wch = (nw + IT - 1) / IT;
    const int q0 = wlo + tid * wch, q1 = min(whi, q0 + wch);
    auto word_at = [&](int q) -> uint32_t {
        uint32_t x = bits[q];
        const int b = q * 32;
        if (p0 > b) x &= p0 - b >= 32 ? 0u : (~0u << (p0 - b));
        if (p1 < b + 32) x &= p1 - b <= 0 ? 0u : (~0u >> (32 - (p1 - b)));
        return x;
    };
    unsigned long long tt = (ss.on && tid == 0) ? wall_clock64() : 0;
    auto phase = [&](int k) {
        if (ss.on && tid == 0) { const unsigned long long t = wall_clock64(); ss.tph[k] += t - tt; tt = t; }
    };
    int mine = 0;
    for (int q = q0; q < q1; ++q) mine += __popc(word_at(q));
    int present;
    const int off = block_scan(mine, &present, sbuf);
    if (present <= cand_lim) {
        {
            int j = off;
            for (int q = q0; q < q1; ++q) {
                uint32_t x = word_at(q);
                while (x) {
                    const int b = __ffs((int)x) - 1;
                    x &= x - 1u;
                    ss.pos[j++] = (uint16_t)(q * 32 + b);
                }
            }
        }
        __syncthreads();
        phase(0);
        // candidate t is handled by thread t % IT in round t / IT, so that the
        // lanes of a wave touch consecutive LDS words and window entries;
        // rounds go in groups of RPT
        const int rounds = (present + IT - 1) / IT, groups = (rounds + RPT - 1) / RPT;
        // groups of RPT rounds; the loads of the next group are in flight while
        // a group is processed (at most 3 groups: CAND_MAX = 3 * RPT * IT)
        static_assert(CAND_MAX <= 3 * RPT * IT, "staging groups");
        int live = 0;
        auto load_group = [&](double2 (&v)[RPT], int gq) {
#pragma unroll
            for (int u = 0; u < RPT; ++u) {
                const int t = (gq * RPT + u) * IT + tid;
                if (t < present) v[u] = w[ss.pos[t]];
            }
        };
        auto key_group = [&](const double2 (&v)[RPT], int gq) {
#pragma unroll
            for (int u = 0; u < RPT; ++u) {
                const int t = (gq * RPT + u) * IT + tid;
                if (t < present) {
                    const double m2 = v[u].x * v[u].x + v[u].y * v[u].y;
                    const bool cand = !(m2 == 0.0 || m2 < tau2);
                    ss.key[t] = cand ? key_of(m2) : 0ull;
                    live += cand;
                }
            }
        };
        {
            double2 va[RPT], vb[RPT];
            load_group(va, 0);
            if (groups > 1) load_group(vb, 1);
            key_group(va, 0);
            if (groups > 2) load_group(va, 2);
            if (groups > 1) key_group(vb, 1);
            if (groups > 2) key_group(va, 2);
        }
        const int tot = block_sum(live, sbuf);   // (its barriers also order the key writes)
        phase(1);
        const bool cap = tot > lfil;
        if (ss.on && tid == 0) ss.tph[11] += cap;
        unsigned long long thr = 0ull;   // a candidate is kept when its key exceeds thr (dropped keys are 0)
        if (cap) {
            int n_gt = 0;
            // lfil = 0 keeps nothing: K above every key, no ties taken
            const unsigned long long K = lfil > 0 ? select_kth_lds(ss.key, present, lfil, &n_gt, hist, sbuf + 4) : ~0ull;
            phase(2);
            const int take = lfil - n_gt;
            // take = 0 (the usual case: the select ends where the lfil-th and
            // the next key fall in different digit ranges): the kept keys are
            // exactly those above K.  Otherwise the first `take` ties at K in
            // column order are kept, and the keys are replaced by the
            // decision (1 kept, 0 not).
            if (take <= 0) thr = K;
            int base = 0;
            for (int gq = 0; gq < (take > 0 ? groups : 0); ++gq) {
                bool f[RPT];
                unsigned long long kk[RPT];
#pragma unroll
                for (int u = 0; u < RPT; ++u) {
                    const int t = (gq * RPT + u) * IT + tid;
                    kk[u] = t < present ? ss.key[t] : 0ull;
                    f[u] = kk[u] != 0ull && kk[u] == K;
                }
                int r[RPT], tg;
                strided_rank(f, r, &tg, ss);
#pragma unroll
                for (int u = 0; u < RPT; ++u) {
                    const int t = (gq * RPT + u) * IT + tid;
                    if (t < present) ss.key[t] = (kk[u] != 0ull && (kk[u] > K || (f[u] && base + r[u] < take))) ? 1ull : 0ull;
                }
                base += tg;
            }
            __syncthreads();
        }
        // output: ranks of the kept candidates in column order, then the
        // loads and stores of a group (consecutive lanes, consecutive ranks)
        int base = 0;
        struct OutGroup {
            bool f[RPT];
            int pp[RPT];
            double2 v[RPT];
        };
        auto fetch_group = [&](OutGroup& o, int gq) {
#pragma unroll
            for (int u = 0; u < RPT; ++u) {
                const int t = (gq * RPT + u) * IT + tid;
                o.f[u] = t < present && ss.key[t] > thr;
                o.pp[u] = t < present ? (int)ss.pos[t] : 0;
            }
#pragma unroll
            for (int u = 0; u < RPT; ++u)
                if (o.f[u]) o.v[u] = w[o.pp[u]];
        };
        auto store_group = [&](const OutGroup& o) {
            int r[RPT], tg;
            strided_rank(o.f, r, &tg, ss);
#pragma unroll
            for (int u = 0; u < RPT; ++u)
                if (o.f[u]) {
                    if (check_finite && (!isfinite(o.v[u].x) || !isfinite(o.v[u].y))) *bad = true;
                    ocol[base + r[u]] = (int32_t)(lo + o.pp[u]);
                    oval[base + r[u]] = o.v[u];
                }
            base += tg;
        };
        {
            OutGroup oa, ob;
            fetch_group(oa, 0);
            if (groups > 1) fetch_group(ob, 1);
            store_group(oa);
            if (groups > 2) fetch_group(oa, 2);
            if (groups > 1) store_group(ob);
            if (groups > 2) store_group(oa);
        }
        phase(3);
        if (ss.on && tid == 0) ++ss.tph[4];
        return base;
    }
    // more present entries than the staging arrays hold: keys from the window
    if (ss.on && tid == 0) ++ss.tph[6];
    // the select counts the candidates in its first pass (cap or not); lfil = 0
    // keeps nothing: K above every key, no ties taken
    bool cap = true;
    unsigned long long K = ~0ull;
    int n_gt = 0;
    if (lfil > 0) K = select_kth(w, bits, p0, p1, tau2, lfil, &n_gt, hist, sbuf + 4, &cap);
    const int chunk = (p1 - p0 + IT - 1) / IT;
    const int c0 = p0 + tid * chunk, c1 = min(p1, c0 + chunk);
    int keep = 0, eq = 0;
    for (int pb = c0; pb < c1; pb += WB) {
        double2 vb[WB];
#pragma unroll
        for (int u = 0; u < WB; ++u) vb[u] = w[min(pb + u, c1 - 1)];
#pragma unroll
        for (int u = 0; u < WB; ++u) {
            const int pp = pb + u;
            if (pp >= c1 || !((bits[pp >> 5] >> (pp & 31)) & 1u)) continue;
            const double m2 = vb[u].x * vb[u].x + vb[u].y * vb[u].y;
            if (m2 == 0.0 || m2 < tau2) continue;
            const unsigned long long key = key_of(m2);
            if (!cap || key > K) ++keep; else if (key == K) ++eq;
        }
    }
    int tmp;
    const int eq_before = block_scan(eq, &tmp, sbuf);
    const int take = cap ? max(0, min(eq, lfil - n_gt - eq_before)) : 0;
    int total = 0;
    const int out = block_scan(keep + take, &total, sbuf);
    int written = 0, e = 0;
    for (int pb = c0; pb < c1; pb += WB) {
        double2 vb[WB];
#pragma unroll
        for (int u = 0; u < WB; ++u) vb[u] = w[min(pb + u, c1 - 1)];
#pragma unroll
        for (int u = 0; u < WB; ++u) {
            const int pp = pb + u;
            if (pp >= c1 || !((bits[pp >> 5] >> (pp & 31)) & 1u)) continue;
            const double2 v = vb[u];
            const double m2 = v.x * v.x + v.y * v.y;
            if (m2 == 0.0 || m2 < tau2) continue;
            const unsigned long long key = key_of(m2);
            bool kp = !cap || key > K;
            if (cap && key == K) kp = e++ < take;
            if (kp) {
                if (check_finite && (!isfinite(v.x) || !isfinite(v.y))) *bad = true;
                ocol[out + written] = (int32_t)(lo + pp);
                oval[out + written] = v;
                ++written;
            }
        }
    }
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(IT, 2) void ilut_row_kernel(IlutDevArgs a) {
    __shared__ uint32_t bits[WBITS_MAX / 32];
    __shared__ unsigned int hist[RADIX];
    __shared__ int sbuf[16];
    __shared__ double sred[IWAVES];
    __shared__ int s_row, s_stop, s_or[IWAVES];
    __shared__ int s_k[2], s_flag[2], s_ulen[2];
    __shared__ int64_t s_uoff[2];
    __shared__ double2 s_m[2];
    __shared__ SideShared side;
    // Every loop below is controlled by wave-uniform values (read with
    // readfirstlane from shared memory) and has no early exit; per-lane work
    // (lane 0 fetching the next row, publishing a row) sits between two
    // barriers, never at a loop head or latch.  Otherwise the compiler may let
    // the lanes of one wave take different trips through a loop that contains
    // barriers, and the waves of a block drift apart.
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int W = a.W, nwords = (W + 31) >> 5;
    double2* w = a.work + (int64_t)blockIdx.x * a.wstride;
    static_assert(WIN_N * sizeof(double2) <= CAND_MAX * (sizeof(unsigned long long) + sizeof(uint16_t)),
                  "window cache larger than the staging arrays");
    double2* swin = reinterpret_cast<double2*>(side.key);
    const int cbase = a.lb - WIN_N / 2;   // window position held at swin[0]
    auto wget = [&](int p) -> double2 {
        const unsigned q = (unsigned)(p - cbase);
        return q < (unsigned)WIN_N ? swin[q] : w[p];
    };
    auto wput = [&](int p, double2 v) {
        const unsigned q = (unsigned)(p - cbase);
        if (q < (unsigned)WIN_N) swin[q] = v;
        else w[p] = v;
    };

    // diagnostics (thread 0): ticks in the pivot steps of wave 0, in waits
    // for unfinished rows, in updates and in the dropping and output; counts
    // of rows, steps, updating steps and updated entries
    unsigned long long st_piv = 0, st_wait = 0, st_upd = 0, st_fin = 0, st_rows = 0, st_steps = 0, st_usteps = 0,
                       st_ent = 0, st_finu = 0, st_pub = 0, tq = 0;
    unsigned long long n_upd = 0;   // U-row entries read by this workgroup's eliminations (thread 0)
    if (tid == 0) {
        side.on = a.tstat != nullptr;
        for (int k = 0; k < 12; ++k) side.tph[k] = 0;
    }
    if (tid == 0) {
        s_row = atomicAdd(a.next_row, 1);
        s_stop = ld_flag(a.abort_flag);
    }
    __syncthreads();
    int64_t i = __builtin_amdgcn_readfirstlane(s_row);
    int stop = __builtin_amdgcn_readfirstlane(s_stop);

    while (i < a.n && !stop) {
        for (int q = tid; q < nwords; q += IT) bits[q] = 0u;
        __syncthreads();
        const int64_t lo = i - a.lb;
        // 1. row i of A
        const int32_t r0 = a.row_ptr[i], r1 = a.row_ptr[i + 1];
        double mx = 0.0;
        for (int32_t t = r0 + tid; t < r1; t += IT) {
            const int p = (int)(a.col[t] - lo);
            const double2 v = a.val[t];
            wput(p, v);
            atomicOr(&bits[p >> 5], 1u << (p & 31));
            const double m = sqrt(v.x * v.x + v.y * v.y);
            mx = m > mx ? m : mx;
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_down(mx, off, 64);
            mx = o > mx ? o : mx;
        }
        if (lane == 0) sred[wave] = mx;
        __syncthreads();
        double rowinf = 0.0;
        for (int q = 0; q < IWAVES; ++q) rowinf = sred[q] > rowinf ? sred[q] : rowinf;
        const double tau = a.drop_tol * rowinf;
        const double tau2 = tau * tau;
        const int64_t nnz_row = r1 - r0;
        const int lfil = a.capped ? (int)fmax(0.0, floor((a.fill_factor * (double)nnz_row - 1.0) / 2.0)) : 0x7fffffff;
        const int dpos = a.lb;   // window position of the diagonal

        // 2. elimination.  Wave 0 decides each step (next column, readiness,
        // multiplier) and publishes it in a parity-indexed slot; the other waves
        // read the slot after the barrier, so two steps never share one.
        int kprev = -1;
        bool badrow = false;   // a U-row column outside the window was met
        int64_t rlo = -(1ll << 40);     // wave 0: rows rlo..rlo+63 whose flags are cached in rmask
        unsigned long long rmask = 0ull;
        int par = 0;
        int going = 1;
        while (going) {
            if (a.tstat && tid == 0) tq = wall_clock64();
            if (wave == 0) {
                // Settle the present columns left of the diagonal in order.  The
                // columns of one bitmap word whose rows are finished are decided
                // together (lane = bit): entry, pivot and row data in one round of
                // loads per lane; multipliers below tau are dropped, which changes
                // no other entry, so every column up to the first kept multiplier
                // is settled at once and only that one becomes a step.
                int found = -1, flag = 0;
                double mr = 0.0, mi = 0.0;
                int64_t uoff = 0;
                int ulen = 0;
                int kscan = kprev;   // positions <= kscan are settled
                bool searching = true;
                while (searching) {
                    uint32_t wl = 0u;
                    int wbase = -1;
                    for (int base = (kscan + 1) >> 5; base <= ((dpos - 1) >> 5); base += 64) {
                        const int wi = base + lane;
                        uint32_t word = 0u;
                        if (wi <= ((dpos - 1) >> 5) && wi < nwords) {
                            word = bits[wi];
                            const int lowb = wi * 32, hib = lowb + 32;
                            if (kscan + 1 > lowb) word &= ~0u << (kscan + 1 - lowb);   // positions > kscan
                            if (dpos < hib) word &= (dpos - lowb) >= 32 ? ~0u : ((1u << (dpos - lowb)) - 1u);   // < dpos
                        }
                        const unsigned long long bal = __ballot(word != 0u);
                        if (bal) {
                            const int l = __ffsll((long long)bal) - 1;
                            wl = (uint32_t)__shfl((int)word, l, 64);
                            wbase = (base + l) * 32;
                            break;
                        }
                    }
                    if (wbase < 0) break;   // no column left: the row is eliminated
                    const int first = __ffs((int)wl) - 1;
                    const int64_t k0 = lo + wbase + first;
                    if (k0 < 0) {   // a column left of 0: the window is corrupt
                        flag = -2;
                        found = wbase + first;
                        break;
                    }
                    if (!(k0 >= rlo && k0 + 31 < rlo + 64)) {
                        rlo = k0;
                        const int64_t r = k0 + lane;
                        rmask = __ballot(r < i && ld_flag(a.ready + r * FLAG_STRIDE) == (int32_t)a.epoch);
                        // rows seen finished: their data, read below with ordinary
                        // loads, must not come from lines cached before
                        if (rmask && a.acq_fence) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    }
                    const bool mem = lane < 32 && ((wl >> lane) & 1u);
                    const int64_t kl = lo + wbase + lane;
                    const bool rdyl = mem && kl >= rlo && kl < rlo + 64 && ((rmask >> (kl - rlo)) & 1ull);
                    const unsigned long long notready = __ballot(mem && !rdyl);
                    if ((notready >> first) & 1ull) {
                        // the first column's row is unfinished: wait for it
                        int ok = 1;
                        if (lane == 0) {
                            const unsigned long long tw = a.tstat ? wall_clock64() : 0;
                            ok = wait_flag(a.ready + k0 * FLAG_STRIDE, (int32_t)a.epoch, a.abort_flag, a.wait_ticks,
                                           a.status + 2, i, k0, (unsigned int)a.max_pause);
                            if (a.tstat) st_wait += wall_clock64() - tw;
                        }
                        ok = __shfl(ok, 0, 64);
                        if (!ok) {
                            flag = -1;
                            found = wbase + first;
                            break;
                        }
                        rmask |= 1ull << (k0 - rlo);
                        if (a.acq_fence) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                        continue;
                    }
                    // columns before the first unfinished row are decided now
                    const int lim = notready ? __ffsll((long long)notready) - 1 : 64;
                    const bool elig = mem && lane < lim;
                    double2 x = make_double2(0.0, 0.0), d = make_double2(1.0, 0.0);
                    int64_t uo = 0, uo1 = 0;
                    int ul = 0;
                    if (elig) {
                        x = wget(wbase + lane);
                        d = ld_coh(a.udiag + kl);
                        uo = a.u_off[kl];
                        uo1 = a.u_off[kl + 1];
                        ul = ld_flag(a.u_len + kl);
                    }
                    const bool nz = elig && (x.x != 0.0 || x.y != 0.0);
                    double ml = 0.0, nl = 0.0;
                    bool keep = false;
                    if (nz) {
                        const double den = d.x * d.x + d.y * d.y;
                        ml = (x.x * d.x + x.y * d.y) / den;
                        nl = (x.y * d.x - x.x * d.y) / den;
                        keep = !(ml * ml + nl * nl < tau2);
                    }
                    const unsigned long long kb = __ballot(keep);
                    const int fk = kb ? __ffsll((long long)kb) - 1 : 64;
                    if (nz && lane < fk) wput(wbase + lane, make_double2(0.0, 0.0));   // dropped multipliers
                    if (kb) {
                        found = wbase + fk;
                        mr = __shfl(ml, fk, 64);
                        mi = __shfl(nl, fk, 64);
                        uoff = (int64_t)__shfl((long long)uo, fk, 64);
                        ulen = __shfl(ul, fk, 64);
                        const int64_t uend = (int64_t)__shfl((long long)uo1, fk, 64);
                        if (lane == fk) wput(found, make_double2(mr, mi));
                        flag = 1;
                        if (ulen < 1 || uoff + ulen > uend) flag = -2;
                        searching = false;
                    } else {
                        kscan = wbase + (lim < 32 ? lim - 1 : 31);
                    }
                }
                if (lane == 0) {
                    s_k[par] = found;
                    s_flag[par] = flag;
                    s_m[par] = make_double2(mr, mi);
                    s_uoff[par] = uoff;
                    s_ulen[par] = ulen;
                }
            }
            __syncthreads();
            if (a.tstat && tid == 0) { const unsigned long long t = wall_clock64(); st_piv += t - tq; tq = t; ++st_steps; }
            const int kp = __builtin_amdgcn_readfirstlane(s_k[par]);
            const int fl = __builtin_amdgcn_readfirstlane(s_flag[par]);
            if (kp < 0 || fl < 0) {
                going = 0;
                if (fl == -2) stop = 1;   // recorded below
                if (fl == -1) stop = 1;   // a wait failed: the launch is being abandoned
            } else if (fl == 1) {
                const double mr = s_m[par].x, mi = s_m[par].y;
                const int64_t ub0 = s_uoff[par];
                const int len = __builtin_amdgcn_readfirstlane(s_ulen[par]);
                bool badcol = false;
                // UF entries per thread at a time (the columns of a U row are
                // distinct, so the updates of one step never meet); the U-row
                // loads of the next round are issued before a round's window
                // entries are read, so the two latencies overlap
                auto load_u = [&](int q0, int (&pc)[UF], double2 (&uv)[UF]) {
#pragma unroll
                    for (int j = 0; j < UF; ++j) {
                        const int q = q0 + j * IT;
                        pc[j] = -1;
                        if (q < len) {
                            pc[j] = a.u_col[ub0 + q];
                            uv[j] = a.u_val[ub0 + q];
                        }
                    }
                };
                auto update = [&](int q0, int (&pc)[UF], const double2 (&uv)[UF]) {
                    bool have[UF];
                    double2 wv[UF];
#pragma unroll
                    for (int j = 0; j < UF; ++j) {
                        have[j] = false;
                        if (q0 + j * IT < len) {
                            const int p = (int)(pc[j] - lo);
                            if (p <= kp || p >= W) {
                                badcol = true;
                                pc[j] = -1;
                            } else {
                                pc[j] = p;
                                have[j] = (bits[p >> 5] >> (p & 31)) & 1u;
                                if (have[j]) wv[j] = wget(p);
                            }
                        } else {
                            pc[j] = -1;
                        }
                    }
#pragma unroll
                    for (int j = 0; j < UF; ++j) {
                        const int p = pc[j];
                        if (p < 0) continue;
                        const double pr = mr * uv[j].x - mi * uv[j].y;
                        const double pi = mr * uv[j].y + mi * uv[j].x;
                        if (have[j]) {
                            double2 c = wv[j];
                            c.x -= pr;
                            c.y -= pi;
                            wput(p, c);
                        } else {
                            wput(p, make_double2(-pr, -pi));
                            atomicOr(&bits[p >> 5], 1u << (p & 31));
                        }
                    }
                };
                {
                    constexpr int RS = IT * UF;   // entries per round
                    int pca[UF], pcb[UF];
                    double2 uva[UF], uvb[UF];
                    load_u(1 + tid, pca, uva);
                    for (int q0 = 1 + tid; q0 < len; q0 += 2 * RS) {
                        if (q0 + RS < len) load_u(q0 + RS, pcb, uvb);
                        update(q0, pca, uva);
                        if (q0 + RS < len) {
                            if (q0 + 2 * RS < len) load_u(q0 + 2 * RS, pca, uva);
                            update(q0 + RS, pcb, uvb);
                        }
                    }
                }
                badrow |= badcol;   // checked once the row is eliminated (bad columns are skipped)
                if (tid == 0) n_upd += (unsigned long long)(len - 1);
                if (a.tstat && tid == 0) { st_upd += wall_clock64() - tq; ++st_usteps; st_ent += len; }
            }
            if (stop && fl == -2 && tid == 0)
                __hip_atomic_store(a.status + 4, (int32_t)(i + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            kprev = kp;
            par ^= 1;
            going = __builtin_amdgcn_readfirstlane(going);
            stop = __builtin_amdgcn_readfirstlane(stop);
        }
        if (block_or(badrow, s_or)) {
            stop = 1;
            if (tid == 0) __hip_atomic_store(a.status + 4, (int32_t)(i + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (a.tstat && tid == 0) tq = wall_clock64();
        if (stop) {
            if (tid == 0) publish_flag(a.abort_flag, 1);
        } else {
            // 3. dropping, cap, output.  The U row and the pivot come first and
            // are published at once (later rows wait only for them); the L row
            // is written afterwards.
            // the part of the working row held in LDS goes back to the window
            for (int q = tid; q < WIN_N; q += IT) {
                const int pp = cbase + q;
                if (pp >= 0 && pp < W && ((bits[pp >> 5] >> (pp & 31)) & 1u)) w[pp] = swin[q];
            }
            __syncthreads();
            const int64_t lb0 = a.l_off[i], ub0 = a.u_off[i];
            bool bad = false;
            double2 dg = make_double2(0.0, 0.0);
            if (tid == 0 && ((bits[dpos >> 5] >> (dpos & 31)) & 1u)) dg = w[dpos];
            const int nu = output_side(w, bits, dpos + 1, W, lo, tau2, lfil, a.u_col + ub0 + 1, a.u_val + ub0 + 1, true,
                                       &bad, side, hist, sbuf, a.cand_lim);
            if (tid == 0) {
                if (!isfinite(dg.x) || !isfinite(dg.y)) bad = true;
                const double fl = 1e-14 * rowinf;
                const double dmag = sqrt(dg.x * dg.x + dg.y * dg.y);
                if (!bad && (dmag < fl || dmag == 0.0)) {
                    if (dmag > 0.0) dg = make_double2(fl * dg.x / dmag, fl * dg.y / dmag);
                    else if (fl > 0.0) dg = make_double2(fl, 0.0);
                    else dg = make_double2(1.0, 0.0);
                    atomicAdd(a.status + 1, 1);
                }
                a.u_col[ub0] = (int32_t)i;
                a.u_val[ub0] = dg;
                a.udiag[i] = dg;
                a.u_len[i] = nu + 1;
            }
            if (block_or(bad, s_or)) {
                stop = 1;
                if (tid == 0) {
                    atomicCAS(a.status, 0, (int32_t)(i + 1));
                    publish_flag(a.abort_flag, 1);
                }
            } else {
                if (a.tstat && tid == 0) { const unsigned long long t = wall_clock64(); st_finu += t - tq; }
                if (tid == 0) {
                    // the release writes the row back from L2 before the flag
                    const unsigned long long tp = a.tstat ? wall_clock64() : 0;
                    publish_flag(a.ready + i * FLAG_STRIDE, (int32_t)a.epoch);
                    if (a.tstat) st_pub += wall_clock64() - tp;
                    if ((i & 4095) == 0) __hip_atomic_store(a.host_progress, (int32_t)i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                }
                const int nl = output_side(w, bits, 0, dpos, lo, tau2, lfil, a.l_col + lb0, a.l_val + lb0, false, &bad,
                                           side, hist, sbuf, a.cand_lim);
                if (tid == 0) a.l_len[i] = nl;
            }
        }
        // next row
        __syncthreads();
        if (a.tstat && tid == 0) { st_fin += wall_clock64() - tq; ++st_rows; }
        if (tid == 0) {
            s_row = atomicAdd(a.next_row, 1);
            s_stop = ld_flag(a.abort_flag);
        }
        __syncthreads();
        i = __builtin_amdgcn_readfirstlane(s_row);
        stop = __builtin_amdgcn_readfirstlane(stop | s_stop);
    }
    if (tid == 0) atomicAdd(reinterpret_cast<unsigned long long*>(a.status + 38), n_upd);
    if (a.tstat && tid == 0) {
        atomicAdd(a.tstat + 0, st_piv);
        atomicAdd(a.tstat + 1, st_wait);
        atomicAdd(a.tstat + 2, st_upd);
        atomicAdd(a.tstat + 3, st_fin);
        atomicAdd(a.tstat + 4, st_rows);
        atomicAdd(a.tstat + 5, st_steps);
        atomicAdd(a.tstat + 6, st_usteps);
        atomicAdd(a.tstat + 7, st_ent);
        atomicAdd(a.tstat + 8, st_finu);
        for (int k = 0; k < 12; ++k) atomicAdd(a.tstat + 9 + k, side.tph[k]);
        atomicAdd(a.tstat + 21, st_pub);
    }
}

// Factor item `item` of A on the device; the CSR factor is returned on the
// host in F (same layout as ilut_factor_host).
om_status ilut_factor_dev(const om_csr* A, int item, double drop_tol, double fill_factor, DevFactor* D,
                          std::string* err, hipStream_t s) {
    const int64_t n = A->n;
    om_csr* Am = const_cast<om_csr*>(A);
    OM_TRY(ensure_host_pattern(Am, s));
    // band of A
    int64_t lb = 0, ub = 0;
    for (int64_t r = 0; r < n; ++r)
        for (int64_t t = Am->h_row_ptr[r]; t < Am->h_row_ptr[r + 1]; ++t) {
            const int64_t d = Am->h_col[t] - r;
            lb = std::max(lb, -d);
            ub = std::max(ub, d);
        }
    const int64_t W = lb + ub + 1;
    if (W > WBITS_MAX) { set_error("band window %lld exceeds the device ILUT limit %d", (long long)W, WBITS_MAX); return OM_EINVAL; }
    const bool capped = std::isfinite(fill_factor);
    // row capacities in multiples of 32 entries, so that both the value
    // (16-byte) and the column (4-byte) storage of a row are 128-byte aligned
    std::vector<int64_t> loff(n + 1, 0), uoff(n + 1, 0);
    for (int64_t r = 0; r < n; ++r) {
        const int64_t nz = Am->h_row_ptr[r + 1] - Am->h_row_ptr[r];
        int64_t lf = capped ? std::max<int64_t>(0, (int64_t)std::floor((fill_factor * (double)nz - 1.0) / 2.0)) : INT64_MAX;
        const int64_t cl = std::min<int64_t>(lf, std::min<int64_t>(lb, r));
        const int64_t cu = std::min<int64_t>(lf, std::min<int64_t>(ub, n - 1 - r)) + 1;
        loff[r + 1] = loff[r] + ((cl + 31) & ~31ll);
        uoff[r + 1] = uoff[r] + ((cu + 31) & ~31ll);
    }
    int dev = 0, cus = 0, per = 0, coop = 0, clk_khz = 0;
    OM_HIP(hipGetDevice(&dev));
    OM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    OM_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    OM_HIP(hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, dev));
    OM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, ilut_row_kernel, IT, 0));
    if (!coop || per < 1) { set_error("cooperative launch unavailable for the device ILUT"); return OM_EINVAL; }
    int G = (int)std::min<int64_t>((int64_t)cus * per, std::max<int64_t>(1, n));
    if (const char* e = getenv("OMSS_ILUT_GRID")) G = std::max(1, std::min(G, atoi(e)));
    DevBuf<int64_t>& dloff = D->l_off;
    DevBuf<int64_t>& duoff = D->u_off;
    OM_TRY(dloff.upload(loff.data(), loff.size(), s));
    OM_TRY(duoff.upload(uoff.data(), uoff.size(), s));
    DevBuf<int32_t>& llen = D->l_len;
    DevBuf<int32_t>& ulen = D->u_len;
    DevBuf<int32_t>& lcol = D->l_col;
    DevBuf<int32_t>& ucol = D->u_col;
    DevBuf<double2>& lval = D->l_val;
    DevBuf<double2>& uval = D->u_val;
    D->n = n;
    DevBuf<int32_t> ready, misc;
    DevBuf<double2> work, udiag;
    OM_TRY(llen.alloc(n));
    OM_TRY(ulen.alloc(n));
    OM_TRY(lcol.alloc(std::max<int64_t>(1, loff[n])));
    OM_TRY(lval.alloc(std::max<int64_t>(1, loff[n])));
    OM_TRY(ucol.alloc(uoff[n]));
    OM_TRY(uval.alloc(uoff[n]));
    OM_TRY(ready.alloc((size_t)n * FLAG_STRIDE));
    OM_TRY(udiag.alloc(n));
    OM_TRY(misc.alloc(64));   // [0] row counter, [2..17] status, [32] abort flag (a line of its own), [40..41] U-row entries read
    const int64_t wstride = (W + 7) & ~7ll;
    OM_TRY(work.alloc((size_t)G * wstride));
    OM_HIP(hipMemsetAsync(ready.p, 0, ready.bytes(), s));
    OM_HIP(hipMemsetAsync(misc.p, 0, misc.bytes(), s));
    // everything the launch reads is in place before it starts
    OM_HIP(hipStreamSynchronize(s));
    IlutDevArgs a;
    a.n = n; a.lb = (int32_t)lb; a.ub = (int32_t)ub; a.W = (int32_t)W; a.wstride = wstride;
    a.row_ptr = A->row_ptr.p; a.col = A->col.p; a.val = A->val.p + (size_t)item * A->nnz;
    a.drop_tol = drop_tol; a.fill_factor = fill_factor; a.capped = capped;
    a.l_off = dloff.p; a.u_off = duoff.p; a.l_len = llen.p; a.u_len = ulen.p;
    a.l_col = lcol.p; a.l_val = lval.p; a.u_col = ucol.p; a.u_val = uval.p;
    a.udiag = udiag.p; a.ready = ready.p; a.epoch = 1; a.work = work.p;
    double wait_s = 30.0;   // bound of one wait (OMSS_ILUT_WAIT_S)
    if (const char* e = getenv("OMSS_ILUT_WAIT_S")) wait_s = std::max(0.1, atof(e));
    a.wait_ticks = (long long)((double)std::max(clk_khz, 1000) * 1000.0 * wait_s);
    a.next_row = misc.p; a.abort_flag = misc.p + 32; a.status = misc.p + 2;
    a.acq_fence = 1;
    a.max_pause = 32;
    if (const char* e = getenv("OMSS_ILUT_BACKOFF")) a.max_pause = std::max(1, std::min(1024, atoi(e)));
    if (const char* e = getenv("OMSS_ILUT_FENCE")) a.acq_fence = atoi(e) != 0;
    // OMSS_ILUT_STAGE=c: a lower limit of the LDS staging of the dropping (the
    // factor does not depend on it; tests use small limits so that small
    // operators also take the path that reads the keys from the working row)
    a.cand_lim = CAND_MAX;
    if (const char* e = getenv("OMSS_ILUT_STAGE")) a.cand_lim = std::max(0, std::min(CAND_MAX, atoi(e)));
    DevBuf<unsigned long long> tstat;
    a.tstat = nullptr;
    if (getenv("OMSS_ILUT_STATS")) {
        OM_TRY(tstat.alloc(22));
        OM_HIP(hipMemsetAsync(tstat.p, 0, tstat.bytes(), s));
        OM_HIP(hipStreamSynchronize(s));
        a.tstat = tstat.p;
    }
    // progress word in pinned host memory, written by the kernel now and then
    int32_t* hprog = nullptr;
    OM_HIP(hipHostMalloc((void**)&hprog, 256, hipHostMallocMapped | hipHostMallocCoherent));
    struct HostFree { int32_t* p; ~HostFree() { if (p) (void)hipHostFree(p); } } hprog_guard{hprog};
    *(volatile int32_t*)hprog = 0;
    OM_HIP(hipHostGetDevicePointer((void**)&a.host_progress, hprog, 0));
    void* args[] = {(void*)&a};
    const bool verbose = std::getenv("OMSS_VERBOSE") != nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    // rows are handed out dynamically, so the blocks need not be co-resident:
    // an ordinary launch (OMSS_ILUT_COOP=1 selects a cooperative one)
    const char* ce = getenv("OMSS_ILUT_COOP");
    ProfScope prof("ilut", s, 0.0);
    if (ce && atoi(ce) == 1) {
        OM_HIP(hipLaunchCooperativeKernel((const void*)ilut_row_kernel, dim3(G), dim3(IT), args, 0, s));
    } else {
        hipLaunchKernelGGL(ilut_row_kernel, dim3(G), dim3(IT), 0, s, a);
        OM_HIP(hipGetLastError());
    }
    prof.stop();
    double next_report = 20.0;
    while (true) {
        const hipError_t q = hipStreamQuery(s);
        if (q == hipSuccess) break;
        if (q != hipErrorNotReady) OM_HIP(q);
        std::this_thread::sleep_for(std::chrono::milliseconds(20));
        const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (verbose && el >= next_report) {
            fprintf(stderr, "[omss] device ILUT: ~%d/%lld rows after %.0f s\n", *(volatile int32_t*)hprog,
                    (long long)n, el);
            next_report += 20.0;
        }
    }
    int32_t hs[64];
    OM_HIP(hipMemcpyAsync(hs, misc.p, sizeof hs, hipMemcpyDeviceToHost, s));
    OM_HIP(hipStreamSynchronize(s));
    if (verbose)
        fprintf(stderr, "[omss] device ILUT: n %lld, window %lld, %d workgroups, %.3f s\n", (long long)n, (long long)W, G,
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    if (a.tstat) {
        unsigned long long h[22];
        OM_HIP(hipMemcpy(h, a.tstat, sizeof h, hipMemcpyDeviceToHost));
        const double us = 1e6 / ((double)std::max(clk_khz, 1000) * 1000.0);
        const double rows = (double)std::max(1ull, h[4]);
        fprintf(stderr, "[ilut stats] %d workgroups, window %lld: per row %.1f steps (%.1f updating, %.0f entries); "
                "per row us: pivot steps %.1f (of which waiting %.1f), updates %.1f, dropping and output %.1f (U side "
                "to its publication %.1f)\n", G, (long long)W, h[5] / rows, h[6] / rows, h[7] / rows, h[0] * us / rows,
                h[1] * us / rows, h[2] * us / rows, h[3] * us / rows, h[8] * us / rows);
        fprintf(stderr, "[ilut stats] dropping and output per row us (both triangles, staged path): positions %.1f, "
                "keys %.1f, select %.1f, output %.1f\n", h[9] * us / rows, h[10] * us / rows, h[11] * us / rows,
                h[12] * us / rows);
        fprintf(stderr, "[ilut stats] triangle outputs: %llu staged in LDS (%llu capped), %llu from the window; "
                "publication (release) per row %.1f us\n", h[13], h[20], h[15], h[21] * us / rows);
    }
    if (hs[2] != 0) {
        if (err) *err = "ILUT breakdown: non-finite pivot or entry in row " + std::to_string(hs[2] - 1) +
                        " (the incomplete factorisation is unstable for this drop tolerance and fill)";
        return OM_EBREAKDOWN;
    }
    if (hs[6] != 0) {
        set_error("device ILUT: inconsistent row data met while eliminating row %d", hs[6] - 1);
        return OM_EHIP;
    }
    if (hs[32] != 0) {
        std::vector<int32_t> rd(n);
        OM_HIP(hipMemcpy2D(rd.data(), sizeof(int32_t), ready.p, FLAG_STRIDE * sizeof(int32_t), sizeof(int32_t), n,
                           hipMemcpyDeviceToHost));
        int64_t published = 0, first_missing = -1;
        for (int64_t r = 0; r < n; ++r) {
            if (rd[r] == 1) ++published;
            else if (first_missing < 0) first_missing = r;
        }
        set_error("device ILUT: a wait timed out (row %d waited for row %d; %lld of %lld rows published, first "
                  "missing %lld)", hs[4] - 1, hs[5] - 1, (long long)published, (long long)n, (long long)first_missing);
        return OM_ETIMEOUT;
    }
    // entry counts
    {
        std::vector<int32_t> hl(n), hu(n);
        OM_HIP(hipMemcpyAsync(hl.data(), llen.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        OM_HIP(hipMemcpyAsync(hu.data(), ulen.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        OM_HIP(hipStreamSynchronize(s));
        D->nnz_l = D->nnz_u = 0;
        for (int64_t r = 0; r < n; ++r) {
            D->nnz_l += hl[r];
            D->nnz_u += hu[r];
        }
    }
    D->repaired = hs[3];
    // algorithmic bytes: the U-row entries read by the eliminations, row i of
    // A, and the factor written (4-byte column + 16-byte value per entry)
    D->upd_entries = (int64_t)((uint64_t)(uint32_t)hs[40] | ((uint64_t)(uint32_t)hs[41] << 32));
    prof.set_bytes(20.0 * ((double)D->upd_entries + (double)A->nnz + (double)(D->nnz_l + D->nnz_u)));
    return OM_OK;
}

// Copy of a device factor into the host CSR layout of ilut_factor_host.
om_status devfactor_to_host(const DevFactor& D, HostFactor* F, hipStream_t s) {
    const int64_t n = D.n;
    std::vector<int64_t> loff(n + 1), uoff(n + 1);
    std::vector<int32_t> hl(n), hu(n);
    OM_HIP(hipMemcpyAsync(loff.data(), D.l_off.p, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    OM_HIP(hipMemcpyAsync(uoff.data(), D.u_off.p, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    OM_HIP(hipMemcpyAsync(hl.data(), D.l_len.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    OM_HIP(hipMemcpyAsync(hu.data(), D.u_len.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    OM_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> acol(std::max<int64_t>(1, loff[n])), bcol(std::max<int64_t>(1, uoff[n]));
    std::vector<double2> aval(std::max<int64_t>(1, loff[n])), bval(std::max<int64_t>(1, uoff[n]));
    OM_HIP(hipMemcpyAsync(acol.data(), D.l_col.p, loff[n] * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    OM_HIP(hipMemcpyAsync(aval.data(), D.l_val.p, loff[n] * sizeof(double2), hipMemcpyDeviceToHost, s));
    OM_HIP(hipMemcpyAsync(bcol.data(), D.u_col.p, uoff[n] * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    OM_HIP(hipMemcpyAsync(bval.data(), D.u_val.p, uoff[n] * sizeof(double2), hipMemcpyDeviceToHost, s));
    OM_HIP(hipStreamSynchronize(s));
    F->n = n;
    F->l_ptr.assign(n + 1, 0);
    F->u_ptr.assign(n + 1, 0);
    for (int64_t r = 0; r < n; ++r) {
        F->l_ptr[r + 1] = F->l_ptr[r] + hl[r];
        F->u_ptr[r + 1] = F->u_ptr[r] + hu[r];
    }
    F->l_col.resize(F->l_ptr[n]);
    F->l_val.resize(2 * F->l_ptr[n]);
    F->u_col.resize(F->u_ptr[n]);
    F->u_val.resize(2 * F->u_ptr[n]);
    for (int64_t r = 0; r < n; ++r) {
        for (int q = 0; q < hl[r]; ++q) {
            F->l_col[F->l_ptr[r] + q] = acol[loff[r] + q];
            F->l_val[2 * (F->l_ptr[r] + q)] = aval[loff[r] + q].x;
            F->l_val[2 * (F->l_ptr[r] + q) + 1] = aval[loff[r] + q].y;
        }
        for (int q = 0; q < hu[r]; ++q) {
            F->u_col[F->u_ptr[r] + q] = bcol[uoff[r] + q];
            F->u_val[2 * (F->u_ptr[r] + q)] = bval[uoff[r] + q].x;
            F->u_val[2 * (F->u_ptr[r] + q) + 1] = bval[uoff[r] + q].y;
        }
    }
    F->perm.resize(n);
    for (int64_t r = 0; r < n; ++r) F->perm[r] = (int32_t)r;
    F->repaired = D.repaired;
    F->pivots = 0;
    return OM_OK;
}

}  // namespace omss
