// Solve schedules for the ILU factors (host side).
//
// Each of the four triangular solves used by the preconditioner (L, U and,
// for adjoint solves, U^H and L^H) is brought to one form: a unit lower
// triangular matrix T in "solve coordinates" plus an optional row scaling of
// the right-hand side (dinv), so that T x = dinv .* y.  An upper factor is
// stored with rows and columns reversed (i -> n-1-i), which makes it lower;
// the pivots of U are divided out of its rows and applied to the
// right-hand side instead.
//
// Rows are grouped in blocks of 64 (one wavefront).  The entries of a block
// that lie left of the block are stored slot-major (ELL): slot s of row r at
// [(off[g] + s) * 64 + r], columns increasing with s, short rows padded with
// column 0 and value 0.  The strictly-lower part of the 64x64 diagonal block is
// stored dense and packed by column.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

#include "common.hpp"
#include "ilut.hpp"
#include "schedule.hpp"

namespace omss {

static constexpr int BLK = 64;
static constexpr int TRI = BLK * (BLK - 1) / 2;

static inline int64_t tri_index(int c, int r) {  // r > c
    return (int64_t)c * (BLK - 1) - (int64_t)c * (c - 1) / 2 + (r - c - 1);
}

int64_t level_depth(int64_t n, const std::vector<int64_t>& ptr, const std::vector<int32_t>& col) {
    std::vector<int32_t> lev(n, 0);
    int32_t depth = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t l = 0;
        for (int64_t t = ptr[i]; t < ptr[i + 1]; ++t) l = std::max(l, lev[col[t]] + 1);
        lev[i] = l;
        depth = std::max(depth, l + 1);
    }
    return n ? depth : 0;
}

void build_host_tri(const SolveCSR& T, HostTri& H) {
    const int64_t n = T.n;
    H.n = n;
    H.nblk = (n + BLK - 1) / BLK;
    H.depth = level_depth(n, T.ptr, T.col);
    H.nnz = T.ptr[n];
    H.off.assign(H.nblk + 1, 0);
    for (int64_t g = 0; g < H.nblk; ++g) {
        const int64_t r0 = g * BLK;
        int64_t ns = 0;
        for (int r = 0; r < BLK && r0 + r < n; ++r) {
            const int64_t i = r0 + r;
            int64_t c = 0;
            for (int64_t t = T.ptr[i]; t < T.ptr[i + 1] && T.col[t] < r0; ++t) ++c;
            ns = std::max(ns, c);
        }
        H.off[g + 1] = H.off[g] + ns;
    }
    const int64_t nslots = H.off[H.nblk];
    H.col.assign((size_t)nslots * BLK, 0);
    H.val.assign((size_t)nslots * BLK * 2, 0.0);
    H.dg.assign((size_t)H.nblk * TRI * 2, 0.0);
    for (int64_t g = 0; g < H.nblk; ++g) {
        const int64_t r0 = g * BLK;
        for (int r = 0; r < BLK && r0 + r < n; ++r) {
            const int64_t i = r0 + r;
            int64_t s = 0;
            for (int64_t t = T.ptr[i]; t < T.ptr[i + 1]; ++t) {
                const int64_t c = T.col[t];
                if (c < r0) {
                    const int64_t at = (H.off[g] + s) * BLK + r;
                    H.col[at] = (int32_t)c;
                    H.val[2 * at] = T.val[2 * t];
                    H.val[2 * at + 1] = T.val[2 * t + 1];
                    ++s;
                } else {
                    const int cc = (int)(c - r0);
                    const int64_t at = g * TRI + tri_index(cc, r);
                    H.dg[2 * at] = T.val[2 * t];
                    H.dg[2 * at + 1] = T.val[2 * t + 1];
                }
            }
        }
    }
    H.dinv = T.dinv;
    H.rev = T.rev;
}

static inline void cdiv(double ar, double ai, double br, double bi, double& rr, double& ri) {
    const double den = br * br + bi * bi;
    rr = (ar * br + ai * bi) / den;
    ri = (ai * br - ar * bi) / den;
}

void factor_to_solve(const HostFactor& F, int kind, SolveCSR& T) {
    const int64_t n = F.n;
    T = SolveCSR();
    // 0: L as stored
    if (kind == 0) {
        T.n = n; T.rev = false;
        T.ptr = F.l_ptr; T.col = F.l_col; T.val = F.l_val; T.dinv.clear();
    }
    // 1: U reversed, rows scaled by 1/u_ii
    if (kind == 1) {
        T.n = n; T.rev = true;
        T.ptr.assign(n + 1, 0);
        for (int64_t ip = 0; ip < n; ++ip) {
            const int64_t i = n - 1 - ip;
            T.ptr[ip + 1] = T.ptr[ip] + (F.u_ptr[i + 1] - F.u_ptr[i] - 1);
        }
        T.col.resize(T.ptr[n]);
        T.val.resize(2 * T.ptr[n]);
        T.dinv.resize(2 * n);
        for (int64_t ip = 0; ip < n; ++ip) {
            const int64_t i = n - 1 - ip;
            const int64_t d = F.u_ptr[i];
            const double ur = F.u_val[2 * d], ui = F.u_val[2 * d + 1];
            cdiv(1.0, 0.0, ur, ui, T.dinv[2 * ip], T.dinv[2 * ip + 1]);
            int64_t o = T.ptr[ip];
            for (int64_t t = F.u_ptr[i + 1] - 1; t > d; --t) {  // descending j = ascending j'
                T.col[o] = (int32_t)(n - 1 - F.u_col[t]);
                cdiv(F.u_val[2 * t], F.u_val[2 * t + 1], ur, ui, T.val[2 * o], T.val[2 * o + 1]);
                ++o;
            }
        }
    }
    // 2: U^H (lower), rows scaled by 1/conj(u_ii)
    if (kind == 2) {
        T.n = n; T.rev = false;
        T.ptr.assign(n + 1, 0);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t t = F.u_ptr[i] + 1; t < F.u_ptr[i + 1]; ++t) T.ptr[F.u_col[t] + 1]++;
        for (int64_t i = 0; i < n; ++i) T.ptr[i + 1] += T.ptr[i];
        T.col.resize(T.ptr[n]);
        T.val.resize(2 * T.ptr[n]);
        T.dinv.resize(2 * n);
        std::vector<int64_t> pos(T.ptr.begin(), T.ptr.end() - 1);
        for (int64_t j = 0; j < n; ++j) {       // row j of U = column j of U^H, ascending
            for (int64_t t = F.u_ptr[j] + 1; t < F.u_ptr[j + 1]; ++t) {
                const int64_t i = F.u_col[t];
                const int64_t o = pos[i]++;
                T.col[o] = (int32_t)j;
                T.val[2 * o] = F.u_val[2 * t];
                T.val[2 * o + 1] = -F.u_val[2 * t + 1];
            }
        }
        for (int64_t i = 0; i < n; ++i) {
            const int64_t d = F.u_ptr[i];
            const double cr = F.u_val[2 * d], ci = -F.u_val[2 * d + 1];   // conj(u_ii)
            cdiv(1.0, 0.0, cr, ci, T.dinv[2 * i], T.dinv[2 * i + 1]);
            for (int64_t o = T.ptr[i]; o < T.ptr[i + 1]; ++o) {
                double a = T.val[2 * o], b = T.val[2 * o + 1];
                cdiv(a, b, cr, ci, T.val[2 * o], T.val[2 * o + 1]);
            }
        }
    }
    // 3: L^H (unit upper) reversed
    if (kind == 3) {
        T.n = n; T.rev = true;
        // column counts of L
        std::vector<int64_t> cnt(n + 1, 0);
        for (int64_t t = 0; t < (int64_t)F.l_col.size(); ++t) cnt[F.l_col[t] + 1]++;
        for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
        // gather column i of L (rows j > i, ascending)
        std::vector<int32_t> crow(F.l_col.size());
        std::vector<double> cval(F.l_val.size());
        std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
        for (int64_t j = 0; j < n; ++j)
            for (int64_t t = F.l_ptr[j]; t < F.l_ptr[j + 1]; ++t) {
                const int64_t o = pos[F.l_col[t]]++;
                crow[o] = (int32_t)j;
                cval[2 * o] = F.l_val[2 * t];
                cval[2 * o + 1] = -F.l_val[2 * t + 1];
            }
        T.ptr.assign(n + 1, 0);
        for (int64_t ip = 0; ip < n; ++ip) {
            const int64_t i = n - 1 - ip;
            T.ptr[ip + 1] = T.ptr[ip] + (cnt[i + 1] - cnt[i]);
        }
        T.col.resize(T.ptr[n]);
        T.val.resize(2 * T.ptr[n]);
        T.dinv.clear();
        for (int64_t ip = 0; ip < n; ++ip) {
            const int64_t i = n - 1 - ip;
            int64_t o = T.ptr[ip];
            for (int64_t t = cnt[i + 1] - 1; t >= cnt[i]; --t) {   // descending j = ascending j'
                T.col[o] = (int32_t)(n - 1 - crow[t]);
                T.val[2 * o] = cval[2 * t];
                T.val[2 * o + 1] = cval[2 * t + 1];
                ++o;
            }
        }
    }
}

template <typename T>
static om_status up(DevBuf<T>& d, const void* h, size_t count) {
    OM_TRY(d.alloc(count));
    if (count) OM_HIP(hipMemcpy(d.p, h, count * sizeof(T), hipMemcpyHostToDevice));
    return OM_OK;
}

static void narrow(const std::vector<double>& in, std::vector<float>& out) {
    out.resize(in.size());
    for (size_t i = 0; i < in.size(); ++i) out[i] = (float)in[i];
}

om_status upload_tri(const HostTri& H, bool c64, TriSched& S) {
    S.n = H.n;
    S.nblk = H.nblk;
    S.nslots = H.off.empty() ? 0 : H.off.back();
    S.rev = H.rev;
    S.depth = H.depth;
    S.nnz = H.nnz;
    S.has_dinv = !H.dinv.empty();
    OM_TRY(up(S.off, H.off.data(), H.off.size()));
    OM_TRY(up(S.col, H.col.data(), H.col.size()));
    OM_TRY(up(S.val, H.val.data(), H.val.size() / 2));
    OM_TRY(up(S.dg, H.dg.data(), H.dg.size() / 2));
    if (!H.dinv.empty()) OM_TRY(up(S.dinv, H.dinv.data(), H.dinv.size() / 2));
    else S.dinv.release();
    if (c64) {
        std::vector<float> f;
        narrow(H.val, f);
        OM_TRY(up(S.val32, f.data(), f.size() / 2));
        narrow(H.dg, f);
        OM_TRY(up(S.dg32, f.data(), f.size() / 2));
        if (!H.dinv.empty()) {
            narrow(H.dinv, f);
            OM_TRY(up(S.dinv32, f.data(), f.size() / 2));
        }
    }
    return OM_OK;
}

}  // namespace omss
