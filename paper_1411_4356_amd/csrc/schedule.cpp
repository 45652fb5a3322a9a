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
// that lie left of it are stored slot-major (ELL) in three lists by the block
// of their column: "near" (block g-1), "mid" (block g-2) and "far" (older);
// slot s of row r of block g is at [(off[g] + s) * 64 + r], columns
// increasing with s, short rows padded with value 0.  Near and mid rows start
// at slot 0 and are padded at the end; far rows end at the last slot and are
// padded at the start, so that the far slots read older blocks first and the
// slots that need the newest blocks are few (each far slot takes the newest
// block of its 64 rows, and a row padded at the end would reach its own
// newest columns early).  For every far slot, need[slot] is the newest
// column block it reads.  The strictly-lower part of
// the 64x64 diagonal block is stored dense and packed by column.
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
    H.far_off.assign(H.nblk + 1, 0);
    H.mid_off.assign(H.nblk + 1, 0);
    H.near_off.assign(H.nblk + 1, 0);
    // class of a column c for block g: 0 far, 1 mid, 2 near, 3 diagonal block
    auto cls = [](int64_t c, int64_t g) -> int {
        const int64_t cb = c / BLK;
        if (cb == g) return 3;
        if (cb == g - 1) return 2;
        if (cb == g - 2) return 1;
        return 0;
    };
    std::vector<int64_t>* offs[3] = {&H.far_off, &H.mid_off, &H.near_off};
    for (int64_t g = 0; g < H.nblk; ++g) {
        const int64_t r0 = g * BLK;
        int64_t mx[3] = {0, 0, 0};
        for (int r = 0; r < BLK && r0 + r < n; ++r) {
            const int64_t i = r0 + r;
            int64_t cnt[4] = {0, 0, 0, 0};
            for (int64_t t = T.ptr[i]; t < T.ptr[i + 1]; ++t) cnt[cls(T.col[t], g)]++;
            for (int k = 0; k < 3; ++k) mx[k] = std::max(mx[k], cnt[k]);
        }
        for (int k = 0; k < 3; ++k) (*offs[k])[g + 1] = (*offs[k])[g] + mx[k];
    }
    const int64_t nsf = H.far_off[H.nblk], nsm = H.mid_off[H.nblk], nsn = H.near_off[H.nblk];
    H.far_col.assign((size_t)nsf * BLK, 0);
    H.far_val.assign((size_t)nsf * BLK * 2, 0.0);
    H.far_need.assign((size_t)nsf, 0);
    H.mid_col.assign((size_t)nsm * BLK, 0);
    H.mid_val.assign((size_t)nsm * BLK * 2, 0.0);
    H.near_col.assign((size_t)nsn * BLK, 0);
    H.near_val.assign((size_t)nsn * BLK * 2, 0.0);
    H.dg.assign((size_t)H.nblk * TRI * 2, 0.0);
    std::vector<int32_t>* cols[3] = {&H.far_col, &H.mid_col, &H.near_col};
    std::vector<double>* vals[3] = {&H.far_val, &H.mid_val, &H.near_val};
    for (int64_t g = 0; g < H.nblk; ++g) {
        const int64_t r0 = g * BLK;
        // padding: a column of the list's own block (value 0), so that no read
        // reaches an unfinished block
        for (int k = 1; k < 3; ++k) {
            const int32_t pad = (int32_t)std::max<int64_t>(0, (g - 3 + k) * BLK);
            for (int64_t s = (*offs[k])[g]; s < (*offs[k])[g + 1]; ++s)
                for (int r = 0; r < BLK; ++r) (*cols[k])[s * BLK + r] = pad;
        }
        for (int r = 0; r < BLK && r0 + r < n; ++r) {
            const int64_t i = r0 + r;
            int64_t nfar = 0;
            for (int64_t t = T.ptr[i]; t < T.ptr[i + 1]; ++t) nfar += cls(T.col[t], g) == 0;
            int64_t sl[3] = {H.far_off[g + 1] - H.far_off[g] - nfar, 0, 0};
            for (int64_t t = T.ptr[i]; t < T.ptr[i + 1]; ++t) {
                const int64_t c = T.col[t];
                const int k = cls(c, g);
                if (k == 3) {
                    const int64_t at = g * TRI + tri_index((int)(c - r0), r);
                    H.dg[2 * at] = T.val[2 * t];
                    H.dg[2 * at + 1] = T.val[2 * t + 1];
                    continue;
                }
                const int64_t slot = (*offs[k])[g] + sl[k]++;
                const int64_t at = slot * BLK + r;
                (*cols[k])[at] = (int32_t)c;
                (*vals[k])[2 * at] = T.val[2 * t];
                (*vals[k])[2 * at + 1] = T.val[2 * t + 1];
                if (k == 0) H.far_need[slot] = std::max<int32_t>(H.far_need[slot], (int32_t)(c / BLK));
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
    S.rev = H.rev;
    S.depth = H.depth;
    S.nnz = H.nnz;
    S.has_dinv = !H.dinv.empty();
    S.nslots_far = H.far_off.back();
    S.nslots_near = H.near_off.back() + H.mid_off.back();
    OM_TRY(up(S.far_off, H.far_off.data(), H.far_off.size()));
    OM_TRY(up(S.mid_off, H.mid_off.data(), H.mid_off.size()));
    OM_TRY(up(S.near_off, H.near_off.data(), H.near_off.size()));
    OM_TRY(up(S.far_col, H.far_col.data(), H.far_col.size()));
    OM_TRY(up(S.far_need, H.far_need.data(), H.far_need.size()));
    OM_TRY(up(S.mid_col, H.mid_col.data(), H.mid_col.size()));
    OM_TRY(up(S.near_col, H.near_col.data(), H.near_col.size()));
    OM_TRY(up(S.far_val, H.far_val.data(), H.far_val.size() / 2));
    OM_TRY(up(S.mid_val, H.mid_val.data(), H.mid_val.size() / 2));
    OM_TRY(up(S.near_val, H.near_val.data(), H.near_val.size() / 2));
    OM_TRY(up(S.dg, H.dg.data(), H.dg.size() / 2));
    if (!H.dinv.empty()) OM_TRY(up(S.dinv, H.dinv.data(), H.dinv.size() / 2));
    else S.dinv.release();
    if (c64) {
        std::vector<float> f;
        narrow(H.far_val, f);
        OM_TRY(up(S.far_val32, f.data(), f.size() / 2));
        narrow(H.mid_val, f);
        OM_TRY(up(S.mid_val32, f.data(), f.size() / 2));
        narrow(H.near_val, f);
        OM_TRY(up(S.near_val32, f.data(), f.size() / 2));
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
