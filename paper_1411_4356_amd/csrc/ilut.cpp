// Dual-threshold incomplete LU factorisation with threshold column pivoting
// on the host (Sec. II: iLUTP with drop tolerance d and fill limit p).
//
// Row-wise ILUTP: row i is copied into a dense work row w, eliminated against
// the already-final rows of U in increasing pivot position (fill included);
// a multiplier with |w_k| < tau_i = d * ||a_i||_inf is dropped before use
// (first rule).  Afterwards every off-diagonal entry below tau_i is dropped
// (second rule); if the diagonal is smaller than permtol times the largest
// remaining entry of the upper part, the two columns are exchanged (threshold
// pivoting, a column permutation Q with A Q ~ L U); then at most
// lfil_i = floor((p * nnz(a_i) - 1) / 2) entries are kept in each triangle,
// largest modulus first, ties to the lower column.  A pivot below
// 1e-14 * ||a_i||_inf is raised to that floor (same phase) and counted.
// Magnitudes are compared as squared moduli.  A non-finite pivot or U entry
// stops the factorisation (breakdown: the incomplete factors have grown
// without bound, which happens when too much fill is dropped).
//
// Columns are tracked by their original index while the factorisation runs
// (pivoting renumbers positions >= i only, so positions < i are final); the
// factor is returned in position coordinates: L strictly lower (unit diagonal
// implied), U with the diagonal first in every row, perm[position] = column.
#include "ilut.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <queue>
#include <string>
#include <vector>

namespace omss {

namespace {

struct Entry {
    int32_t col;   // original column
    int32_t pos;   // position (for ordering ties)
    double re, im;
    double mag2() const { return re * re + im * im; }
};

// total order used by the per-row cap: larger modulus first, then lower position
inline bool keep_before(const Entry& a, const Entry& b) {
    const double ma = a.mag2(), mb = b.mag2();
    if (ma != mb) return ma > mb;
    return a.pos < b.pos;
}

}  // namespace

int ilut_factor_host(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val, double drop_tol,
                     double fill_factor, double permtol, HostFactor* out, std::string* err) {
    const bool capped = std::isfinite(fill_factor);
    const bool pivoting = permtol > 0.0;
    std::vector<double> wre(n, 0.0), wim(n, 0.0);
    std::vector<int64_t> mark(n, -1);
    std::vector<int32_t> perm(n), iperm(n);   // position -> column, column -> position
    for (int64_t i = 0; i < n; ++i) perm[i] = iperm[i] = (int32_t)i;
    std::vector<int32_t> nz;
    nz.reserve(1024);
    std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> heap;   // positions
    std::vector<Entry> lower, upper;

    HostFactor& F = *out;
    F.n = n;
    F.l_ptr.assign(1, 0);
    F.u_ptr.assign(1, 0);
    F.l_col.clear(); F.l_val.clear(); F.u_col.clear(); F.u_val.clear();
    F.repaired = 0;
    F.pivots = 0;
    const double floor_rel = 1e-14;

    for (int64_t i = 0; i < n; ++i) {
        const int64_t a0 = row_ptr[i], a1 = row_ptr[i + 1];
        double rowinf = 0.0;
        nz.clear();
        for (int64_t t = a0; t < a1; ++t) {
            const int32_t c = col[t];
            const double re = val[2 * t], im = val[2 * t + 1];
            rowinf = std::max(rowinf, std::sqrt(re * re + im * im));
            if (mark[c] != i) {
                mark[c] = i;
                wre[c] = re; wim[c] = im;
                nz.push_back(c);
                if (iperm[c] < i) heap.push(iperm[c]);
            } else {
                wre[c] += re; wim[c] += im;
            }
        }
        const double tau = drop_tol * rowinf;
        const double tau2 = tau * tau;
        const int64_t nnz_row = a1 - a0;
        const int64_t lfil = capped ? std::max<int64_t>(0, (int64_t)std::floor((fill_factor * (double)nnz_row - 1.0) / 2.0))
                                    : INT64_MAX;

        int32_t last = -1;
        while (!heap.empty()) {
            const int32_t k = heap.top();   // position of the pivot row
            heap.pop();
            if (k == last) continue;
            last = k;
            const int32_t c = perm[k];
            const double xr = wre[c], xi = wim[c];
            if (xr == 0.0 && xi == 0.0) continue;
            const int64_t u0 = F.u_ptr[k];
            const double dr = F.u_val[2 * u0], di = F.u_val[2 * u0 + 1];
            const double den = dr * dr + di * di;
            const double mr = (xr * dr + xi * di) / den;
            const double mi = (xi * dr - xr * di) / den;
            if (mr * mr + mi * mi < tau2) {   // first dropping rule
                wre[c] = 0.0; wim[c] = 0.0;
                continue;
            }
            wre[c] = mr; wim[c] = mi;
            const int64_t u1 = F.u_ptr[k + 1];
            for (int64_t t = u0 + 1; t < u1; ++t) {
                const int32_t cc = F.u_col[t];
                const double ur = F.u_val[2 * t], ui = F.u_val[2 * t + 1];
                const double pr = mr * ur - mi * ui;
                const double pi = mr * ui + mi * ur;
                if (mark[cc] == i) {
                    wre[cc] -= pr; wim[cc] -= pi;
                } else {
                    mark[cc] = i;
                    wre[cc] = -pr; wim[cc] = -pi;
                    nz.push_back(cc);
                    if (iperm[cc] < i) heap.push(iperm[cc]);
                }
            }
        }

        // second dropping rule
        lower.clear(); upper.clear();
        int32_t dcol = perm[i];
        double dgr = 0.0, dgi = 0.0;
        if (mark[dcol] == i) { dgr = wre[dcol]; dgi = wim[dcol]; }
        for (int32_t c : nz) {
            if (c == dcol) continue;
            const double re = wre[c], im = wim[c];
            const double m2 = re * re + im * im;
            if (m2 == 0.0 || m2 < tau2) continue;
            const int32_t p = iperm[c];
            (p < i ? lower : upper).push_back(Entry{c, p, re, im});
        }
        // threshold column pivoting on the upper part
        if (pivoting && !upper.empty()) {
            size_t best = 0;
            for (size_t t = 1; t < upper.size(); ++t)
                if (keep_before(upper[t], upper[best])) best = t;
            const double dm2 = dgr * dgr + dgi * dgi;
            if (dm2 < permtol * permtol * upper[best].mag2()) {
                const Entry e = upper[best];
                const int32_t p2 = e.pos;
                perm[i] = e.col; perm[p2] = dcol;
                iperm[e.col] = (int32_t)i; iperm[dcol] = p2;
                upper[best] = Entry{dcol, p2, dgr, dgi};
                if (dm2 == 0.0 || dm2 < tau2) {   // the old diagonal is subject to the dropping rule
                    upper[best] = upper.back();
                    upper.pop_back();
                }
                dcol = e.col; dgr = e.re; dgi = e.im;
                F.pivots++;
            }
        }
        if ((int64_t)lower.size() > lfil) {
            std::nth_element(lower.begin(), lower.begin() + lfil, lower.end(), keep_before);
            lower.resize(lfil);
        }
        if ((int64_t)upper.size() > lfil) {
            std::nth_element(upper.begin(), upper.begin() + lfil, upper.end(), keep_before);
            upper.resize(lfil);
        }
        std::sort(lower.begin(), lower.end(), [](const Entry& a, const Entry& b) { return a.pos < b.pos; });

        if (!std::isfinite(dgr) || !std::isfinite(dgi)) {
            if (err) *err = "ILUT breakdown: non-finite pivot in row " + std::to_string(i) +
                            " (the incomplete factorisation is unstable for this drop tolerance and fill)";
            return 1;
        }
        for (const Entry& e : upper)
            if (!std::isfinite(e.re) || !std::isfinite(e.im)) {
                if (err) *err = "ILUT breakdown: non-finite entry in row " + std::to_string(i);
                return 1;
            }
        const double fl = floor_rel * rowinf;
        const double dmag = std::sqrt(dgr * dgr + dgi * dgi);
        if (dmag < fl || dmag == 0.0) {
            if (dmag > 0.0) { dgr = fl * dgr / dmag; dgi = fl * dgi / dmag; }
            else if (fl > 0.0) { dgr = fl; dgi = 0.0; }
            else { dgr = 1.0; dgi = 0.0; }
            F.repaired++;
        }
        for (const Entry& e : lower) {   // positions < i are final
            F.l_col.push_back(e.pos);
            F.l_val.push_back(e.re); F.l_val.push_back(e.im);
        }
        F.l_ptr.push_back((int64_t)F.l_col.size());
        F.u_col.push_back(dcol);   // original columns until the end
        F.u_val.push_back(dgr); F.u_val.push_back(dgi);
        for (const Entry& e : upper) {
            F.u_col.push_back(e.col);
            F.u_val.push_back(e.re); F.u_val.push_back(e.im);
        }
        F.u_ptr.push_back((int64_t)F.u_col.size());
        for (int32_t c : nz) { wre[c] = 0.0; wim[c] = 0.0; }
    }
    // U to position coordinates, sorted (diagonal first)
    std::vector<std::pair<int32_t, int64_t>> tmp;
    std::vector<double> vtmp;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t u0 = F.u_ptr[i], u1 = F.u_ptr[i + 1];
        tmp.clear();
        for (int64_t t = u0; t < u1; ++t) tmp.emplace_back(iperm[F.u_col[t]], t);
        std::sort(tmp.begin() + 1, tmp.end());
        vtmp.assign(2 * (u1 - u0), 0.0);
        for (int64_t q = 0; q < u1 - u0; ++q) {
            vtmp[2 * q] = F.u_val[2 * tmp[q].second];
            vtmp[2 * q + 1] = F.u_val[2 * tmp[q].second + 1];
        }
        for (int64_t q = 0; q < u1 - u0; ++q) {
            F.u_col[u0 + q] = tmp[q].first;
            F.u_val[2 * (u0 + q)] = vtmp[2 * q];
            F.u_val[2 * (u0 + q) + 1] = vtmp[2 * q + 1];
        }
    }
    F.perm = perm;
    return 0;
}

}  // namespace omss
