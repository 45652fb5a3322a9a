// Dual-threshold incomplete LU factorisation on the host (Sec. II).
//
// Row-wise ILUT: row i is copied into a dense work row w, eliminated against
// the already-final rows of U in increasing column order (fill included),
// with the multiplier dropped when |w_k| < tau_i = d * ||a_i||_inf (first
// rule); afterwards every off-diagonal entry below tau_i is dropped (second
// rule) and at most lfil_i = floor((p * nnz(a_i) - 1) / 2) entries are kept in
// each triangle, largest magnitude first, ties to the lower column.  No
// pivoting; a pivot below 1e-14 * ||a_i||_inf is raised to that floor (same
// phase) and counted.  Magnitudes are compared as squared moduli.
//
// The factor is produced in CSR: L strictly lower (unit diagonal implied),
// U with the diagonal as the first entry of every row.
#include "ilut.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <queue>
#include <vector>

namespace omss {

namespace {

struct Entry {
    int32_t col;
    double re, im;
    double mag2() const { return re * re + im * im; }
};

// total order used by the per-row cap: larger modulus first, then lower column
inline bool keep_before(const Entry& a, const Entry& b) {
    double ma = a.mag2(), mb = b.mag2();
    if (ma != mb) return ma > mb;
    return a.col < b.col;
}

}  // namespace

int ilut_factor_host(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                     double drop_tol, double fill_factor, HostFactor* out, std::string* err) {
    const bool capped = std::isfinite(fill_factor);
    std::vector<double> wre(n, 0.0), wim(n, 0.0);
    std::vector<int64_t> mark(n, -1);
    std::vector<int32_t> nz;           // columns present in w
    nz.reserve(1024);
    std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> heap;
    std::vector<Entry> lower, upper;

    HostFactor& F = *out;
    F.n = n;
    F.l_ptr.assign(1, 0);
    F.u_ptr.assign(1, 0);
    F.l_col.clear(); F.l_val.clear(); F.u_col.clear(); F.u_val.clear();
    F.repaired = 0;
    const double floor_rel = 1e-14;

    for (int64_t i = 0; i < n; ++i) {
        const int64_t a0 = row_ptr[i], a1 = row_ptr[i + 1];
        double rowinf = 0.0;
        nz.clear();
        for (int64_t t = a0; t < a1; ++t) {
            int32_t c = col[t];
            double re = val[2 * t], im = val[2 * t + 1];
            rowinf = std::max(rowinf, std::sqrt(re * re + im * im));
            if (mark[c] != i) {
                mark[c] = i;
                wre[c] = re; wim[c] = im;
                nz.push_back(c);
                if (c < i) heap.push(c);
            } else {  // duplicate entries are summed
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
            int32_t k = heap.top();
            heap.pop();
            if (k == last) continue;  // a column may be pushed once per row only, but be safe
            last = k;
            double xr = wre[k], xi = wim[k];
            if (xr == 0.0 && xi == 0.0) continue;
            // multiplier m = w_k / u_kk
            const int64_t u0 = F.u_ptr[k];
            const double dr = F.u_val[2 * u0], di = F.u_val[2 * u0 + 1];
            const double den = dr * dr + di * di;
            const double mr = (xr * dr + xi * di) / den;
            const double mi = (xi * dr - xr * di) / den;
            if (mr * mr + mi * mi < tau2) {  // first dropping rule
                wre[k] = 0.0; wim[k] = 0.0;
                continue;
            }
            wre[k] = mr; wim[k] = mi;
            const int64_t u1 = F.u_ptr[k + 1];
            for (int64_t t = u0 + 1; t < u1; ++t) {
                const int32_t c = F.u_col[t];
                const double ur = F.u_val[2 * t], ui = F.u_val[2 * t + 1];
                const double pr = mr * ur - mi * ui;
                const double pi = mr * ui + mi * ur;
                if (mark[c] == i) {
                    wre[c] -= pr; wim[c] -= pi;
                } else {
                    mark[c] = i;
                    wre[c] = -pr; wim[c] = -pi;
                    nz.push_back(c);
                    if (c < i) heap.push(c);
                }
            }
        }

        // second dropping rule and the per-row cap
        lower.clear(); upper.clear();
        double dgr = 0.0, dgi = 0.0;
        for (int32_t c : nz) {
            const double re = wre[c], im = wim[c];
            if (c == i) { dgr = re; dgi = im; continue; }
            const double m2 = re * re + im * im;
            if (m2 == 0.0 || m2 < tau2) continue;
            (c < i ? lower : upper).push_back(Entry{c, re, im});
        }
        if (mark[i] != i) { dgr = 0.0; dgi = 0.0; }
        if ((int64_t)lower.size() > lfil) {
            std::nth_element(lower.begin(), lower.begin() + lfil, lower.end(), keep_before);
            lower.resize(lfil);
        }
        if ((int64_t)upper.size() > lfil) {
            std::nth_element(upper.begin(), upper.begin() + lfil, upper.end(), keep_before);
            upper.resize(lfil);
        }
        auto by_col = [](const Entry& a, const Entry& b) { return a.col < b.col; };
        std::sort(lower.begin(), lower.end(), by_col);
        std::sort(upper.begin(), upper.end(), by_col);

        const double fl = floor_rel * rowinf;
        const double dmag = std::sqrt(dgr * dgr + dgi * dgi);
        if (dmag < fl || dmag == 0.0) {
            if (dmag > 0.0) { dgr = fl * dgr / dmag; dgi = fl * dgi / dmag; }
            else if (fl > 0.0) { dgr = fl; dgi = 0.0; }
            else { dgr = 1.0; dgi = 0.0; }
            F.repaired++;
        }
        for (const Entry& e : lower) {
            F.l_col.push_back(e.col);
            F.l_val.push_back(e.re); F.l_val.push_back(e.im);
        }
        F.l_ptr.push_back((int64_t)F.l_col.size());
        F.u_col.push_back((int32_t)i);
        F.u_val.push_back(dgr); F.u_val.push_back(dgi);
        for (const Entry& e : upper) {
            F.u_col.push_back(e.col);
            F.u_val.push_back(e.re); F.u_val.push_back(e.im);
        }
        F.u_ptr.push_back((int64_t)F.u_col.size());
        for (int32_t c : nz) { wre[c] = 0.0; wim[c] = 0.0; }
    }
    (void)err;
    return 0;
}

}  // namespace omss
