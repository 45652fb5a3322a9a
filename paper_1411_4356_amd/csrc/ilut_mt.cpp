// Row-pipelined multi-threaded ILUT on the host (same factor as
// ilut_factor_host without pivoting, bit for bit).
//
// Thread t factors rows t, t+T, t+2T, ... in increasing order.  Row i is
// eliminated against rows k < i in increasing k (as in the sequential
// algorithm); before using row k of U it waits for that row's ready flag.
// Progress is guaranteed: the smallest unfinished row r is being factored by
// its own thread (all that thread's earlier rows are smaller, hence done) and
// r waits only for rows < r.  Finished rows are stored in per-thread chunked
// arenas that never move, so other threads can read them while the owner keeps
// appending; the CSR factor is assembled at the end.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <queue>
#include <string>
#include <thread>
#include <vector>

#include "ilut.hpp"

namespace omss {

namespace {

struct Entry {
    int32_t col;
    double re, im;
    double mag2() const { return re * re + im * im; }
};

inline bool keep_before(const Entry& a, const Entry& b) {
    const double ma = a.mag2(), mb = b.mag2();
    if (ma != mb) return ma > mb;
    return a.col < b.col;
}

// append-only storage whose existing elements never move
struct Arena {
    static constexpr size_t CHUNK = (size_t)1 << 22;
    std::vector<std::unique_ptr<int32_t[]>> cols;
    std::vector<std::unique_ptr<double[]>> vals;
    size_t used = CHUNK;
    // returns storage for `len` entries, contiguous
    void reserve(size_t len, int32_t*& c, double*& v) {
        if (len == 0) { c = nullptr; v = nullptr; return; }
        if (used + len > CHUNK) {
            const size_t sz = std::max(CHUNK, len);
            cols.emplace_back(new int32_t[sz]);
            vals.emplace_back(new double[2 * sz]);
            used = 0;
            if (len > CHUNK) {   // oversized row gets its own chunk
                c = cols.back().get();
                v = vals.back().get();
                used = CHUNK;
                return;
            }
        }
        c = cols.back().get() + used;
        v = vals.back().get() + 2 * used;
        used += len;
    }
};

struct RowRef {
    const int32_t* col = nullptr;
    const double* val = nullptr;
    int64_t len = 0;
};

}  // namespace

int ilut_factor_host_mt(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val, double drop_tol,
                        double fill_factor, int threads, HostFactor* out, std::string* err) {
    const bool capped = std::isfinite(fill_factor);
    const int T = std::max(1, threads);
    std::vector<RowRef> Lr(n), Ur(n);          // U rows: diagonal first, then columns > i (sorted)
    std::unique_ptr<std::atomic<uint8_t>[]> ready(new std::atomic<uint8_t>[n]);
    for (int64_t i = 0; i < n; ++i) ready[i].store(0, std::memory_order_relaxed);
    std::atomic<int> failed{0};
    std::vector<std::string> errs(T);
    std::vector<int64_t> repaired(T, 0);
    const bool verbose = std::getenv("OMSS_VERBOSE") != nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    std::atomic<int64_t> rows_done{0};
    std::vector<Arena> arenas(T);

    auto worker = [&](int t) {
        std::vector<double> wre(n, 0.0), wim(n, 0.0);
        std::vector<int64_t> mark(n, -1);
        std::vector<int32_t> nz;
        nz.reserve(1024);
        std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> heap;
        std::vector<Entry> lower, upper;
        Arena& arena = arenas[t];
        const double floor_rel = 1e-14;
        double last_report = 0.0;
        for (int64_t i = t; i < n; i += T) {
            if (failed.load(std::memory_order_relaxed)) return;
            const int64_t a0 = row_ptr[i], a1 = row_ptr[i + 1];
            double rowinf = 0.0;
            nz.clear();
            for (int64_t q = a0; q < a1; ++q) {
                const int32_t c = col[q];
                const double re = val[2 * q], im = val[2 * q + 1];
                rowinf = std::max(rowinf, std::sqrt(re * re + im * im));
                if (mark[c] != i) {
                    mark[c] = i;
                    wre[c] = re; wim[c] = im;
                    nz.push_back(c);
                    if (c < i) heap.push(c);
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
                const int32_t k = heap.top();
                heap.pop();
                if (k == last) continue;
                last = k;
                const double xr = wre[k], xi = wim[k];
                if (xr == 0.0 && xi == 0.0) continue;
                // wait for row k of U
                if (!ready[k].load(std::memory_order_acquire)) {
                    int spins = 0;
                    while (!ready[k].load(std::memory_order_acquire)) {
                        if (failed.load(std::memory_order_relaxed)) return;
                        if (++spins > 64) std::this_thread::yield();
                    }
                }
                const RowRef& U = Ur[k];
                const double dr = U.val[0], di = U.val[1];
                const double den = dr * dr + di * di;
                const double mr = (xr * dr + xi * di) / den;
                const double mi = (xi * dr - xr * di) / den;
                if (mr * mr + mi * mi < tau2) {
                    wre[k] = 0.0; wim[k] = 0.0;
                    continue;
                }
                wre[k] = mr; wim[k] = mi;
                for (int64_t q = 1; q < U.len; ++q) {
                    const int32_t c = U.col[q];
                    const double ur = U.val[2 * q], ui = U.val[2 * q + 1];
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
            lower.clear(); upper.clear();
            double dgr = 0.0, dgi = 0.0;
            if (mark[i] == i) { dgr = wre[i]; dgi = wim[i]; }
            for (int32_t c : nz) {
                if (c == i) continue;
                const double re = wre[c], im = wim[c];
                const double m2 = re * re + im * im;
                if (m2 == 0.0 || m2 < tau2) continue;
                (c < i ? lower : upper).push_back(Entry{c, re, im});
            }
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
            bool bad = !std::isfinite(dgr) || !std::isfinite(dgi);
            for (const Entry& e : upper) bad = bad || !std::isfinite(e.re) || !std::isfinite(e.im);
            if (bad) {
                errs[t] = "ILUT breakdown: non-finite pivot or entry in row " + std::to_string(i) +
                          " (the incomplete factorisation is unstable for this drop tolerance and fill)";
                failed.store(1);
                return;
            }
            const double fl = floor_rel * rowinf;
            const double dmag = std::sqrt(dgr * dgr + dgi * dgi);
            if (dmag < fl || dmag == 0.0) {
                if (dmag > 0.0) { dgr = fl * dgr / dmag; dgi = fl * dgi / dmag; }
                else if (fl > 0.0) { dgr = fl; dgi = 0.0; }
                else { dgr = 1.0; dgi = 0.0; }
                repaired[t]++;
            }
            int32_t* c;
            double* v;
            arena.reserve(lower.size(), c, v);
            for (size_t q = 0; q < lower.size(); ++q) {
                c[q] = lower[q].col;
                v[2 * q] = lower[q].re;
                v[2 * q + 1] = lower[q].im;
            }
            Lr[i] = RowRef{c, v, (int64_t)lower.size()};
            arena.reserve(upper.size() + 1, c, v);
            c[0] = (int32_t)i;
            v[0] = dgr;
            v[1] = dgi;
            for (size_t q = 0; q < upper.size(); ++q) {
                c[q + 1] = upper[q].col;
                v[2 * (q + 1)] = upper[q].re;
                v[2 * (q + 1) + 1] = upper[q].im;
            }
            Ur[i] = RowRef{c, v, (int64_t)upper.size() + 1};
            ready[i].store(1, std::memory_order_release);
            for (int32_t cc : nz) { wre[cc] = 0.0; wim[cc] = 0.0; }
            if (verbose && t == 0) {
                const int64_t done = rows_done.fetch_add(T) + T;
                const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                if (el - last_report > 20.0) {
                    last_report = el;
                    fprintf(stderr, "[omss] ilut: ~%lld/%lld rows after %.0f s\n", (long long)std::min(done, n), (long long)n, el);
                }
            }
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < T; ++t) th.emplace_back(worker, t);
    worker(0);
    for (auto& x : th) x.join();
    if (failed.load()) {
        for (const std::string& e : errs)
            if (!e.empty()) { if (err) *err = e; break; }
        return 1;
    }
    // assemble the CSR factor
    HostFactor& F = *out;
    F.n = n;
    F.l_ptr.assign(n + 1, 0);
    F.u_ptr.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
        F.l_ptr[i + 1] = F.l_ptr[i] + Lr[i].len;
        F.u_ptr[i + 1] = F.u_ptr[i] + Ur[i].len;
    }
    F.l_col.resize(F.l_ptr[n]);
    F.l_val.resize(2 * F.l_ptr[n]);
    F.u_col.resize(F.u_ptr[n]);
    F.u_val.resize(2 * F.u_ptr[n]);
    auto copy_rows = [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) {
            std::copy(Lr[i].col, Lr[i].col + Lr[i].len, F.l_col.begin() + F.l_ptr[i]);
            std::copy(Lr[i].val, Lr[i].val + 2 * Lr[i].len, F.l_val.begin() + 2 * F.l_ptr[i]);
            std::copy(Ur[i].col, Ur[i].col + Ur[i].len, F.u_col.begin() + F.u_ptr[i]);
            std::copy(Ur[i].val, Ur[i].val + 2 * Ur[i].len, F.u_val.begin() + 2 * F.u_ptr[i]);
        }
    };
    {
        std::vector<std::thread> cp;
        for (int t = 0; t < T; ++t) cp.emplace_back(copy_rows, n * t / T, n * (t + 1) / T);
        for (auto& x : cp) x.join();
    }
    F.perm.resize(n);
    for (int64_t i = 0; i < n; ++i) F.perm[i] = (int32_t)i;
    F.repaired = 0;
    for (int64_t r : repaired) F.repaired += r;
    F.pivots = 0;
    return 0;
}

}  // namespace omss
