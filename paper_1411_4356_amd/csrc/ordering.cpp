// Host graph algorithms on CSR patterns.
//
// Reverse Cuthill-McKee follows Sec. III: the graph is the structure of
// A + A^T; a breadth-first search starts at an unvisited node of lowest degree
// (degree = number of nonzeros in the row of A + A^T, diagonal included; ties
// to the lower index) and visits the unvisited neighbours of each node in
// order of increasing degree (ties to the lower index); this is repeated for
// every connected component and the visiting order is reversed.
#include "ordering.hpp"

#include <algorithm>
#include <cstdlib>
#include <numeric>
#include <thread>

namespace omss {

int host_threads() {
    if (const char* e = std::getenv("OMSS_HOST_THREADS")) {
        int v = std::atoi(e);
        if (v > 0) return v;
    }
    unsigned h = std::thread::hardware_concurrency();
    return h == 0 ? 1 : (int)std::min<unsigned>(h, 16);
}

template <typename F>
static void parallel_rows(int64_t n, F&& f) {
    int T = host_threads();
    if (n < 200000 || T <= 1) { f(0, n); return; }
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t) {
        int64_t a = n * t / T, b = n * (t + 1) / T;
        th.emplace_back([&, a, b] { f(a, b); });
    }
    for (auto& x : th) x.join();
}

BandStats band_stats(int64_t n, const int64_t* row_ptr, const int32_t* col) {
    BandStats s{0, 0, 0, 0, 0, 0};
    std::vector<int64_t> colmax(n, 0);
    for (int64_t i = 0; i < n; ++i) {
        int64_t rowup = 0;
        for (int64_t t = row_ptr[i]; t < row_ptr[i + 1]; ++t) {
            const int64_t j = col[t];
            const int64_t dj = j - i;
            if (dj > rowup) rowup = dj;
            if (dj > s.ub) s.ub = dj;
            if (-dj > s.lb) s.lb = -dj;
            if (-dj > colmax[j]) colmax[j] = -dj;
        }
        s.up += rowup;
    }
    for (int64_t j = 0; j < n; ++j) s.lp += colmax[j];
    s.B = s.ub + s.lb + 1;
    s.P = s.up + s.lp;
    return s;
}

void transpose_pattern(int64_t n, const int64_t* row_ptr, const int32_t* col, std::vector<int64_t>& t_ptr,
                       std::vector<int32_t>& t_col, std::vector<int64_t>& src) {
    const int64_t nnz = row_ptr[n];
    t_ptr.assign(n + 1, 0);
    for (int64_t t = 0; t < nnz; ++t) t_ptr[col[t] + 1]++;
    for (int64_t j = 0; j < n; ++j) t_ptr[j + 1] += t_ptr[j];
    t_col.resize(nnz);
    src.resize(nnz);
    std::vector<int64_t> pos(t_ptr.begin(), t_ptr.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t t = row_ptr[i]; t < row_ptr[i + 1]; ++t) {
            const int64_t d = pos[col[t]]++;
            t_col[d] = (int32_t)i;   // rows visited in increasing order: sorted
            src[d] = t;
        }
}

void rcm_order(int64_t n, const int64_t* row_ptr, const int32_t* col, std::vector<int32_t>& perm) {
    // structure of A + A^T: merge row i of A with row i of A^T
    std::vector<int64_t> t_ptr, tsrc;
    std::vector<int32_t> t_col;
    transpose_pattern(n, row_ptr, col, t_ptr, t_col, tsrc);
    tsrc.clear();
    tsrc.shrink_to_fit();
    std::vector<int64_t> s_ptr(n + 1, 0);
    parallel_rows(n, [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) {
            int64_t x = row_ptr[i], xe = row_ptr[i + 1], y = t_ptr[i], ye = t_ptr[i + 1], c = 0;
            while (x < xe || y < ye) {
                if (y >= ye || (x < xe && col[x] < t_col[y])) ++x;
                else if (x >= xe || t_col[y] < col[x]) ++y;
                else { ++x; ++y; }
                ++c;
            }
            s_ptr[i + 1] = c;
        }
    });
    for (int64_t i = 0; i < n; ++i) s_ptr[i + 1] += s_ptr[i];
    std::vector<int32_t> s_col(s_ptr[n]);
    parallel_rows(n, [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) {
            int64_t x = row_ptr[i], xe = row_ptr[i + 1], y = t_ptr[i], ye = t_ptr[i + 1], o = s_ptr[i];
            while (x < xe || y < ye) {
                if (y >= ye || (x < xe && col[x] < t_col[y])) s_col[o++] = col[x++];
                else if (x >= xe || t_col[y] < col[x]) s_col[o++] = t_col[y++];
                else { s_col[o++] = col[x]; ++x; ++y; }
            }
        }
    });
    t_col.clear();
    t_col.shrink_to_fit();
    std::vector<int32_t> deg(n);
    for (int64_t i = 0; i < n; ++i) deg[i] = (int32_t)(s_ptr[i + 1] - s_ptr[i]);

    // start candidates in ascending (degree, index): counting sort by degree
    int32_t maxdeg = 0;
    for (int64_t i = 0; i < n; ++i) maxdeg = std::max(maxdeg, deg[i]);
    std::vector<int64_t> bucket(maxdeg + 2, 0);
    for (int64_t i = 0; i < n; ++i) bucket[deg[i] + 1]++;
    for (int32_t d = 0; d <= maxdeg; ++d) bucket[d + 1] += bucket[d];
    std::vector<int32_t> starts(n);
    for (int64_t i = 0; i < n; ++i) starts[bucket[deg[i]]++] = (int32_t)i;

    std::vector<char> visited(n, 0);
    std::vector<int32_t> order;
    order.reserve(n);
    std::vector<int32_t> nb;
    int64_t si = 0;
    while ((int64_t)order.size() < n) {
        while (visited[starts[si]]) ++si;
        const int32_t s0 = starts[si];
        visited[s0] = 1;
        size_t head = order.size();
        order.push_back(s0);
        while (head < order.size()) {
            const int32_t v = order[head++];
            nb.clear();
            for (int64_t t = s_ptr[v]; t < s_ptr[v + 1]; ++t) {
                const int32_t u = s_col[t];
                if (!visited[u]) nb.push_back(u);
            }
            std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
                return deg[a] != deg[b] ? deg[a] < deg[b] : a < b;
            });
            for (int32_t u : nb) {
                visited[u] = 1;
                order.push_back(u);
            }
        }
    }
    perm.assign(order.rbegin(), order.rend());
}

void permute_pattern(int64_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* perm,
                     std::vector<int64_t>& new_ptr, std::vector<int32_t>& new_col, std::vector<int32_t>& src) {
    std::vector<int32_t> iperm(n);
    for (int64_t i = 0; i < n; ++i) iperm[perm[i]] = (int32_t)i;
    new_ptr.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) new_ptr[i + 1] = new_ptr[i] + (row_ptr[perm[i] + 1] - row_ptr[perm[i]]);
    const int64_t nnz = new_ptr[n];
    new_col.resize(nnz);
    src.resize(nnz);
    parallel_rows(n, [&](int64_t a, int64_t b) {
        std::vector<std::pair<int32_t, int32_t>> tmp;
        for (int64_t i = a; i < b; ++i) {
            const int64_t r = perm[i];
            tmp.clear();
            for (int64_t t = row_ptr[r]; t < row_ptr[r + 1]; ++t) tmp.emplace_back(iperm[col[t]], (int32_t)t);
            std::sort(tmp.begin(), tmp.end());
            int64_t o = new_ptr[i];
            for (auto& e : tmp) { new_col[o] = e.first; src[o] = e.second; ++o; }
        }
    });
}

}  // namespace omss
