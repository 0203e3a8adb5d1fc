// Reordering before conversion (section "Matrix permutation/reordering": a
// Cuthill-McKee breadth-first renumbering places coupled rows and columns
// next to each other, which raises the values per block).
//
// spc_rcm_order computes the reverse Cuthill-McKee order of the pattern of
// A + A^T on the host: the search is a sequential queue walk, and its cost
// (one pass over the pattern) is small beside the conversion it prepares.
// The pattern is copied from the device, symmetrized and deduplicated by
// host threads, walked, and the order is copied back.
//
// Definition (every implementation that follows it gives the same order):
//   G      pattern of A + A^T without the diagonal; deg(v) = distinct
//          neighbours of v;
//   start  the unnumbered vertex of smallest degree, smallest index on ties;
//   BFS    vertices leave the queue in order; each numbers its unnumbered
//          neighbours in (degree, index) order and queues them; an empty
//          queue with vertices left starts again from a new start vertex;
//   RCM    the order reversed: perm[new] = old.
#include <algorithm>
#include <thread>
#include <vector>

#include "common.hpp"

namespace spc {
namespace {

// Runs f(lo, hi) on up to `threads` host threads over [0, n).
template <class F>
void parallel_ranges(int64_t n, int threads, F &&f) {
    if (threads <= 1 || n < 4096) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> pool;
    const int64_t step = (n + threads - 1) / threads;
    for (int t = 0; t < threads; ++t) {
        const int64_t lo = t * step, hi = std::min<int64_t>(n, lo + step);
        if (lo >= hi) break;
        pool.emplace_back([&f, lo, hi] { f(lo, hi); });
    }
    for (auto &th : pool) th.join();
}

int host_threads() {
    const unsigned h = std::thread::hardware_concurrency();
    return (int)std::min<unsigned>(h ? h : 1, 16);
}

}  // namespace
}  // namespace spc

using namespace spc;

extern "C" spc_status spc_rcm_order(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colidx,
                                    int32_t *perm_out, hipStream_t stream) {
    SPC_REQUIRE(n >= 0 && nnz >= 0, SPC_ERR_INVALID_ARG, "negative size");
    SPC_REQUIRE(n < (int64_t(1) << 31) && nnz < (int64_t(1) << 31), SPC_ERR_OVERFLOW,
                "sizes exceed the int32 index range");
    if (n == 0) return SPC_OK;
    SPC_REQUIRE(rowptr && perm_out && (colidx || nnz == 0), SPC_ERR_INVALID_ARG, "null argument");
    std::vector<int32_t> rp((size_t)n + 1), ci((size_t)nnz);
    SPC_HIP(hipMemcpyAsync(rp.data(), rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, stream));
    if (nnz) SPC_HIP(hipMemcpyAsync(ci.data(), colidx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, stream));
    SPC_HIP(hipStreamSynchronize(stream));
    SPC_REQUIRE(rp[0] == 0 && rp[n] == nnz, SPC_ERR_INDEX_RANGE, "rowptr must run from 0 to nnz");
    for (int64_t i = 0; i < n; ++i)
        SPC_REQUIRE(rp[i] <= rp[i + 1], SPC_ERR_INDEX_RANGE, "rowptr decreases at row %lld", (long long)i);
    for (int64_t p = 0; p < nnz; ++p)
        SPC_REQUIRE(ci[p] >= 0 && ci[p] < n, SPC_ERR_INDEX_RANGE, "column %d outside [0, %lld)", ci[p],
                    (long long)n);
    const int threads = host_threads();

    // symmetric pattern: row i gets every j with (i, j) or (j, i) stored, i != j
    std::vector<int64_t> cnt((size_t)n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] != i) {
                ++cnt[i + 1];
                ++cnt[(size_t)ci[p] + 1];
            }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    std::vector<int32_t> adj((size_t)cnt[n]);
    {
        std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
                if (ci[p] != i) {
                    adj[(size_t)fill[i]++] = ci[p];
                    adj[(size_t)fill[ci[p]]++] = (int32_t)i;
                }
    }
    // sort and deduplicate each row; deg = distinct neighbours
    std::vector<int32_t> deg((size_t)n);
    parallel_ranges(n, threads, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            auto b = adj.begin() + cnt[i], e = adj.begin() + cnt[i + 1];
            std::sort(b, e);
            deg[i] = (int32_t)(std::unique(b, e) - b);
        }
    });

    // Cuthill-McKee: breadth-first, neighbours in (degree, index) order
    std::vector<int32_t> order;
    order.reserve((size_t)n);
    std::vector<char> numbered((size_t)n, 0);
    // start candidates in (degree, index) order; the next start is the first
    // of them still unnumbered
    std::vector<int32_t> by_deg((size_t)n);
    for (int64_t i = 0; i < n; ++i) by_deg[i] = (int32_t)i;
    std::stable_sort(by_deg.begin(), by_deg.end(), [&](int32_t a, int32_t b) { return deg[a] < deg[b]; });
    size_t next_start = 0;
    std::vector<int32_t> nb;
    size_t head = 0;
    while (order.size() < (size_t)n) {
        while (numbered[by_deg[next_start]]) ++next_start;
        const int32_t s = by_deg[next_start];
        numbered[s] = 1;
        order.push_back(s);
        while (head < order.size()) {
            const int32_t v = order[head++];
            nb.clear();
            for (int64_t p = cnt[v]; p < cnt[v] + deg[v]; ++p)
                if (!numbered[adj[p]]) nb.push_back(adj[p]);
            std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
                return deg[a] != deg[b] ? deg[a] < deg[b] : a < b;
            });
            for (int32_t w : nb) {
                numbered[w] = 1;
                order.push_back(w);
            }
        }
    }
    std::reverse(order.begin(), order.end());
    SPC_HIP(hipMemcpyAsync(perm_out, order.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, stream));
    SPC_HIP(hipStreamSynchronize(stream));
    return SPC_OK;
}
