// Host-only part of the library (see mc_host.h): the error slot, default
// options, option checks and the exact checks of host CSR inputs (paper,
// Section 2 "Basic Concepts": an undirected graph with non-negative integer
// edge weights, given here as a symmetric CSR).
#include "mc_host.h"

#include <algorithm>
#include <cstring>
#include <utility>
#include <vector>

namespace {
thread_local std::string g_err;
}

std::string& mc_error_slot() { return g_err; }

mc_status mc_fail(mc_status code, const std::string& msg) {
    g_err = msg;
    return code;
}

extern "C" const char* mc_last_error(void) { return g_err.c_str(); }

extern "C" void mc_default_options(mc_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->seed = 1;
    o->heuristic_min_n = 10000;
    o->lp_iters = 2;
    o->pr_tri_deg_cap = 16;
    o->capforest_passes = 0;
    o->pass_len_cap = 0;
    o->capforest_mode = MC_CF_AUTO;
    o->levels_min_n = 0;
    o->deterministic = 0;
    o->validate = 0;
    o->batch_pass_threads = 0;
    o->batch_lp = 0;
}

mc_status mc_options_check(const mc_options* o) {
    if (!o) return mc_fail(MC_E_INVALID_ARG, "options: NULL");
    const int32_t t = o->batch_pass_threads;
    if (t != 0 && t != 64 && t != 128 && t != 256 && t != 512 && t != 1024)
        return mc_fail(MC_E_INVALID_ARG, "options: batch_pass_threads must be 0, 64, 128, 256, 512 or 1024");
    if (o->batch_lp < 0 || o->batch_lp > 2) return mc_fail(MC_E_INVALID_ARG, "options: batch_lp must be 0, 1 or 2");
    if (o->pr_tri_deg_cap < 0 || o->pr_tri_deg_cap > 64)
        return mc_fail(MC_E_INVALID_ARG, "options: pr_tri_deg_cap must be in [0, 64]");
    if (o->lp_iters < 0) return mc_fail(MC_E_INVALID_ARG, "options: lp_iters must be >= 0");
    if (o->capforest_passes < 0) return mc_fail(MC_E_INVALID_ARG, "options: capforest_passes must be >= 0");
    if (o->capforest_mode != MC_CF_PRIVATE && o->capforest_mode != MC_CF_SHARED && o->capforest_mode != MC_CF_AUTO)
        return mc_fail(MC_E_INVALID_ARG, "options: capforest_mode must be MC_CF_PRIVATE, MC_CF_SHARED or MC_CF_AUTO");
    if (o->levels_min_n < 0) return mc_fail(MC_E_INVALID_ARG, "options: levels_min_n must be >= 0");
    if (o->deterministic != 0 && o->deterministic != 1)
        return mc_fail(MC_E_INVALID_ARG, "options: deterministic must be 0 or 1");
    if (o->validate != 0 && o->validate != 1) return mc_fail(MC_E_INVALID_ARG, "options: validate must be 0 or 1");
    if (o->finish_max_n > 1024) return mc_fail(MC_E_INVALID_ARG, "options: finish_max_n must be at most 1024");
    if (o->queue < 0 || o->queue > 2) return mc_fail(MC_E_INVALID_ARG, "options: queue must be 0, 1 or 2");
    if (o->contract_mode < 0 || o->contract_mode > 1)
        return mc_fail(MC_E_INVALID_ARG, "options: contract_mode must be 0 (hash) or 1 (sort)");
    return MC_OK;
}

mc_status check_host_csr(const mc_csr* g, bool symmetric) {
    if (!g) return mc_fail(MC_E_INVALID_ARG, "graph is NULL");
    if (g->n < 2) return mc_fail(MC_E_INVALID_ARG, "need n >= 2");
    if (g->nnz < 0 || !g->row_ptr || (g->nnz > 0 && (!g->col || !g->w)))
        return mc_fail(MC_E_INVALID_ARG, "bad CSR pointers");
    const int32_t n = g->n, nnz = g->nnz;
    if (g->row_ptr[0] != 0 || g->row_ptr[n] != nnz)
        return mc_fail(MC_E_BAD_GRAPH, "row_ptr[0] must be 0 and row_ptr[n] = nnz");
    for (int32_t v = 0; v < n; v++)
        if (g->row_ptr[v + 1] < g->row_ptr[v]) return mc_fail(MC_E_BAD_GRAPH, "row_ptr is not non-decreasing");
    const unsigned long long cap = 1ULL << 62;
    unsigned long long s = 0;
    for (int32_t j = 0; j < nnz; j++) {
        if (g->col[j] < 0 || g->col[j] >= n) return mc_fail(MC_E_BAD_GRAPH, "col out of range");
        if (g->w[j] < 0) return mc_fail(MC_E_BAD_GRAPH, "negative weight");
        // s < 2^62 and w < 2^63 before the add, so the sum cannot wrap
        s += (unsigned long long)g->w[j];
        if (s >= cap) return mc_fail(MC_E_OVERFLOW, "total weight must be below 2^62");
    }
    if (symmetric) {
        // fold each row (loops dropped, parallel entries summed), then every
        // (u, v, s) must have a matching (v, u, s)
        std::vector<std::pair<int64_t, int64_t>> e;  // key u*n+v -> weight
        e.reserve((size_t)nnz);
        for (int32_t u = 0; u < n; u++)
            for (int32_t j = g->row_ptr[u]; j < g->row_ptr[u + 1]; j++)
                if (g->col[j] != u) e.push_back({(int64_t)u * n + g->col[j], g->w[j]});
        std::sort(e.begin(), e.end());
        std::vector<std::pair<int64_t, int64_t>> f;
        for (size_t i = 0; i < e.size();) {
            size_t k = i;
            int64_t t = 0;
            while (k < e.size() && e[k].first == e[i].first) t += e[k++].second;
            f.push_back({e[i].first, t});
            i = k;
        }
        for (const auto& p : f) {
            const int64_t u = p.first / n, v = p.first % n;
            auto it = std::lower_bound(f.begin(), f.end(), std::make_pair(v * n + u, (int64_t)INT64_MIN));
            if (it == f.end() || it->first != v * n + u || it->second != p.second)
                return mc_fail(MC_E_BAD_GRAPH, "edge list is not symmetric");
        }
    }
    return MC_OK;
}

extern "C" mc_status mc_check_graph(const mc_csr* g, int32_t symmetric) {
    if (g && g->location != MC_HOST) return mc_fail(MC_E_INVALID_ARG, "mc_check_graph: host graphs only");
    return check_host_csr(g, symmetric != 0);
}
