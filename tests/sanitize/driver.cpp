// Sanitizer driver (CPU only): exercises the oracle and the library's host
// validation layer under AddressSanitizer and UndefinedBehaviorSanitizer.
// Built with g++ by tests/test_sanitize.py; any sanitizer report or failed
// check ends the process with a non-zero status.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "mincut.h"

extern "C" {
int64_t orc_brute(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w, uint8_t* side);
int64_t orc_stoer_wagner(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w, uint8_t* side);
int64_t orc_noi(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w, uint8_t* side, int32_t* rounds);
int64_t orc_cut_value(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w, const uint8_t* side);
void orc_pr12(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w, int64_t lam, uint8_t* flag1,
              int32_t* ptr2);
void orc_pr34(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w, int64_t lam, int32_t D,
              const int32_t* ptr2, uint8_t* flag4, int32_t* part3, int32_t* acc3);
void orc_lp(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w, const int32_t* lab_in,
            int32_t* lab_out);
}

static int failures = 0;
#define CHECK(c) do { if (!(c)) { std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); failures++; } } while (0)

struct G {
    int32_t n = 0;
    std::vector<int32_t> rp, col;
    std::vector<int64_t> w;
    mc_csr csr() const { return mc_csr{n, (int32_t)col.size(), rp.data(), col.data(), w.data(), MC_HOST}; }
};

// symmetric CSR of a random graph (edge probability p/100, weights 0..wmax)
static G random_graph(int32_t n, int p, int64_t wmax, uint64_t seed) {
    uint64_t x = seed * 0x9E3779B97F4A7C15ULL + 1;
    auto next = [&]() { x ^= x << 13; x ^= x >> 7; x ^= x << 17; return x; };
    std::vector<std::vector<std::pair<int32_t, int64_t>>> adj(n);
    for (int32_t u = 0; u < n; u++)
        for (int32_t v = u + 1; v < n; v++)
            if ((int)(next() % 100) < p) {
                const int64_t c = (int64_t)(next() % (uint64_t)(wmax + 1));
                adj[u].push_back({v, c});
                adj[v].push_back({u, c});
            }
    G g;
    g.n = n;
    g.rp.push_back(0);
    for (int32_t u = 0; u < n; u++) {
        for (auto& e : adj[u]) { g.col.push_back(e.first); g.w.push_back(e.second); }
        g.rp.push_back((int32_t)g.col.size());
    }
    return g;
}

int main() {
    // oracle: three solvers agree, sides recompute, step oracles run clean
    for (uint64_t seed = 1; seed <= 60; seed++) {
        const int32_t n = 2 + (int32_t)(seed % 13);
        G g = random_graph(n, 40 + (int)(seed % 50), 9, seed);
        std::vector<uint8_t> s1(n), s2(n), s3(n);
        int32_t rounds = 0;
        const int64_t a = orc_brute(n, g.rp.data(), g.col.data(), g.w.data(), s1.data());
        const int64_t b = orc_stoer_wagner(n, g.rp.data(), g.col.data(), g.w.data(), s2.data());
        const int64_t c = orc_noi(n, g.rp.data(), g.col.data(), g.w.data(), s3.data(), &rounds);
        CHECK(a == b && b == c);
        CHECK(orc_cut_value(n, g.rp.data(), g.col.data(), g.w.data(), s2.data()) == b);
        CHECK(orc_cut_value(n, g.rp.data(), g.col.data(), g.w.data(), s3.data()) == c);
        std::vector<uint8_t> f1(g.col.size() + 1), f4(g.col.size() + 1);
        std::vector<int32_t> p2(n), p3(n), acc(n), lab(n), out(n);
        orc_pr12(n, g.rp.data(), g.col.data(), g.w.data(), a + 1, f1.data(), p2.data());
        orc_pr34(n, g.rp.data(), g.col.data(), g.w.data(), a + 1, 8, p2.data(), f4.data(), p3.data(), acc.data());
        for (int32_t v = 0; v < n; v++) lab[v] = v % 3;
        orc_lp(n, g.rp.data(), g.col.data(), g.w.data(), lab.data(), out.data());
    }
    // host validation layer
    {
        G g = random_graph(12, 60, 9, 77);
        mc_csr c = g.csr();
        CHECK(mc_check_graph(&c, 1) == MC_OK);
        CHECK(mc_check_graph(nullptr, 0) == MC_E_INVALID_ARG);
        mc_csr d = c;
        d.n = 1;
        CHECK(mc_check_graph(&d, 0) == MC_E_INVALID_ARG);
        d = c;
        d.location = MC_DEVICE;
        CHECK(mc_check_graph(&d, 0) == MC_E_INVALID_ARG);
        G h = g;
        h.rp[3] = h.rp[4] + 1;   // decreasing
        mc_csr e = h.csr();
        CHECK(mc_check_graph(&e, 0) == MC_E_BAD_GRAPH);
        h = g;
        h.col[0] = h.n;          // out of range
        e = h.csr();
        CHECK(mc_check_graph(&e, 0) == MC_E_BAD_GRAPH);
        h = g;
        h.w[1] = -1;             // negative weight
        e = h.csr();
        CHECK(mc_check_graph(&e, 0) == MC_E_BAD_GRAPH);
        h = g;
        h.w[h.w.size() - 1] += 1;   // one direction heavier: asymmetric
        e = h.csr();
        CHECK(mc_check_graph(&e, 0) == MC_OK);
        CHECK(mc_check_graph(&e, 1) == MC_E_BAD_GRAPH);
    }
    {
        // total weight: 2^62 - 1 passes, 2^62 overflows, huge entries do not wrap
        G g;
        g.n = 2;
        g.rp = {0, 1, 2};
        g.col = {1, 0};
        const int64_t half = ((int64_t)1 << 61);
        g.w = {half, half - 1};
        mc_csr c = g.csr();
        CHECK(mc_check_graph(&c, 0) == MC_OK);
        g.w = {half, half};
        c = g.csr();
        CHECK(mc_check_graph(&c, 0) == MC_E_OVERFLOW);
        g.w = {INT64_MAX, INT64_MAX};
        c = g.csr();
        CHECK(mc_check_graph(&c, 0) == MC_E_OVERFLOW);
    }
    {
        mc_options o;
        mc_default_options(&o);
        CHECK(o.seed == 1 && o.pr_tri_deg_cap == 16);
        mc_default_options(nullptr);
        CHECK(mc_last_error() != nullptr);
    }
    if (failures) return 1;
    std::printf("sanitize driver ok\n");
    return 0;
}
