// Union-find over contractible edges, canonical relabelling, the
// Padberg-Rinaldi tests 1 and 2, side tracking and input checks.
//
// Contractible edges found in one round (reduction tests and CAPFOREST,
// Algorithm 1's U.union) all land in one concurrent union-find; the round's
// contraction uses its components. Roots are always the smallest vertex of
// their component (see uf_union), so numbering roots in increasing order
// gives labels that do not depend on the order of the unions.
#include <algorithm>

#include "mc_internal.h"

namespace {

inline int grid_for(int64_t count, int threads, int cap = 8192) {
    int64_t b = (count + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

constexpr int SUB = 16;  // lanes per row for row-wise kernels
// test-1 trees that the byte-label linking handles (k_pr1_trees) and
// the words of its tree-pair bit matrix
constexpr int PR1_TREES = 255;
constexpr int PR1_WORDS = 256 * 256 / 32;

__global__ void k_uf_init(int32_t* par, int32_t n) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        par[v] = (int32_t)v;
}

__global__ __launch_bounds__(256) void k_uf_all_edges(DGraph g, int32_t* par) {
    const int64_t nsub = (int64_t)gridDim.x * (blockDim.x / SUB);
    const int sl = threadIdx.x % SUB;
    for (int64_t v = (int64_t)blockIdx.x * (blockDim.x / SUB) + threadIdx.x / SUB; v < g.n; v += nsub) {
        const int32_t o = g.off[v], l = g.len[v];
        for (int32_t j = sl; j < l; j += SUB) {
            const int32_t x = g.col[o + j];
            if (x > v && g.w[o + j] > 0) uf_union(par, (int32_t)v, x);
        }
    }
}

// Connectivity in the manner of Afforest (Sutton, Ben-Nun and Barak, IPDPS
// 2018), on a graph whose entries all have positive weight (a normalised
// graph). CONNECT_SWEEPS hooking sweeps over the first CONNECT_K entries of
// every row first join much of the graph: in each, a row lowers the root of its own
// tree to the smallest root among those neighbours (parent[] is compressed
// before each sweep, so par[v] is a root); pointers only ever decrease, so
// the forest stays acyclic and the union-find invariant parent[x] <= x
// holds. (Full unions here would be exact sooner, but on power-law graphs
// thousands of them then meet at the root of the growing giant tree, one
// compare-and-swap at a time.) Then the component most sampled vertices fall
// into is found, and the remaining edges are linked (k_uf_link_rest).
// Exactness does not depend on what the sweeps joined: they only join
// connected vertices, and every edge whose endpoints were apart when the
// sweeps ended is linked afterwards.
constexpr int CONNECT_K = 8;   // entries per row the hooking sweeps look at
// Three sweeps, not two: on geometric graphs (hyperbolic, 32-core) two
// leave thousands of trees and the linking pass then runs millions of
// unions; the third costs about 0.2 ms and saves about 0.4 ms there.
constexpr int CONNECT_SWEEPS = 3;

__global__ __launch_bounds__(256) void k_uf_root_min(DGraph g, int32_t* par) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t o = g.off[v], l = g.len[v] < CONNECT_K ? g.len[v] : CONNECT_K;
        const int32_t r = ld_acq(&par[v]);
        // all targets, then all their parents, in flight at once
        int32_t x[CONNECT_K];
#pragma unroll
        for (int j = 0; j < CONNECT_K; j++) x[j] = j < l ? g.col[o + j] : (int32_t)v;
        int32_t m = r;
#pragma unroll
        for (int j = 0; j < CONNECT_K; j++) {
            const int32_t px = j < l ? ld_acq(&par[x[j]]) : r;
            m = px < m ? px : m;
        }
        if (m < r && m < ld_acq(&par[r])) atomicMin(&par[r], m);
    }
}

__global__ __launch_bounds__(1024) void k_uf_sample_mode(const int32_t* par, int32_t n, int32_t* mode) {
    __shared__ int32_t smp[1024];
    __shared__ int32_t bestc[1024], bestr[1024];
    const uint32_t h = hash32(threadIdx.x * 2654435761u + 12345u);
    const int32_t v = (int32_t)(((uint64_t)h * (uint64_t)n) >> 32);
    int32_t x = v, p = ld_acq(&par[x]);
    while (p != x) { x = p; p = ld_acq(&par[x]); }
    smp[threadIdx.x] = x;
    __syncthreads();
    int32_t c = 0;
    for (int k = 0; k < 1024; k++) c += smp[k] == x;
    bestc[threadIdx.x] = c;
    bestr[threadIdx.x] = x;
    __syncthreads();
    for (int s2 = 512; s2 > 0; s2 >>= 1) {
        if (threadIdx.x < s2 && bestc[threadIdx.x + s2] > bestc[threadIdx.x]) {
            bestc[threadIdx.x] = bestc[threadIdx.x + s2];
            bestr[threadIdx.x] = bestr[threadIdx.x + s2];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        mode[0] = bestr[0];
        mode[1] = bestc[0];   // samples (of 1024) in that component
    }
}

// After a compress: snap[v] = v's root, inbig[v] = 1 iff that root is the
// root of the largest sampled component.
__global__ void k_uf_snapshot(const int32_t* par, int32_t n, const int32_t* mode, uint8_t* inbig, int32_t* snap,
                              const int32_t* ntree = nullptr) {
    if (ntree && *ntree <= PR1_TREES) return;   // the trees are linked by k_pr1_trees
    const int32_t big = *mode;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = par[v];
        snap[v] = r;
        inbig[v] = r == big;
    }
}

// The edges still to link: those whose endpoints were in different trees
// at the snapshot. Rows of the largest sampled component skip whole, so an
// edge is linked from its smaller endpoint's row, or from the outside
// endpoint's row when the other endpoint is in that component. The
// snapshot is taken before any of these unions (roots move while they run).
__global__ __launch_bounds__(256) void k_uf_link_rest(DGraph g, int32_t* par, const uint8_t* __restrict__ inbig,
                                                     const int32_t* __restrict__ snap, unsigned long long* pb) {
    const int64_t nsub = (int64_t)gridDim.x * (blockDim.x / SUB);
    const int sl = threadIdx.x % SUB;
    int64_t bytes = 0;
    for (int64_t v = (int64_t)blockIdx.x * (blockDim.x / SUB) + threadIdx.x / SUB; v < g.n; v += nsub) {
        if (sl == 0) bytes += 1;
        if (inbig[v]) continue;
        const int32_t o = g.off[v], l = g.len[v], rv = snap[v];
        for (int32_t j = sl; j < l; j += SUB) {
            const int32_t x = g.col[o + j];
            if ((x > v || inbig[x]) && snap[x] != rv) uf_union(par, (int32_t)v, x);
        }
        if (sl == 0) bytes += 12 + 9 * (int64_t)l;
    }
    if (pb) prof_add(pb, bytes);
}

// After all unions: point every vertex at its root. Each thread writes only
// its own entry, so concurrent finds still see valid ancestors.
__global__ void k_uf_compress(int32_t* par, int32_t n) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int32_t x = (int32_t)v, p = ld_acq(&par[x]);
        while (p != x) { x = p; p = ld_acq(&par[x]); }
        st_rel(&par[v], x);
    }
}

__global__ void k_root_flag(const int32_t* par, int32_t n, int32_t* flag) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        flag[v] = par[v] == v;
}

__global__ void k_label(const int32_t* par, const int32_t* newid, int32_t n, int32_t* L, DevScalars* sc) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        L[v] = newid[par[v]];
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->n2 = newid[n];
}

// Padberg-Rinaldi tests on the current graph with bound lam:
//  test 1: an edge of weight >= lam joins two vertices whose connectivity is
//          at least lam, so no cut below lam separates them; the test-1
//          edges are joined as Afforest joins a graph: each row's first
//          two test-1 neighbours are unioned, then the component most
//          sampled vertices fall into is found, and only rows outside it
//          union their test-1 entries to other trees of that snapshot (once
//          the bound is small nearly every edge passes, and nearly every
//          row or entry then skips);
//  test 2: if 2 c(v,p) >= c(v) for v's heaviest neighbour p (smallest id on
//          ties), moving v to p's side of any cut does not increase it; one
//          such pointer per vertex may be contracted together with all
//          connectivity-based marks of the round.
// Rows longer than PR_LONG are handed to k_pr12_long (many workgroups per
// row) so one giant collapsed vertex does not serialise the launch.
constexpr int32_t PR_LONG = 2048;
constexpr int32_t PR_CHUNK = 4096;

// Algorithmic bytes (profiling): 12 B per entry (col, w) and 16 B per row
// (off, len, deg) of the rows this kernel tests.
__global__ __launch_bounds__(256) void k_pr12(DGraph g, const int64_t* lamp, const int32_t* vinst, int32_t* par,
                                             unsigned long long* marks, uint8_t* flag1, int32_t* ptr2,
                                             int32_t* long_list, int32_t* long_cnt, int32_t* first, int32_t* second,
                                             int32_t* heavy_cnt, unsigned long long* pb) {
    // 16 lanes take 16 consecutive rows: the rows' offsets, lengths,
    // degrees and bounds come in one load, each lane then loads up to four
    // entries of a row at once, and the rows' results (test-2 unions
    // included) are written by one lane each, all 16 at the same time
    const int64_t lam0 = *lamp;
    const int64_t nsub = (int64_t)gridDim.x * (blockDim.x / SUB);
    const int sl = threadIdx.x % SUB;
    unsigned long long joined = 0;
    int64_t bytes = 0;
    for (int64_t v0 = ((int64_t)blockIdx.x * (blockDim.x / SUB) + threadIdx.x / SUB) * SUB; v0 < g.n;
         v0 += nsub * SUB) {
        const int32_t rows = g.n - v0 < SUB ? (int32_t)(g.n - v0) : SUB;
        const int32_t mv = (int32_t)v0 + sl;
        int32_t my_o = 0, my_l = 0;
        int64_t my_lam = lam0, my_deg = 0;
        if (sl < rows) {
            my_o = g.off[mv];
            my_l = g.len[mv];
            my_deg = g.deg[mv];
            if (vinst) my_lam = lamp[vinst[mv]];   // bound of the row's instance
            if (my_l > PR_LONG) {
                long_list[atomicAdd(long_cnt, 1)] = mv;
                first[mv] = -1;       // a long row unions its test-1 entries itself
                second[mv] = -1;
                heavy_cnt[mv] = 0;
            }
        }
        int64_t my_bw = -1;
        int32_t my_bx = -1, my_hj = INT32_MAX, my_hj2 = INT32_MAX, my_hn = 0;
        for (int32_t r = 0; r < rows; r++) {
            const int32_t l = __shfl(my_l, r, SUB);
            if (l > PR_LONG) continue;
            const int32_t o = __shfl(my_o, r, SUB);
            const int64_t lam = __shfl(my_lam, r, SUB);
            int64_t bw = -1;
            int32_t bx = -1;
            // first and second test-1 entries, test-1 entries
            int32_t hj = INT32_MAX, hj2 = INT32_MAX, hn = 0;
            for (int32_t j0 = 0; j0 < l; j0 += 4 * SUB) {
                int32_t x[4];
                int64_t c[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int32_t j = j0 + u * SUB + sl;
                    x[u] = j < l ? g.col[o + j] : -1;
                    c[u] = j < l ? g.w[o + j] : -1;
                }
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int32_t j = j0 + u * SUB + sl;
                    if (j >= l) continue;
                    const bool heavy = c[u] >= lam;
                    if (flag1) flag1[o + j] = heavy;
                    // a lane meets its entries in increasing j
                    if (heavy) {
                        hn++;
                        if (hj == INT32_MAX) hj = j;
                        else if (hj2 == INT32_MAX) hj2 = j;
                    }
                    if (c[u] > bw || (c[u] == bw && x[u] < bx)) { bw = c[u]; bx = x[u]; }
                }
            }
            for (int k = SUB / 2; k > 0; k >>= 1) {
                int64_t w2 = __shfl_xor(bw, k, SUB);
                int32_t x2 = __shfl_xor(bx, k, SUB);
                if (x2 >= 0 && (bx < 0 || w2 > bw || (w2 == bw && x2 < bx))) { bw = w2; bx = x2; }
                // the two smallest of two sorted pairs
                const int32_t oj = __shfl_xor(hj, k, SUB), oj2 = __shfl_xor(hj2, k, SUB);
                if (oj < hj) {
                    hj2 = hj < oj2 ? hj : oj2;
                    hj = oj;
                } else {
                    hj2 = hj2 < oj ? hj2 : oj;
                }
                hn += __shfl_xor(hn, k, SUB);
            }
            if (sl == r) { my_bw = bw; my_bx = bx; my_hj = hj; my_hj2 = hj2; my_hn = hn; }
            if (sl == 0) bytes += 16 + 12 * (int64_t)l;
        }
        if (sl < rows && my_l <= PR_LONG) {
            const bool take = my_bx >= 0 && 2 * my_bw >= my_deg;
            if (ptr2) ptr2[mv] = take ? my_bx : -1;
            first[mv] = my_hj != INT32_MAX ? g.col[my_o + my_hj] : -1;
            second[mv] = my_hj2 != INT32_MAX ? g.col[my_o + my_hj2] : -1;
            heavy_cnt[mv] = my_hn;
            if (take && uf_union(par, mv, my_bx)) joined++;
        }
    }
    // marks go to one of SPREAD partial counters (128 B apart): a single
    // counter would take one atomic from every wavefront of the launch
    joined = (unsigned long long)wave_sum_i64((int64_t)joined);
    if (lane_id() == 0 && joined) {
        const unsigned slot = (blockIdx.x * (blockDim.x / MC_WAVE) + threadIdx.x / MC_WAVE) % SPREAD;
        atomicAdd(&marks[(size_t)slot * SPREAD_STRIDE], joined);
    }
    if (pb) prof_add(pb, bytes);
}

// Joins u and v as Afforest's link does: climb from their parents and
// hang the larger root under the smaller with a CAS. Finds write nothing
// here (a compress pass follows), so many threads climbing one tree do not
// contend on its nodes. True if this call joined two trees.
__device__ __forceinline__ bool uf_link(int32_t* par, int32_t u, int32_t v) {
    int32_t p1 = ld_acq(&par[u]), p2 = ld_acq(&par[v]);
    while (p1 != p2) {
        const int32_t high = p1 > p2 ? p1 : p2, low = p1 + p2 - high;
        const int32_t ph = ld_acq(&par[high]);
        if (ph == low) return false;
        if (ph == high && atomicCAS(&par[high], high, low) == high) return true;
        p1 = ld_acq(&par[ph]);
        p2 = ld_acq(&par[low]);
    }
    return false;
}

// each row's first (round 0) or second (round 1) test-1 neighbour, with a
// compress between the rounds (marks go to the partial counters). Two per
// row, not one: on geometric graphs the first neighbours alone leave many
// small trees, and the linking of the trees then has far more to do.
__global__ __launch_bounds__(256) void k_pr1_first(const int32_t* __restrict__ nb, int32_t n, int32_t* par,
                                                  unsigned long long* marks, unsigned long long* pb) {
    unsigned long long joined = 0;
    int64_t bytes = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = nb[v];
        if (x >= 0 && uf_link(par, (int32_t)v, x)) joined++;
        bytes += 4 + 4 * (x >= 0);   // the neighbour; the parent word of the union
    }
    if (pb) prof_add(pb, bytes);
    joined = (unsigned long long)wave_sum_i64((int64_t)joined);
    if (lane_id() == 0 && joined) {
        const unsigned slot = (blockIdx.x * (blockDim.x / MC_WAVE) + threadIdx.x / MC_WAVE) % SPREAD;
        atomicAdd(&marks[(size_t)slot * SPREAD_STRIDE], joined);
    }
}

// Linking the test-1 trees through a small tree graph. On geometric graphs
// the first two unions of every row leave a few hundred trees of similar
// size and no giant one (hyperbolic n = 2^23 at bound 2: 135 trees, the
// largest with 3 % of the vertices), so skipping the rows of the sampled
// tree saves nothing and every remaining test-1 entry would gather a 32-bit
// root from a 6.6 MB array and try a union. When at most PR1_TREES trees
// remain, each vertex instead gets its tree's number in one byte (1.6 MB,
// which stays in L2), the entries between two trees only set a bit of a
// 256 x 256 matrix, and one workgroup joins the trees along the set bits
// and repoints every vertex at its component's root. When the tree most
// sampled vertices fall into holds at least half of them, its rows are
// skipped (an edge into it is seen from the other side); otherwise every
// edge is looked at once, from its smaller endpoint, and only there are
// its weight and the target's tree loaded. (Sampling the first entries of
// each row, or the longest rows, before the full pass joins little on
// these graphs: the trees are angular sectors, and the entries between
// them are few and spread over all rows.)

// tree number of every vertex (trees numbered by root, so in the order of
// their smallest vertex) and the root of every tree; tscan holds the
// exclusive prefix count of the roots
__global__ void k_tree_label(const int32_t* __restrict__ par, const int32_t* __restrict__ tscan, int32_t n,
                             uint8_t* lab8, int32_t* troot) {
    if (tscan[n] <= 1 || tscan[n] > PR1_TREES) return;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = par[v];
        lab8[v] = (uint8_t)tscan[r];
        if (r == v) troot[tscan[v]] = (int32_t)v;
    }
}

// the test-1 entries of rows with more than two of them (a row with at
// most two was joined by k_pr1_first) that join two trees, as bits (a < b),
// from the smaller endpoint or from outside into the sampled tree.
// As in k_pr12, 16 lanes take 16 consecutive rows, whose metadata comes in
// one load, and each lane keeps four entries and their trees in flight.
__global__ __launch_bounds__(256) void k_pr1_trees(DGraph g, const int64_t* lamp, const int32_t* vinst,
                                                  const int32_t* __restrict__ heavy_cnt,
                                                  const uint8_t* __restrict__ lab8,
                                                  const int32_t* __restrict__ tscan, const int32_t* mode,
                                                  uint32_t* bits, unsigned long long* pb) {
    if (tscan[g.n] <= 1 || tscan[g.n] > PR1_TREES) return;
    __shared__ uint32_t sb[PR1_WORDS];
    for (int i = threadIdx.x; i < PR1_WORDS; i += blockDim.x) sb[i] = 0;
    __syncthreads();
    // the sampled tree's rows are skipped only when it holds at least half
    // of the samples; else big = -1 and every edge is taken from its
    // smaller endpoint
    const int32_t big = 2 * mode[1] >= 1024 ? tscan[mode[0]] : -1;
    const int64_t lam0 = *lamp;
    const int64_t nsub = (int64_t)gridDim.x * (blockDim.x / SUB);
    const int sl = threadIdx.x % SUB;
    int64_t bytes = 0;
    for (int64_t v0 = ((int64_t)blockIdx.x * (blockDim.x / SUB) + threadIdx.x / SUB) * SUB; v0 < g.n;
         v0 += nsub * SUB) {
        const int32_t rows = g.n - v0 < SUB ? (int32_t)(g.n - v0) : SUB;
        const int32_t mv = (int32_t)v0 + sl;
        int32_t my_o = 0, my_l = 0, my_lv = 0;
        int64_t my_lam = lam0;
        if (sl < rows) {
            my_lv = lab8[mv];
            if (heavy_cnt[mv] > 2 && my_lv != big) {
                my_o = g.off[mv];
                my_l = g.len[mv];
                if (vinst) my_lam = lamp[vinst[mv]];   // bound of the row's instance
            }
        }
        if (sl == 0) bytes += 5 * (int64_t)rows;   // test-1 count and tree of every row
        for (int32_t r = 0; r < rows; r++) {
            const int32_t l = __shfl(my_l, r, SUB);
            if (l == 0) continue;
            const int32_t o = __shfl(my_o, r, SUB), lv = __shfl(my_lv, r, SUB);
            const int64_t lam = __shfl(my_lam, r, SUB);
            const int32_t v = (int32_t)v0 + r;
            if (sl == 0) bytes += 8 + 4 * (int64_t)l;   // off, len; col of each entry
            for (int32_t j0 = 0; j0 < l; j0 += 4 * SUB) {
                int32_t x[4], lx[4];
                int64_t c[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int32_t j = j0 + u * SUB + sl;
                    x[u] = j < l ? g.col[o + j] : -1;
                }
                // without a skipped tree only x > v is needed: the weight
                // and the target's tree are loaded for those alone
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const bool want = x[u] >= 0 && (big >= 0 || x[u] > v);
                    c[u] = want ? g.w[o + j0 + u * SUB + sl] : -1;
                    bytes += want ? 9 : 0;   // w and the target's tree
                }
#pragma unroll
                for (int u = 0; u < 4; u++) lx[u] = c[u] >= lam ? lab8[x[u]] : lv;
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    if (lx[u] == lv || (x[u] < v && lx[u] != big)) continue;
                    const int32_t a = lv < lx[u] ? lv : lx[u], b = lv < lx[u] ? lx[u] : lv;
                    const int32_t bit = a * 256 + b;
                    atomicOr(&sb[bit >> 5], 1u << (bit & 31));
                }
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < PR1_WORDS; i += blockDim.x)
        if (sb[i]) atomicOr(&bits[i], sb[i]);
    if (pb) prof_add(pb, bytes);
}

// one workgroup: components of the tree graph by a lock-free union-find
// on the tree numbers in LDS (the smaller number as root), one thread per
// word of the bit matrix; then the root vertex of each tree's component.
// Counts the joins as marks.
__device__ __forceinline__ int32_t lds_ld(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__global__ __launch_bounds__(256) void k_tree_join(const int32_t* __restrict__ tscan, int32_t n,
                                                  const uint32_t* __restrict__ bits, const int32_t* __restrict__ troot,
                                                  int32_t* tmap, unsigned long long* marks) {
    const int32_t T = tscan[n];
    if (T <= 1 || T > PR1_TREES) return;
    __shared__ int32_t tp[256];
    __shared__ unsigned long long sj;
    for (int t = threadIdx.x; t < 256; t += blockDim.x) tp[t] = t;
    if (threadIdx.x == 0) sj = 0;
    __syncthreads();
    unsigned long long joined = 0;
    for (int i = threadIdx.x; i < PR1_WORDS; i += blockDim.x) {
        for (uint32_t m = bits[i]; m; m &= m - 1) {
            const int bit = i * 32 + __ffs(m) - 1;
            int32_t x = bit >> 8, y = bit & 255;
            for (;;) {
                for (int32_t p = lds_ld(&tp[x]); p != x; p = lds_ld(&tp[x])) x = p;
                for (int32_t p = lds_ld(&tp[y]); p != y; p = lds_ld(&tp[y])) y = p;
                if (x == y) break;
                if (x > y) { const int32_t t = x; x = y; y = t; }
                if (atomicCAS(&tp[y], y, x) == y) { joined++; break; }
            }
        }
    }
    if (joined) atomicAdd(&sj, joined);
    __syncthreads();
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
        int32_t x = t;
        while (tp[x] != x) x = tp[x];
        tmap[t] = troot[x];
    }
    if (threadIdx.x == 0 && sj) atomicAdd(marks, sj);
}

// every vertex points at the root of its tree's component
__global__ void k_tree_apply(const int32_t* __restrict__ tscan, const uint8_t* __restrict__ lab8,
                             const int32_t* __restrict__ tmap, int32_t n, int32_t* par) {
    if (tscan[n] <= 1 || tscan[n] > PR1_TREES) return;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = tmap[lab8[v]];
        if (par[v] != r) par[v] = r;
    }
}

// rows with more than two test-1 entries, outside the sampled
// component: union all of them (an edge into that component from a row
// inside it is seen from this side)
__global__ __launch_bounds__(256) void k_pr1_rest(DGraph g, const int64_t* lamp, const int32_t* vinst, int32_t* par,
                                                 const int32_t* __restrict__ heavy_cnt,
                                                 const uint8_t* __restrict__ inbig, const int32_t* __restrict__ snap,
                                                 const int32_t* ntree, unsigned long long* marks,
                                                 unsigned long long* pb) {
    if (*ntree <= PR1_TREES) return;   // the trees are linked by k_pr1_trees
    const int64_t lam0 = *lamp;
    const int64_t nsub = (int64_t)gridDim.x * (blockDim.x / SUB);
    const int sl = threadIdx.x % SUB;
    unsigned long long joined = 0;
    int64_t bytes = 0;
    for (int64_t v = (int64_t)blockIdx.x * (blockDim.x / SUB) + threadIdx.x / SUB; v < g.n; v += nsub) {
        if (sl == 0) bytes += 5;   // test-1 count and component flag of every row
        if (heavy_cnt[v] <= 2 || inbig[v]) continue;
        // off, len, snapshot root of the row; col, w, flag and root of each target
        if (sl == 0) bytes += 12 + 17 * (int64_t)g.len[v];
        const int32_t o = g.off[v], l = g.len[v], rv = snap[v];
        const int64_t lam = vinst ? lamp[vinst[v]] : lam0;
        // as in k_uf_link_rest: edges between different snapshot trees,
        // from the smaller endpoint or from outside into the sampled
        // component (a long row links all of its test-1 entries itself, and
        // a row with at most two test-1 entries was linked by k_pr1_first)
        for (int32_t j = sl; j < l; j += SUB) {
            const int32_t x = g.col[o + j];
            if (g.w[o + j] >= lam && (x > v || inbig[x]) && snap[x] != rv && uf_union(par, (int32_t)v, x)) joined++;
        }
    }
    if (pb) prof_add(pb, bytes);
    joined = (unsigned long long)wave_sum_i64((int64_t)joined);
    if (lane_id() == 0 && joined) {
        const unsigned slot = (blockIdx.x * (blockDim.x / MC_WAVE) + threadIdx.x / MC_WAVE) % SPREAD;
        atomicAdd(&marks[(size_t)slot * SPREAD_STRIDE], joined);
    }
}

// fold the partial counters of k_pr12 into the round's mark count
__global__ __launch_bounds__(64) void k_pr12_fold(unsigned long long* spread, unsigned long long* marks) {
    const int64_t v = wave_sum_i64((int64_t)spread[(size_t)threadIdx.x * SPREAD_STRIDE]);
    if (threadIdx.x == 0 && v) atomicAdd(marks, (unsigned long long)v);
}

// task offsets of the long rows: ceil(len / PR_CHUNK) tasks each
__global__ __launch_bounds__(1024) void k_pr12_long_scan(const DGraph g, const int32_t* long_list,
                                                        const int32_t* long_cnt, int32_t* task_off) {
    __shared__ int32_t part[1024];
    const int32_t nl = *long_cnt;
    const int32_t per = (nl + 1023) / 1024;
    const int32_t b = threadIdx.x * per, e = b + per < nl ? b + per : nl;
    int32_t s = 0;
    for (int32_t i = b; i < e; i++) s += (g.len[long_list[i]] + PR_CHUNK - 1) / PR_CHUNK;
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int k = 0; k < 1024; k++) { int32_t t = part[k]; part[k] = run; run += t; }
        task_off[nl] = run;
    }
    __syncthreads();
    int32_t run = part[threadIdx.x];
    for (int32_t i = b; i < e; i++) {
        task_off[i] = run;
        run += (g.len[long_list[i]] + PR_CHUNK - 1) / PR_CHUNK;
    }
}

__device__ __forceinline__ int32_t last_le_g(const int32_t* a, int32_t n, int64_t key) {
    int32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        int32_t mid = lo + (hi - lo) / 2;
        if ((int64_t)a[mid] <= key) lo = mid; else hi = mid;
    }
    return lo;
}

// one workgroup per PR_CHUNK-entry piece of a long row: test 1 unions and
// the piece's heaviest entry
__global__ __launch_bounds__(256) void k_pr12_long(DGraph g, const int64_t* lamp, const int32_t* vinst, int32_t* par,
                                                  unsigned long long* marks, uint8_t* flag1,
                                                  const int32_t* long_list, const int32_t* long_cnt,
                                                  const int32_t* task_off, int64_t* part_w, int32_t* part_x) {
    __shared__ int64_t sw[4];
    __shared__ int32_t sx[4];
    __shared__ int32_t s_rv;
    const int64_t lam0 = *lamp;
    const int32_t nl = *long_cnt;
    const int32_t ntask = task_off[nl];
    unsigned long long joined = 0;
    for (int32_t t = blockIdx.x; t < ntask; t += gridDim.x) {
        const int32_t i = last_le_g(task_off, nl, t);
        const int32_t v = long_list[i];
        const int32_t o = g.off[v], l = g.len[v];
        const int64_t lam = vinst ? lamp[vinst[v]] : lam0;
        const int32_t j0 = (t - task_off[i]) * PR_CHUNK;
        const int32_t j1 = j0 + PR_CHUNK < l ? j0 + PR_CHUNK : l;
        // every union of the piece involves v: find its root once, so the
        // threads do not all walk (and shorten) v's path at the same time
        if (threadIdx.x == 0) s_rv = uf_find(par, v);
        __syncthreads();
        const int32_t rv = s_rv;
        int64_t bw = -1;
        int32_t bx = -1;
        for (int32_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
            const int32_t x = g.col[o + j];
            const int64_t c = g.w[o + j];
            const bool heavy = c >= lam;
            if (flag1) flag1[o + j] = heavy;
            if (heavy && uf_union(par, rv, x)) joined++;
            if (c > bw || (c == bw && x < bx)) { bw = c; bx = x; }
        }
        int32_t aux = 0;
        wave_argmax(bw, bx, aux);
        __syncthreads();
        if (lane_id() == 0) { sw[threadIdx.x / MC_WAVE] = bw; sx[threadIdx.x / MC_WAVE] = bx; }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int k = 1; k < 4; k++)
                if (sx[k] >= 0 && (bx < 0 || sw[k] > bw || (sw[k] == bw && sx[k] < bx))) { bw = sw[k]; bx = sx[k]; }
            part_w[t] = bw;
            part_x[t] = bx;
        }
    }
    joined = (unsigned long long)wave_sum_i64((int64_t)joined);
    if (lane_id() == 0 && joined) atomicAdd(marks, joined);
}

// one wavefront per long row: fold its pieces, apply test 2
__global__ __launch_bounds__(64) void k_pr12_long_final(DGraph g, int32_t* par, unsigned long long* marks,
                                                       int32_t* ptr2, const int32_t* long_list,
                                                       const int32_t* long_cnt, const int32_t* task_off,
                                                       const int64_t* part_w, const int32_t* part_x) {
    const int32_t nl = *long_cnt;
    for (int32_t i = blockIdx.x; i < nl; i += gridDim.x) {
        int64_t bw = -1;
        int32_t bx = -1;
        for (int32_t t = task_off[i] + threadIdx.x; t < task_off[i + 1]; t += MC_WAVE) {
            const int64_t w2 = part_w[t];
            const int32_t x2 = part_x[t];
            if (x2 >= 0 && (bx < 0 || w2 > bw || (w2 == bw && x2 < bx))) { bw = w2; bx = x2; }
        }
        int32_t aux = 0;
        wave_argmax(bw, bx, aux);
        if (threadIdx.x == 0) {
            const int32_t v = long_list[i];
            const bool take = bx >= 0 && 2 * bw >= g.deg[v];
            if (ptr2) ptr2[v] = take ? bx : -1;
            if (take && uf_union(par, v, bx)) atomicAdd(marks, 1ULL);
        }
    }
}

// Padberg-Rinaldi tests 3 and 4 (the remaining two of the four local tests;
// applied in one sweep over candidate edges, which may miss edges, as the
// linear-time sweeps of App. A do): candidates are the edges {v,x} whose
// rows both have at most D entries. With c(.) the degrees:
//   s = c(v,x) + sum over common neighbours u of min(c(v,u), c(x,u));
//   test 4: s >= lam -- the edge and the two-edge paths through the common
//           neighbours are edge-disjoint, so v and x are at least s-connected
//           and the edge joins the union-find like test 1;
//   test 3: some common u has 2 (c(v,x) + c(v,u)) >= c(v) and
//           2 (c(v,x) + c(x,u)) >= c(x) -- an exchange argument like test 2,
//           so only a matching is applied: every vertex proposes its
//           smallest test-3 partner, mutual proposals between vertices that
//           touch no test-2 pointer are accepted (k_pr3_accept).
// One group of TRI_SUB lanes per vertex v of at most D entries: N(v) goes
// to an LDS hash, then for every neighbour x > v with a short row the lanes
// scan N(x) against it.
constexpr int TRI_SUB = 16;
constexpr int TRI_T = 256;
constexpr int TRI_MAXD = 64;
constexpr int TRI_SLOTS = 2 * TRI_MAXD;
constexpr int32_t TRI_NONE = INT32_MAX;

__global__ __launch_bounds__(TRI_T) void k_pr34(DGraph g, const int64_t* lamp, const int32_t* vinst, int32_t D,
                                               int32_t* par, unsigned long long* marks, int32_t* part3,
                                               uint8_t* flag4) {
    __shared__ int32_t hk[TRI_T / TRI_SUB][TRI_SLOTS];
    __shared__ int64_t hv[TRI_T / TRI_SUB][TRI_SLOTS];
    const int64_t lam0 = *lamp;
    const int grp = threadIdx.x / TRI_SUB, sl = threadIdx.x % TRI_SUB;
    int32_t* K = hk[grp];
    int64_t* W = hv[grp];
    const int64_t ngrp = (int64_t)gridDim.x * (TRI_T / TRI_SUB);
    unsigned long long joined = 0;
    // uniform trip count over the workgroup (the LDS tables are per group,
    // but the loop shape keeps every lane in step for the shuffles)
    const int64_t top = ((int64_t)g.n + ngrp - 1) / ngrp * ngrp;
    for (int64_t v0 = (int64_t)blockIdx.x * (TRI_T / TRI_SUB) + grp; v0 < top; v0 += ngrp) {
        const int32_t v = (int32_t)v0;
        const bool live = v0 < g.n && g.len[v] <= D && g.len[v] > 0;
        const int32_t o = live ? g.off[v] : 0, l = live ? g.len[v] : 0;
        for (int k = sl; k < TRI_SLOTS; k += TRI_SUB) K[k] = -1;
        wave_sync();
        for (int32_t j = sl; j < l; j += TRI_SUB) {
            const int32_t x = g.col[o + j];
            uint32_t h = hash32((uint32_t)x) & (TRI_SLOTS - 1);
            while (atomicCAS(&K[h], -1, x) != -1) h = (h + 1) & (TRI_SLOTS - 1);
            W[h] = g.w[o + j];
        }
        wave_sync();
        const int64_t cv = live ? g.deg[v] : 0;
        const int64_t lam = live && vinst ? lamp[vinst[v]] : lam0;   // bound of v's instance
        for (int32_t j = 0; j < l; j++) {
            const int32_t x = g.col[o + j];
            if (x <= v || g.len[x] > D) continue;          // uniform over the group
            const int64_t cvx = g.w[o + j];
            const int64_t cx = g.deg[x];
            const int32_t ox = g.off[x], lx = g.len[x];
            int64_t sum = 0;
            int t3 = 0;
            int32_t back = -1;
            for (int32_t b = sl; b < lx; b += TRI_SUB) {
                const int32_t u = g.col[ox + b];
                if (u == v) { back = ox + b; continue; }
                uint32_t h = hash32((uint32_t)u) & (TRI_SLOTS - 1);
                for (;;) {
                    const int32_t k = K[h];
                    if (k == u || k == -1) break;
                    h = (h + 1) & (TRI_SLOTS - 1);
                }
                if (K[h] != u) continue;
                const int64_t cvu = W[h], cxu = g.w[ox + b];
                sum += cvu < cxu ? cvu : cxu;
                if (2 * (cvx + cvu) >= cv && 2 * (cvx + cxu) >= cx) t3 = 1;
            }
            for (int d = TRI_SUB / 2; d > 0; d >>= 1) {
                sum += __shfl_xor(sum, d, TRI_SUB);
                t3 |= __shfl_xor(t3, d, TRI_SUB);
                const int32_t b2 = __shfl_xor(back, d, TRI_SUB);
                back = b2 > back ? b2 : back;
            }
            if (sl == 0) {
                const bool t4 = cvx + sum >= lam;
                if (flag4) {
                    flag4[o + j] = t4;
                    if (back >= 0) flag4[back] = t4;
                }
                if (t4 && uf_union(par, v, x)) joined++;
                if (t3) {
                    atomicMin(&part3[v], x);
                    atomicMin(&part3[x], v);
                }
            }
        }
        wave_sync();
    }
    joined = (unsigned long long)wave_sum_i64((int64_t)joined);
    if (lane_id() == 0 && joined) {
        const unsigned slot = (blockIdx.x * (blockDim.x / MC_WAVE) + threadIdx.x / MC_WAVE) % SPREAD;
        atomicAdd(&marks[(size_t)slot * SPREAD_STRIDE], joined);
    }
}

// vertices that are the source or the target of a test-2 pointer
__global__ void k_pr2_touch(const int32_t* ptr2, int32_t n, uint8_t* touch) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        if (ptr2[v] >= 0) { touch[v] = 1; touch[ptr2[v]] = 1; }
}

// mutual smallest test-3 partners away from test-2 pointers are contracted
__global__ void k_pr3_accept(const int32_t* part3, const uint8_t* touch, int32_t n, int32_t* par,
                             unsigned long long* marks, int32_t* acc3) {
    unsigned long long joined = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = part3[v];
        const bool ok = x != TRI_NONE && part3[x] == (int32_t)v && !touch[v] && !touch[x];
        if (acc3) acc3[v] = ok ? x : -1;
        if (ok && x > v && uf_union(par, (int32_t)v, x)) joined++;
    }
    joined = (unsigned long long)wave_sum_i64((int64_t)joined);
    if (lane_id() == 0 && joined) {
        const unsigned slot = (blockIdx.x * (blockDim.x / MC_WAVE) + threadIdx.x / MC_WAVE) % SPREAD;
        atomicAdd(&marks[(size_t)slot * SPREAD_STRIDE], joined);
    }
}

// (entries of -1 stand for input vertices no longer tracked and stay -1)
__global__ void k_map_update(int32_t* map0, const int32_t* L, int32_t n0) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n0; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t m = map0[v];
        if (m >= 0) map0[v] = L[m];
    }
}

__global__ void k_side_vertex(uint8_t* side, const int32_t* map0, int32_t n0, const int32_t* target) {
    const int32_t t = *target;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n0; v += (int64_t)gridDim.x * blockDim.x)
        side[v] = map0[v] == t;
}

__global__ void k_mark_prefix(uint8_t* flag, const int32_t* order, const int32_t* lenp) {
    const int32_t len = *lenp;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len; k += (int64_t)gridDim.x * blockDim.x)
        flag[order[k]] = 1;
}

__global__ void k_side_flag(uint8_t* side, const int32_t* map0, int32_t n0, const uint8_t* flag) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n0; v += (int64_t)gridDim.x * blockDim.x)
        side[v] = flag[map0[v]];
}

// side[v] = 1 iff input vertex v lies outside the component of vertex 0;
// map (may be null: the identity) takes input vertices to the vertices of
// the graph whose compressed forest par is
__global__ void k_side_comp(uint8_t* side, const int32_t* par, const int32_t* map, int32_t n0) {
    const int32_t r0 = par[map ? map[0] : 0];
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n0; v += (int64_t)gridDim.x * blockDim.x)
        side[v] = par[map ? map[v] : (int32_t)v] != r0;
}

__global__ void k_csr_to_padded(const int32_t* rp, int32_t n, int32_t* off, int32_t* len) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        off[v] = rp[v];
        len[v] = rp[v + 1] - rp[v];
    }
}

constexpr unsigned long long WCAP = 1ULL << 62;

__device__ void set_err(DevScalars* sc, int32_t code) { atomicCAS(&sc->err, 0, code); }

// saturating sum of the block partials (each at most WCAP, so a pairwise
// sum fits in 64 bits before it saturates)
__global__ __launch_bounds__(256) void k_validate_sum(const unsigned long long* part, int nb, DevScalars* sc) {
    __shared__ unsigned long long bs[256];
    unsigned long long t = 0;
    for (int k = threadIdx.x; k < nb; k += 256) { t += part[k]; if (t >= WCAP) t = WCAP; }
    bs[threadIdx.x] = t;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            unsigned long long u = bs[threadIdx.x] + bs[threadIdx.x + o];
            bs[threadIdx.x] = u >= WCAP ? WCAP : u;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && bs[0] >= WCAP) set_err(sc, MC_E_OVERFLOW);
}

// Normalisation fast path: a row whose targets strictly increase, with no
// loop and only positive weights, is already in normal form (a simple
// graph, nothing to merge). Writes len and the degrees of every row, and
// sets *noncanon when some row is not normal. With sc (a device input) the
// same pass checks the input: row bounds within
// [0, nnz] and non-decreasing (a row that fails is not read), targets in
// range, weights non-negative, and the weights' sum, saturated at WCAP, into
// part[blockIdx.x] for k_validate_sum. With lp1, the same pass writes the
// first label-propagation round from singleton labels (Section 2.1
// heuristic): every row's heaviest neighbour, the smallest on ties, or the
// row itself when it has none; it is that round's result when the input is
// in normal form (the caller drops it otherwise).
__global__ __launch_bounds__(256) void k_canon(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                              const int64_t* __restrict__ w, int32_t n, int32_t nnz,
                                              int32_t* __restrict__ len, int64_t* __restrict__ deg,
                                              int32_t* noncanon, DevScalars* sc, unsigned long long* part,
                                              int32_t* __restrict__ lp1) {
    // 16 lanes take 16 consecutive rows: their offsets come in one load,
    // and each lane then loads up to four entries of a row at once
    const int64_t nsub = (int64_t)gridDim.x * (blockDim.x / SUB);
    const int sl = threadIdx.x % SUB;
    bool bad_any = false;
    unsigned long long wsum = 0;
    if (sc && blockIdx.x == 0 && threadIdx.x == 0 && (rp[0] != 0 || rp[n] != nnz)) set_err(sc, MC_E_BAD_GRAPH);
    for (int64_t v0 = ((int64_t)blockIdx.x * (blockDim.x / SUB) + threadIdx.x / SUB) * SUB; v0 < n; v0 += nsub * SUB) {
        int32_t my_o = v0 + sl <= n ? rp[v0 + sl] : 0;
        int32_t my_e = v0 + sl < n ? rp[v0 + sl + 1] : my_o;
        if (sc && v0 + sl < n && (my_o < 0 || my_e < my_o || my_e > nnz)) {
            set_err(sc, MC_E_BAD_GRAPH);
            my_e = my_o = 0;
        }
        int64_t my_d = 0;
        int32_t my_lp = INT32_MAX;
        const int32_t rows = n - v0 < SUB ? (int32_t)(n - v0) : SUB;
        for (int32_t r = 0; r < rows; r++) {
            const int32_t v = (int32_t)v0 + r;
            const int32_t o = __shfl(my_o, r, SUB), e = __shfl(my_e, r, SUB), l = e - o;
            int64_t d = 0;
            int64_t bw = 0;
            int32_t bx = INT32_MAX;
            bool bad = false;
            for (int32_t j0 = 0; j0 < l; j0 += 4 * SUB) {
                int32_t x[4], xp[4];
                int64_t c[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int32_t j = j0 + u * SUB + sl;
                    x[u] = j < l ? col[o + j] : INT32_MAX;
                    xp[u] = j > 0 && j < l ? col[o + j - 1] : -1;
                    c[u] = j < l ? w[o + j] : 1;
                }
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    if (j0 + u * SUB + sl < l) {
                        d += c[u];
                        bad |= x[u] == v || c[u] <= 0 || xp[u] >= x[u];
                        if (x[u] != v && c[u] > 0 && (c[u] > bw || (c[u] == bw && x[u] < bx))) {
                            bw = c[u];
                            bx = x[u];
                        }
                        if (sc) {
                            if (x[u] < 0 || x[u] >= n || c[u] < 0) set_err(sc, MC_E_BAD_GRAPH);
                            if (c[u] > 0) {
                                wsum += (unsigned long long)c[u];
                                if (wsum >= WCAP || (unsigned long long)c[u] >= WCAP) wsum = WCAP;
                            }
                        }
                    }
                }
            }
            for (int k = SUB / 2; k > 0; k >>= 1) d += __shfl_xor(d, k, SUB);
            if (lp1) {
                for (int k = SUB / 2; k > 0; k >>= 1) {
                    const int64_t w2 = __shfl_xor(bw, k, SUB);
                    const int32_t x2 = __shfl_xor(bx, k, SUB);
                    if (w2 > bw || (w2 == bw && x2 < bx)) { bw = w2; bx = x2; }
                }
            }
            if (sl == r) { my_d = d; my_lp = bx; }
            bad_any |= bad;
        }
        if (v0 + sl < n) {
            len[v0 + sl] = my_e - my_o;
            deg[v0 + sl] = my_d;
            if (lp1) lp1[v0 + sl] = my_lp != INT32_MAX ? my_lp : (int32_t)(v0 + sl);
        }
    }
    if (__ballot(bad_any) && lane_id() == 0 && ld_acq(noncanon) == 0) st_rel(noncanon, 1);
    if (sc) {
        __shared__ unsigned long long bs[256];
        bs[threadIdx.x] = wsum;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0;
            for (int k = 0; k < 256; k++) { t += bs[k]; if (t >= WCAP) t = WCAP; }
            part[blockIdx.x] = t;
        }
    }
}

}  // namespace

bool uf_init(int32_t* parent, int32_t n, hipStream_t s) {
    k_uf_init<<<grid_for(n, 256), 256, 0, s>>>(parent, n);
    MC_LAUNCHED("k_uf_init");
    return true;
}

bool uf_all_edges(const DGraph& g, int32_t* parent, hipStream_t s) {
    k_uf_all_edges<<<grid_for((int64_t)g.n * SUB, 256), 256, 0, s>>>(g, parent);
    MC_LAUNCHED("k_uf_all_edges");
    return true;
}

bool uf_connectivity(const DGraph& g, int32_t* parent, int32_t* tmp, uint8_t* inbig, int32_t* snap, hipStream_t s) {
    const int rows = grid_for((int64_t)g.n * SUB, 256);
    for (int sweep = 0; sweep < CONNECT_SWEEPS; sweep++) {
        k_uf_root_min<<<grid_for(g.n, 256), 256, 0, s>>>(g, parent);
        MC_LAUNCHED("k_uf_root_min");
        k_uf_compress<<<grid_for(g.n, 256), 256, 0, s>>>(parent, g.n);
        MC_LAUNCHED("k_uf_compress");
    }
    k_uf_sample_mode<<<1, 1024, 0, s>>>(parent, g.n, tmp);
    MC_LAUNCHED("k_uf_sample_mode");
    k_uf_snapshot<<<grid_for(g.n, 256), 256, 0, s>>>(parent, g.n, tmp, inbig, snap);
    MC_LAUNCHED("k_uf_snapshot");
    prof_begin(PK_UF_LINK_REST, s);
    k_uf_link_rest<<<rows, 256, 0, s>>>(g, parent, inbig, snap, prof_dev_bytes(PK_UF_LINK_REST));
    MC_LAUNCHED("k_uf_link_rest");
    prof_end(PK_UF_LINK_REST, s);
    return true;
}

bool uf_labels(int32_t* parent, int32_t n, int32_t* L, int32_t* flag_tmp, int32_t* scan_tmp, DevScalars* sc,
               hipStream_t s) {
    k_uf_compress<<<grid_for(n, 256), 256, 0, s>>>(parent, n);
    MC_LAUNCHED("k_uf_compress");
    k_root_flag<<<grid_for(n, 256), 256, 0, s>>>(parent, n, flag_tmp);
    MC_LAUNCHED("k_root_flag");
    if (!scan_i32(flag_tmp, flag_tmp, n, scan_tmp, s)) return false;
    k_label<<<grid_for(n, 256), 256, 0, s>>>(parent, flag_tmp, n, L, sc);
    MC_LAUNCHED("k_label");
    return true;
}

void pr12_ws_carve(Arena& a, int32_t n, int64_t cap, Pr12WS& w) {
    // rows longer than PR_LONG: at most n and at most cap / PR_LONG
    const size_t nlong = (size_t)std::min<int64_t>(n, cap / PR_LONG + 1) + 64;
    w.long_list = a.take<int32_t>(nlong);
    w.counters = a.take<int32_t>(4);
    w.task_off = a.take<int32_t>(nlong + 1);
    const size_t tasks = (size_t)(cap / PR_CHUNK) + nlong;
    w.part_w = a.take<int64_t>(tasks);
    w.part_x = a.take<int32_t>(tasks);
    w.spread = a.take<unsigned long long>((size_t)SPREAD * SPREAD_STRIDE);
    w.first = a.take<int32_t>((size_t)n + 1);
    w.second = a.take<int32_t>((size_t)n + 1);
    w.heavy = a.take<int32_t>((size_t)n + 1);
    w.mode = a.take<int32_t>(4);
    w.inbig = a.take<uint8_t>((size_t)n + 1);
    w.snap = a.take<int32_t>((size_t)n + 1);
    w.tscan = a.take<int32_t>((size_t)n + 1);
    w.scan_tmp = a.take<int32_t>(scan_tmp_elems((int64_t)n) + 1);
    w.tbits = a.take<uint32_t>(PR1_WORDS);
    w.troot = a.take<int32_t>(256);
    w.tmap = a.take<int32_t>(256);
}

bool pr12(const DGraph& g, const int64_t* lam, int32_t* parent, unsigned long long* marks, uint8_t* flag1,
          int32_t* ptr2, Pr12WS& w, hipStream_t s, const int32_t* vinst) {
    if (!fill_i32(w.counters, 0, 4, s)) return false;
    if (!fill_i64((int64_t*)w.spread, 0, (int64_t)SPREAD * SPREAD_STRIDE, s)) return false;
    prof_begin(PK_PR12, s);
    k_pr12<<<grid_for(g.n, 256), 256, 0, s>>>(g, lam, vinst, parent, w.spread, flag1, ptr2, w.long_list,
                                                            w.counters, w.first, w.second, w.heavy,
                                                            prof_dev_bytes(PK_PR12));
    MC_LAUNCHED("k_pr12");
    prof_end(PK_PR12, s);
    for (int round = 0; round < 2; round++) {
        prof_begin(PK_PR1_FIRST, s);
        k_pr1_first<<<grid_for(g.n, 256), 256, 0, s>>>(round ? w.second : w.first, g.n, parent, w.spread,
                                                      prof_dev_bytes(PK_PR1_FIRST));
        MC_LAUNCHED("k_pr1_first");
        prof_end(PK_PR1_FIRST, s);
        k_uf_compress<<<grid_for(g.n, 256), 256, 0, s>>>(parent, g.n);
        MC_LAUNCHED("k_uf_compress");
    }
    // trees numbered by root: with at most PR1_TREES of them the byte-label
    // path links them (k_pr1_trees ... k_tree_apply), otherwise the
    // snapshot path (k_uf_snapshot, k_pr1_rest); each kernel of the path
    // not taken returns at once
    k_root_flag<<<grid_for(g.n, 256), 256, 0, s>>>(parent, g.n, w.tscan);
    MC_LAUNCHED("k_root_flag");
    if (!scan_i32(w.tscan, w.tscan, g.n, w.scan_tmp, s)) return false;
    if (!fill_i32((int32_t*)w.tbits, 0, PR1_WORDS, s)) return false;
    k_uf_sample_mode<<<1, 1024, 0, s>>>(parent, g.n, w.mode);
    MC_LAUNCHED("k_uf_sample_mode");
    k_tree_label<<<grid_for(g.n, 256), 256, 0, s>>>(parent, w.tscan, g.n, w.inbig, w.troot);
    MC_LAUNCHED("k_tree_label");
    k_uf_snapshot<<<grid_for(g.n, 256), 256, 0, s>>>(parent, g.n, w.mode, w.inbig, w.snap, w.tscan + g.n);
    MC_LAUNCHED("k_uf_snapshot");
    prof_begin(PK_PR1_REST, s);
    k_pr1_trees<<<grid_for((int64_t)g.n * SUB, 256), 256, 0, s>>>(g, lam, vinst, w.heavy, w.inbig, w.tscan, w.mode,
                                                                 w.tbits, prof_dev_bytes(PK_PR1_REST));
    MC_LAUNCHED("k_pr1_trees");
    k_pr1_rest<<<grid_for((int64_t)g.n * SUB, 256), 256, 0, s>>>(g, lam, vinst, parent, w.heavy, w.inbig, w.snap,
                                                                w.tscan + g.n, w.spread,
                                                                prof_dev_bytes(PK_PR1_REST));
    MC_LAUNCHED("k_pr1_rest");
    prof_end(PK_PR1_REST, s);
    k_tree_join<<<1, 256, 0, s>>>(w.tscan, g.n, w.tbits, w.troot, w.tmap, marks);
    MC_LAUNCHED("k_tree_join");
    k_tree_apply<<<grid_for(g.n, 256), 256, 0, s>>>(w.tscan, w.inbig, w.tmap, g.n, parent);
    MC_LAUNCHED("k_tree_apply");
    k_pr12_fold<<<1, SPREAD, 0, s>>>(w.spread, marks);
    MC_LAUNCHED("k_pr12_fold");
    k_pr12_long_scan<<<1, 1024, 0, s>>>(g, w.long_list, w.counters, w.task_off);
    MC_LAUNCHED("k_pr12_long_scan");
    k_pr12_long<<<2048, 256, 0, s>>>(g, lam, vinst, parent, marks, flag1, w.long_list, w.counters, w.task_off, w.part_w,
                                     w.part_x);
    MC_LAUNCHED("k_pr12_long");
    k_pr12_long_final<<<256, 64, 0, s>>>(g, parent, marks, ptr2, w.long_list, w.counters, w.task_off, w.part_w,
                                         w.part_x);
    MC_LAUNCHED("k_pr12_long_final");
    return true;
}

bool pr34(const DGraph& g, const int64_t* lam, int32_t D, int32_t* parent, unsigned long long* marks,
          const int32_t* ptr2, Pr34WS& w, uint8_t* flag4, int32_t* acc3, hipStream_t s, const int32_t* vinst) {
    if (D > TRI_MAXD) D = TRI_MAXD;
    if (!fill_i64((int64_t*)w.spread, 0, (int64_t)SPREAD * SPREAD_STRIDE, s) || !fill_i32(w.part3, TRI_NONE, g.n, s) ||
        !fill_u8(w.touch, 0, g.n, s))
        return false;
    if (flag4 && !fill_u8(flag4, 0, g.cap, s)) return false;
    k_pr2_touch<<<grid_for(g.n, 256), 256, 0, s>>>(ptr2, g.n, w.touch);
    MC_LAUNCHED("k_pr2_touch");
    k_pr34<<<grid_for((int64_t)g.n * TRI_SUB, TRI_T), TRI_T, 0, s>>>(g, lam, vinst, D, parent, w.spread, w.part3, flag4);
    MC_LAUNCHED("k_pr34");
    k_pr3_accept<<<grid_for(g.n, 256), 256, 0, s>>>(w.part3, w.touch, g.n, parent, w.spread, acc3);
    MC_LAUNCHED("k_pr3_accept");
    k_pr12_fold<<<1, SPREAD, 0, s>>>(w.spread, marks);
    MC_LAUNCHED("k_pr12_fold");
    return true;
}

void pr34_ws_carve(Arena& a, int32_t n, Pr34WS& w) {
    w.part3 = a.take<int32_t>((size_t)n + 1);
    w.touch = a.take<uint8_t>((size_t)n + 1);
    w.ptr2 = a.take<int32_t>((size_t)n + 1);
    w.spread = a.take<unsigned long long>((size_t)SPREAD * SPREAD_STRIDE);
}

bool map_update(int32_t* map0, const int32_t* L, int32_t n0, hipStream_t s) {
    k_map_update<<<grid_for(n0, 256), 256, 0, s>>>(map0, L, n0);
    MC_LAUNCHED("k_map_update");
    return true;
}

bool side_from_flag(uint8_t* side, const int32_t* map0, int32_t n0, const uint8_t* flag, hipStream_t s) {
    k_side_flag<<<grid_for(n0, 256), 256, 0, s>>>(side, map0, n0, flag);
    MC_LAUNCHED("k_side_flag");
    return true;
}

bool side_from_vertex(uint8_t* side, const int32_t* map0, int32_t n0, const int32_t* target_dev, hipStream_t s) {
    k_side_vertex<<<grid_for(n0, 256), 256, 0, s>>>(side, map0, n0, target_dev);
    MC_LAUNCHED("k_side_vertex");
    return true;
}

bool side_from_prefix(uint8_t* side, const int32_t* map0, int32_t n0, uint8_t* flag, int32_t n,
                      const int32_t* order, const int32_t* len_dev, hipStream_t s) {
    if (!fill_u8(flag, 0, n, s)) return false;
    k_mark_prefix<<<grid_for(n, 256), 256, 0, s>>>(flag, order, len_dev);
    MC_LAUNCHED("k_mark_prefix");
    k_side_flag<<<grid_for(n0, 256), 256, 0, s>>>(side, map0, n0, flag);
    MC_LAUNCHED("k_side_flag");
    return true;
}

bool side_from_components(uint8_t* side, const int32_t* parent, const int32_t* map, int32_t n0, hipStream_t s) {
    k_side_comp<<<grid_for(n0, 256), 256, 0, s>>>(side, parent, map, n0);
    MC_LAUNCHED("k_side_comp");
    return true;
}

bool csr_to_padded(const int32_t* row_ptr, int32_t n, int32_t* off, int32_t* len, hipStream_t s) {
    k_csr_to_padded<<<grid_for(n, 256), 256, 0, s>>>(row_ptr, n, off, len);
    MC_LAUNCHED("k_csr_to_padded");
    return true;
}

bool canon_check(const int32_t* row_ptr, const int32_t* col, const int64_t* w, int32_t n, int32_t nnz, int32_t* len,
                 int64_t* deg, int32_t* noncanon, DevScalars* sc, unsigned long long* part, int32_t* lp1,
                 hipStream_t s) {
    if (!fill_i32(noncanon, 0, 1, s)) return false;
    // with checks, at most 1024 blocks (the partial sums of the weights)
    const int nb = grid_for(((int64_t)n + SUB - 1) / SUB * SUB, 256, sc ? 1024 : 8192);
    k_canon<<<nb, 256, 0, s>>>(row_ptr, col, w, n, nnz, len, deg, noncanon, sc, part, lp1);
    MC_LAUNCHED("k_canon");
    if (sc) {
        k_validate_sum<<<1, 256, 0, s>>>(part, nb, sc);
        MC_LAUNCHED("k_validate_sum");
    }
    return true;
}

