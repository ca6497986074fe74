// Label propagation for the upper-bound heuristic (paper, Section 2.1
// "Lowering the upper bound": the heuristic clusters the graph by label
// propagation, contracts every cluster to one vertex, applies the
// Padberg-Rinaldi tests, and solves the small graph that remains exactly;
// the cut it returns is a cut of the input, so its value bounds lambda).
//
// One synchronous round over all vertices: lab_out[v] is the label that
// carries the most edge weight among v's neighbours (labels of lab_in), with
// two rules that make the round a pure function: v keeps lab_in[v] unless
// another label is strictly heavier, and among equally heavy other labels
// the smallest wins.
//
// Rows of at most LP_SMALL entries are packed into chunks of at most
// LP_CHUNK (entries + rows), as the contraction packs small groups: one
// workgroup sums the (row, label) weights of a chunk in an LDS hash table and
// then takes every row's maximum in two sweeps over the table. Longer rows
// go to a list and are cut into tasks of LP_TASK entries that any workgroup
// may take: a task merges its entries in LDS and adds the sums to the row's
// global hash table (about twice the row's length); two more sweeps over the
// tables, split the same way, find each row's maximum.
#include <algorithm>

#include "mc_internal.h"

namespace {

// Chunks of 256 (entries + rows) on 128 threads: a chunk's work is a chain
// of dependent loads (rows, entries, labels), and smaller workgroups put
// more chunks in flight per compute unit (against 512 on 256 threads:
// Chung-Lu 2^22 1.49 -> 1.15 ms per solve in this kernel, random hyperbolic
// 2^23 2.16 -> 2.00 ms).
constexpr int LP_CHUNK = 256;
constexpr int LP_SMALL = 256;
constexpr int LP_HSLOTS = 512;
constexpr int LP_T = 128;
constexpr int LP_SUB = 16;
constexpr int LP_NSUB = LP_T / LP_SUB;
constexpr int LP_SEG = 2 * LP_SUB;   // entries of a piece of a row in chunks of fewer than LP_NSUB rows
constexpr int LP_TASK = 1024;     // entries per task of a long row (multiple of 128)
constexpr int LP_TSLOTS = 2 * LP_TASK;   // LDS slots of a task's pre-merge
constexpr int LP_IT = LP_TASK / 4;       // threads of the pre-merge: four entries each
constexpr unsigned long long LP_EMPTY = ~0ULL;

inline int grid_for(int64_t count, int threads, int cap = 8192) {
    int64_t b = (count + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

__global__ void k_row_len(const int32_t* __restrict__ len, int32_t n, int32_t* __restrict__ out) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        out[v] = len[v];
}

// cg[c] = first row v with rstart[v] + v >= c LP_CHUNK
__global__ void k_lp_chunks(const int32_t* __restrict__ rstart, int32_t n, int64_t nchunks, int32_t* __restrict__ cg) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= nchunks; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t key = c * LP_CHUNK;
        int32_t lo = 0, hi = n + 1;
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo) / 2;
            if ((int64_t)rstart[mid] + mid >= key) hi = mid; else lo = mid + 1;
        }
        cg[c] = lo;
    }
}

__device__ __forceinline__ uint32_t lp_hash(uint32_t gl, uint32_t lbl) { return hash32(lbl ^ (gl * 0x9E3779B1u)); }

// Row v of l > LP_SMALL entries to the long-row list: its slot k, its
// global table of round_up(2 l, 256) slots, and its tasks of LP_TASK
// entries (the long-row kernels merge it).
__device__ __forceinline__ void lp_list_long(int32_t v, int32_t l, int32_t* __restrict__ long_list,
                                             int32_t* __restrict__ long_base, int32_t* __restrict__ counters,
                                             unsigned long long* __restrict__ long_best,
                                             unsigned long long* __restrict__ long_own,
                                             int32_t* __restrict__ long_lab, int32_t* __restrict__ task_row,
                                             int32_t* __restrict__ task_idx) {
    const int32_t k = atomicAdd(&counters[0], 1);
    const int32_t nt = (l + LP_TASK - 1) / LP_TASK;
    const int32_t t0 = atomicAdd(&counters[2], nt);
    long_list[k] = v;
    long_base[k] = atomicAdd(&counters[1], (2 * l + 255) / 256 * 256);
    long_best[k] = 0;
    long_own[k] = 0;
    long_lab[k] = INT32_MAX;
    for (int32_t t = 0; t < nt; t++) task_row[t0 + t] = k, task_idx[t0 + t] = t;
}

// Entries [j0, j1) of row v (chunk-local gl) into the chunk's LDS table by
// the LP_SUB lanes of a lane group: four entries per lane at a time, so
// their loads, then their labels' loads, are in flight together.
__device__ __forceinline__ void lp_insert(const DGraph& g, const int32_t* __restrict__ lab_in, int32_t v, int gl,
                                          int32_t o, int32_t j0, int32_t j1, int sl, unsigned long long* hkey,
                                          unsigned long long* hval) {
    for (int32_t jb = j0; jb < j1; jb += 4 * LP_SUB) {
        int32_t x[4];
        unsigned long long c[4];
        uint32_t lb[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int32_t j = jb + u * LP_SUB + sl;
            x[u] = j < j1 ? g.col[o + j] : v;
            c[u] = j < j1 ? (unsigned long long)g.w[o + j] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; u++) lb[u] = x[u] != v ? (uint32_t)lab_in[x[u]] : 0;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            if (x[u] == v) continue;   // a loop, or no entry
            const unsigned long long key = ((unsigned long long)gl << 32) | lb[u];
            uint32_t h = lp_hash((uint32_t)gl, lb[u]) & (LP_HSLOTS - 1);
            for (;;) {
                const unsigned long long k = hkey[h];
                if (k == key) break;
                if (k == LP_EMPTY) {
                    const unsigned long long old = atomicCAS(&hkey[h], LP_EMPTY, key);
                    if (old == LP_EMPTY || old == key) break;
                }
                h = (h + 1) & (LP_HSLOTS - 1);
            }
            atomicAdd(&hval[h], c[u]);
        }
    }
}

// General form (any degree, any vertex count): a table of 64-bit keys (row,
// label) and 64-bit sums; the heaviest other weight, then the smallest other
// label of that weight, in two sweeps.
__global__ __launch_bounds__(LP_T) void k_lp_small(DGraph g, const int32_t* __restrict__ lab_in,
                                                  int32_t* __restrict__ lab_out, const int32_t* __restrict__ rstart,
                                                  const int32_t* __restrict__ cg, int32_t* __restrict__ long_list,
                                                  int32_t* __restrict__ long_base, int32_t* __restrict__ counters,
                                                  unsigned long long* __restrict__ long_best,
                                                  unsigned long long* __restrict__ long_own,
                                                  int32_t* __restrict__ long_lab, int32_t* __restrict__ task_row,
                                                  int32_t* __restrict__ task_idx, unsigned long long* pb) {
    __shared__ unsigned long long hkey[LP_HSLOTS];
    __shared__ unsigned long long hval[LP_HSLOTS];
    __shared__ int32_t own[LP_CHUNK];
    __shared__ unsigned long long own_w[LP_CHUNK], best_w[LP_CHUNK];
    __shared__ int32_t best_l[LP_CHUNK];
    __shared__ int32_t roff[LP_CHUNK], rlen[LP_CHUNK];
    __shared__ int32_t spre[LP_NSUB + 1];   // few-row chunks: prefix of the rows' piece counts
    const int tid = threadIdx.x;
    const int32_t g_lo = cg[blockIdx.x];
    const int32_t g_hi = cg[blockIdx.x + 1] < g.n ? cg[blockIdx.x + 1] : g.n;
    if (g_lo >= g.n || g_lo >= g_hi) return;
    const int32_t ng = g_hi - g_lo;
    for (int i = tid; i < LP_HSLOTS; i += LP_T) { hkey[i] = LP_EMPTY; hval[i] = 0; }
    int32_t my_pieces = 0;   // few-row chunks: pieces of row tid
    for (int i = tid; i < ng; i += LP_T) {
        const int32_t v = g_lo + i;
        own[i] = lab_in[v];
        own_w[i] = 0;
        best_w[i] = 0;
        best_l[i] = INT32_MAX;
        const int32_t l = g.len[v];
        roff[i] = g.off[v];
        rlen[i] = l;
        if (l <= LP_SMALL) my_pieces = (l + LP_SEG - 1) / LP_SEG;
        if (l > LP_SMALL) {
            lp_list_long(v, l, long_list, long_base, counters, long_best, long_own, long_lab, task_row, task_idx);
        }
    }
    if (ng < LP_NSUB && tid < MC_WAVE) {
        // few rows (thread i holds row i): inclusive scan of the piece
        // counts over the first lanes of wave 0
        int32_t x = my_pieces;
        for (int d = 1; d < LP_NSUB; d <<= 1) {
            const int32_t y = __shfl_up(x, d, MC_WAVE);
            if (tid >= d) x += y;
        }
        if (tid == 0) spre[0] = 0;
        if (tid < ng) spre[tid + 1] = x;
    }
    __syncthreads();
    const int sg = tid / LP_SUB, sl = tid % LP_SUB;
    if (ng >= LP_NSUB) {
        // many rows: one lane group per row, its entries from j = 0
        for (int gl = sg; gl < ng; gl += LP_NSUB) {
            const int32_t o = roff[gl], l = rlen[gl];
            if (l > LP_SMALL) continue;
            lp_insert(g, lab_in, g_lo + gl, gl, o, 0, l, sl, hkey, hval);
        }
    } else {
        // a few long rows: pieces of LP_SEG entries of any row, one per lane
        // group, so that every lane group stays busy
        for (int32_t k = sg; k < spre[ng]; k += LP_NSUB) {
            int gl = 0;   // the last row with spre[gl] <= k (it has pieces)
            while (gl + 1 < ng && spre[gl + 1] <= k) gl++;
            const int32_t v = g_lo + gl;
            const int32_t o = roff[gl], l = rlen[gl];
            const int32_t j0 = (k - spre[gl]) * LP_SEG;
            lp_insert(g, lab_in, v, gl, o, j0, j0 + LP_SEG < l ? j0 + LP_SEG : l, sl, hkey, hval);
        }
    }
    __syncthreads();
    // sweep 1: own weight, heaviest other weight
    for (int i = tid; i < LP_HSLOTS; i += LP_T) {
        const unsigned long long k = hkey[i];
        if (k == LP_EMPTY) continue;
        const int gl = (int)(k >> 32);
        const int32_t lbl = (int32_t)(k & 0xFFFFFFFFu);
        if (lbl == own[gl]) own_w[gl] = hval[i];
        else atomicMax(&best_w[gl], hval[i]);
    }
    __syncthreads();
    // sweep 2: smallest other label of that weight
    for (int i = tid; i < LP_HSLOTS; i += LP_T) {
        const unsigned long long k = hkey[i];
        if (k == LP_EMPTY) continue;
        const int gl = (int)(k >> 32);
        const int32_t lbl = (int32_t)(k & 0xFFFFFFFFu);
        if (lbl != own[gl] && hval[i] == best_w[gl]) atomicMin(&best_l[gl], lbl);
    }
    __syncthreads();
    int64_t bytes = 0;
    for (int i = tid; i < ng; i += LP_T) {
        const int32_t v = g_lo + i;
        const int32_t l = rlen[i];
        if (l > LP_SMALL) continue;
        lab_out[v] = best_l[i] != INT32_MAX && best_w[i] > own_w[i] ? best_l[i] : own[i];
        bytes += 16 + 16 * (int64_t)l;   // off, len, own label, new label; col, w, label of each target
    }
    if (pb) prof_add(pb, bytes);
}

// Flat form of k_lp_small for graphs below 2^27 vertices whose maximum
// degree is below 2^32. A chunk spans LPF_CHUNK key units, a row counting its
// entries plus LPF_ROWW, so it starts at most LPF_ROWS rows and holds fewer
// than LPF_CHUNK + LP_SMALL entries of short rows. Its threads take those
// entries in order, each up to LPF_PER of them at once (the row of an entry
// by a search of the chunk's row prefix in LDS), so every lane has work and
// the loads of consecutive entries coalesce. A table slot is one 64-bit word:
// the key (chunk-local row, 5 bits; label, 27 bits) high and the label's
// weight sum low, which a 64-bit add updates without carrying into the key.
constexpr int LPF_CHUNK = 512;
constexpr int LPF_ROWW = 16;
constexpr int LPF_ROWS = LPF_CHUNK / LPF_ROWW;   // 32
constexpr int LPF_T = 128;
constexpr int LPF_PER = (LPF_CHUNK + LP_SMALL + LPF_T - 1) / LPF_T;   // 6
constexpr int LPF_SLOTS = 1024;                  // > 767 entries: load below 3/4
constexpr int LPF_LBITS = 27;
constexpr uint32_t LPF_EMPTY = 0xFFFFFFFFu;      // no row 31 holds label 2^27 - 1 (n < 2^27 - 1)
static_assert(LPF_ROWS <= (1 << (32 - LPF_LBITS)), "row index must fit the key");
static_assert(LPF_PER * LPF_T >= LPF_CHUNK + LP_SMALL - 1, "one pass must cover a chunk");

// cg[c] = first row v with rstart[v] + LPF_ROWW v >= c LPF_CHUNK
__global__ void k_lpf_chunks(const int32_t* __restrict__ rstart, int32_t n, int64_t nchunks, int32_t* __restrict__ cg) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= nchunks; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t key = c * LPF_CHUNK;
        int32_t lo = 0, hi = n + 1;
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo) / 2;
            if ((int64_t)rstart[mid] + (int64_t)LPF_ROWW * mid >= key) hi = mid; else lo = mid + 1;
        }
        cg[c] = lo;
    }
}

__global__ __launch_bounds__(LPF_T) void k_lp_flat(DGraph g, const int32_t* __restrict__ lab_in,
                                                  int32_t* __restrict__ lab_out, const int32_t* __restrict__ cg,
                                                  int32_t* __restrict__ long_list, int32_t* __restrict__ long_base,
                                                  int32_t* __restrict__ counters,
                                                  unsigned long long* __restrict__ long_best,
                                                  unsigned long long* __restrict__ long_own,
                                                  int32_t* __restrict__ long_lab, int32_t* __restrict__ task_row,
                                                  int32_t* __restrict__ task_idx, unsigned long long* pb) {
    __shared__ unsigned long long tab[LPF_SLOTS];
    __shared__ unsigned long long best[LPF_ROWS];   // weight high, complemented label low
    __shared__ int32_t rpre[LPF_ROWS + 1];          // prefix of the short rows' lengths
    __shared__ int32_t roff[LPF_ROWS], rlen[LPF_ROWS], own[LPF_ROWS];
    __shared__ uint32_t own_w[LPF_ROWS];
    const int tid = threadIdx.x;
    const int32_t g_lo = cg[blockIdx.x];
    const int32_t g_hi = cg[blockIdx.x + 1] < g.n ? cg[blockIdx.x + 1] : g.n;
    if (g_lo >= g.n || g_lo >= g_hi) return;
    const int32_t ng = g_hi - g_lo;   // at most LPF_ROWS
    for (int i = tid; i < LPF_SLOTS; i += LPF_T) tab[i] = (unsigned long long)LPF_EMPTY << 32;
    int32_t my_short = 0;
    if (tid < ng) {
        const int32_t v = g_lo + tid;
        const int32_t l = g.len[v];
        own[tid] = lab_in[v];
        roff[tid] = g.off[v];
        rlen[tid] = l;
        own_w[tid] = 0;
        best[tid] = 0;
        if (l <= LP_SMALL) {
            my_short = l;
        } else {
            lp_list_long(v, l, long_list, long_base, counters, long_best, long_own, long_lab, task_row, task_idx);
        }
    }
    if (tid < MC_WAVE) {
        // inclusive scan of the short rows' lengths over the lanes of wave 0
        int32_t x = my_short;
        for (int d = 1; d < LPF_ROWS; d <<= 1) {
            const int32_t y = __shfl_up(x, d, MC_WAVE);
            if (tid >= d) x += y;
        }
        if (tid == 0) rpre[0] = 0;
        if (tid < ng) rpre[tid + 1] = x;
    }
    __syncthreads();
    const int32_t E = rpre[ng];
    int32_t r[LPF_PER], x[LPF_PER];
    uint32_t c[LPF_PER], lb[LPF_PER];
#pragma unroll
    for (int q = 0; q < LPF_PER; q++) {
        const int32_t e = q * LPF_T + tid;
        r[q] = -1;
        x[q] = 0;
        c[q] = 0;
        if (e >= E) continue;
        int32_t lo = 0;   // the last row with rpre[lo] <= e (a row with entries, as e < E)
#pragma unroll
        for (int b = LPF_ROWS / 2; b > 0; b >>= 1)
            if (lo + b < ng && rpre[lo + b] <= e) lo += b;
        const int32_t j = roff[lo] + (e - rpre[lo]);
        r[q] = lo;
        x[q] = g.col[j];
        c[q] = (uint32_t)g.w[j];
    }
#pragma unroll
    for (int q = 0; q < LPF_PER; q++) lb[q] = r[q] >= 0 && x[q] != g_lo + r[q] ? (uint32_t)lab_in[x[q]] : 0;
#pragma unroll
    for (int q = 0; q < LPF_PER; q++) {
        if (r[q] < 0 || x[q] == g_lo + r[q]) continue;   // no entry, or a loop
        const uint32_t key = ((uint32_t)r[q] << LPF_LBITS) | lb[q];
        const unsigned long long kw = (unsigned long long)key << 32;
        uint32_t h = hash32(key) & (LPF_SLOTS - 1);
        for (;;) {
            const uint32_t k = (uint32_t)(tab[h] >> 32);
            if (k == key) break;
            if (k == LPF_EMPTY) {
                const unsigned long long old = atomicCAS(&tab[h], (unsigned long long)LPF_EMPTY << 32, kw);
                if ((uint32_t)(old >> 32) == LPF_EMPTY || (uint32_t)(old >> 32) == key) break;
            }
            h = (h + 1) & (LPF_SLOTS - 1);
        }
        atomicAdd(&tab[h], (unsigned long long)c[q]);
    }
    __syncthreads();
    for (int i = tid; i < LPF_SLOTS; i += LPF_T) {
        const unsigned long long t = tab[i];
        const uint32_t key = (uint32_t)(t >> 32);
        if (key == LPF_EMPTY) continue;
        const int row = (int)(key >> LPF_LBITS);
        const uint32_t lbl = key & ((1u << LPF_LBITS) - 1);
        const uint32_t sum = (uint32_t)t;
        if ((int32_t)lbl == own[row]) own_w[row] = sum;
        else atomicMax(&best[row], ((unsigned long long)sum << 32) | (unsigned long long)(~lbl));
    }
    __syncthreads();
    if (tid < ng && rlen[tid] <= LP_SMALL) {
        // sums are at least 1, so a word of 0 means no other label
        const unsigned long long b = best[tid];
        lab_out[g_lo + tid] = b != 0 && (uint32_t)(b >> 32) > own_w[tid] ? (int32_t)(~(uint32_t)b) : own[tid];
    }
    if (pb) {
        int64_t bytes = 0;
        if (tid < ng && rlen[tid] <= LP_SMALL) bytes = 16 + 16 * (int64_t)rlen[tid];
        prof_add(pb, bytes);
    }
}

// Long rows are cut into tasks of LP_TASK entries; task t of row k owns the
// entries [t LP_TASK, (t+1) LP_TASK) and the table slots
// [2 t LP_TASK, 2 (t+1) LP_TASK) of the row's global table, which covers the
// table (LP_TASK is a multiple of 128, the table a multiple of 256 slots).
struct LongTask {
    int32_t k, t, v, o, l, ts;
    int64_t tb;
};
__device__ __forceinline__ LongTask long_task(const DGraph& g, const int32_t* long_list, const int32_t* long_base,
                                              const int32_t* task_row, const int32_t* task_idx, int32_t i) {
    LongTask x;
    x.k = task_row[i];
    x.t = task_idx[i];
    x.v = long_list[x.k];
    x.o = g.off[x.v];
    x.l = g.len[x.v];
    x.ts = (2 * x.l + 255) / 256 * 256;
    x.tb = long_base[x.k];
    return x;
}

__global__ __launch_bounds__(LP_T) void k_lp_long_clear(DGraph g, const int32_t* __restrict__ long_list,
                                                       const int32_t* __restrict__ long_base,
                                                       const int32_t* __restrict__ counters,
                                                       const int32_t* __restrict__ task_row,
                                                       const int32_t* __restrict__ task_idx, int32_t* __restrict__ tkey,
                                                       int64_t* __restrict__ tval) {
    const int32_t ntask = counters[2];
    for (int32_t i = blockIdx.x; i < ntask; i += gridDim.x) {
        const LongTask x = long_task(g, long_list, long_base, task_row, task_idx, i);
        const int32_t s1 = 2 * (x.t + 1) * LP_TASK < x.ts ? 2 * (x.t + 1) * LP_TASK : x.ts;
        for (int32_t k = 2 * x.t * LP_TASK + threadIdx.x; k < s1; k += LP_T) {
            tkey[x.tb + k] = -1;
            tval[x.tb + k] = 0;
        }
    }
}

// each task merges its entries in LDS, then adds the sums to the row's table
__global__ __launch_bounds__(LP_IT) void k_lp_long_insert(DGraph g, const int32_t* __restrict__ lab_in,
                                                        const int32_t* __restrict__ long_list,
                                                        const int32_t* __restrict__ long_base,
                                                        const int32_t* __restrict__ counters,
                                                        const int32_t* __restrict__ task_row,
                                                        const int32_t* __restrict__ task_idx,
                                                        int32_t* __restrict__ tkey, int64_t* __restrict__ tval) {
    __shared__ unsigned long long hkey[LP_TSLOTS];
    __shared__ unsigned long long hval[LP_TSLOTS];
    const int32_t ntask = counters[2];
    for (int32_t i = blockIdx.x; i < ntask; i += gridDim.x) {
        const LongTask x = long_task(g, long_list, long_base, task_row, task_idx, i);
        __syncthreads();
        for (int k = threadIdx.x; k < LP_TSLOTS; k += LP_IT) { hkey[k] = LP_EMPTY; hval[k] = 0; }
        __syncthreads();
        const int32_t j1 = (x.t + 1) * LP_TASK < x.l ? (x.t + 1) * LP_TASK : x.l;
        // the task's LP_TASK / LP_IT entries per thread: loads, then label
        // loads, all in flight together
        constexpr int PER = LP_TASK / LP_IT;
        int32_t y[PER];
        unsigned long long c[PER];
        uint32_t lb[PER];
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int32_t j = x.t * LP_TASK + u * LP_IT + threadIdx.x;
            y[u] = j < j1 ? g.col[x.o + j] : x.v;
            c[u] = j < j1 ? (unsigned long long)g.w[x.o + j] : 0;
        }
#pragma unroll
        for (int u = 0; u < PER; u++) lb[u] = y[u] != x.v ? (uint32_t)lab_in[y[u]] : 0;
#pragma unroll
        for (int u = 0; u < PER; u++) {
            if (y[u] == x.v) continue;   // a loop, or no entry
            const uint32_t lbl = lb[u];
            uint32_t h = hash32(lbl) & (LP_TSLOTS - 1);
            for (;;) {
                const unsigned long long kk = hkey[h];
                if (kk == lbl) break;
                if (kk == LP_EMPTY) {
                    const unsigned long long old = atomicCAS(&hkey[h], LP_EMPTY, (unsigned long long)lbl);
                    if (old == LP_EMPTY || old == lbl) break;
                }
                h = (h + 1) & (LP_TSLOTS - 1);
            }
            atomicAdd(&hval[h], c[u]);
        }
        __syncthreads();
        for (int k = threadIdx.x; k < LP_TSLOTS; k += LP_IT) {
            const unsigned long long kk = hkey[k];
            if (kk == LP_EMPTY) continue;
            const int32_t lbl = (int32_t)kk;
            uint32_t h = (uint32_t)(((uint64_t)hash32((uint32_t)lbl) * (uint32_t)x.ts) >> 32);
            for (;;) {
                const int32_t cur = ld_acq(&tkey[x.tb + h]);
                if (cur == lbl) break;
                if (cur == -1) {
                    const int32_t old = atomicCAS(&tkey[x.tb + h], -1, lbl);
                    if (old == -1 || old == lbl) break;
                }
                if (++h == (uint32_t)x.ts) h = 0;
            }
            atomic_add_i64(&tval[x.tb + h], (int64_t)hval[k]);
        }
    }
}

// sweep 1 over each task's table slots: the row's own-label weight and its
// heaviest other weight (one atomic per workgroup and row)
__global__ __launch_bounds__(LP_T) void k_lp_long_max(DGraph g, const int32_t* __restrict__ lab_in,
                                                     const int32_t* __restrict__ long_list,
                                                     const int32_t* __restrict__ long_base,
                                                     const int32_t* __restrict__ counters,
                                                     const int32_t* __restrict__ task_row,
                                                     const int32_t* __restrict__ task_idx,
                                                     const int32_t* __restrict__ tkey, const int64_t* __restrict__ tval,
                                                     unsigned long long* __restrict__ long_best,
                                                     unsigned long long* __restrict__ long_own) {
    __shared__ unsigned long long r_w[LP_T / MC_WAVE];
    const int32_t ntask = counters[2];
    for (int32_t i = blockIdx.x; i < ntask; i += gridDim.x) {
        const LongTask x = long_task(g, long_list, long_base, task_row, task_idx, i);
        const int32_t ownl = lab_in[x.v];
        const int32_t s1 = 2 * (x.t + 1) * LP_TASK < x.ts ? 2 * (x.t + 1) * LP_TASK : x.ts;
        unsigned long long bw = 0;
        for (int32_t k = 2 * x.t * LP_TASK + threadIdx.x; k < s1; k += LP_T) {
            const int32_t lbl = tkey[x.tb + k];
            if (lbl < 0) continue;
            const unsigned long long sum = (unsigned long long)tval[x.tb + k];
            if (lbl == ownl) long_own[x.k] = sum;   // one slot holds the own label
            else if (sum > bw) bw = sum;
        }
        for (int d = 32; d > 0; d >>= 1) {
            const unsigned long long b2 = __shfl_xor(bw, d, MC_WAVE);
            bw = b2 > bw ? b2 : bw;
        }
        __syncthreads();
        if (lane_id() == 0) r_w[threadIdx.x / MC_WAVE] = bw;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long b = 0;
            for (int k = 0; k < LP_T / MC_WAVE; k++) b = r_w[k] > b ? r_w[k] : b;
            if (b) atomicMax(&long_best[x.k], b);
        }
    }
}

// sweep 2: the smallest other label of the heaviest weight
__global__ __launch_bounds__(LP_T) void k_lp_long_min(DGraph g, const int32_t* __restrict__ lab_in,
                                                     const int32_t* __restrict__ long_list,
                                                     const int32_t* __restrict__ long_base,
                                                     const int32_t* __restrict__ counters,
                                                     const int32_t* __restrict__ task_row,
                                                     const int32_t* __restrict__ task_idx,
                                                     const int32_t* __restrict__ tkey, const int64_t* __restrict__ tval,
                                                     const unsigned long long* __restrict__ long_best,
                                                     int32_t* __restrict__ long_lab) {
    __shared__ int32_t r_l[LP_T / MC_WAVE];
    const int32_t ntask = counters[2];
    for (int32_t i = blockIdx.x; i < ntask; i += gridDim.x) {
        const LongTask x = long_task(g, long_list, long_base, task_row, task_idx, i);
        const int32_t ownl = lab_in[x.v];
        const unsigned long long best = long_best[x.k];
        const int32_t s1 = 2 * (x.t + 1) * LP_TASK < x.ts ? 2 * (x.t + 1) * LP_TASK : x.ts;
        int32_t bl = INT32_MAX;
        for (int32_t k = 2 * x.t * LP_TASK + threadIdx.x; k < s1; k += LP_T) {
            const int32_t lbl = tkey[x.tb + k];
            if (lbl >= 0 && lbl != ownl && (unsigned long long)tval[x.tb + k] == best && lbl < bl) bl = lbl;
        }
        for (int d = 32; d > 0; d >>= 1) {
            const int32_t b2 = __shfl_xor(bl, d, MC_WAVE);
            bl = b2 < bl ? b2 : bl;
        }
        __syncthreads();
        if (lane_id() == 0) r_l[threadIdx.x / MC_WAVE] = bl;
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t m = INT32_MAX;
            for (int k = 0; k < LP_T / MC_WAVE; k++) m = r_l[k] < m ? r_l[k] : m;
            if (m != INT32_MAX) atomicMin(&long_lab[x.k], m);
        }
    }
}

__global__ void k_lp_long_final(const int32_t* __restrict__ lab_in, int32_t* __restrict__ lab_out,
                                const int32_t* __restrict__ long_list, const int32_t* __restrict__ counters,
                                const unsigned long long* __restrict__ long_best,
                                const unsigned long long* __restrict__ long_own, const int32_t* __restrict__ long_lab) {
    const int32_t nl = counters[0];
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < nl; k += gridDim.x * blockDim.x) {
        const int32_t v = long_list[k];
        lab_out[v] = long_lab[k] != INT32_MAX && long_best[k] > long_own[k] ? long_lab[k] : lab_in[v];
    }
}

// The round from singleton labels (lab_in[v] = v) on a normal graph (no
// loop, no parallel entries, positive weights): every neighbour carries its
// own label, so a label's weight is the weight of the one edge to it, the
// own label weighs nothing, and the rule above picks the heaviest
// neighbour, the smallest one on ties (v itself when the row is empty). One
// streaming pass over the rows, 16 lanes per row; rows longer than LP_SMALL
// are listed and take a workgroup each.
__device__ __forceinline__ void lp_better(int64_t c, int32_t x, int64_t& bw, int32_t& bx) {
    if (c > 0 && (c > bw || (c == bw && x < bx))) { bw = c; bx = x; }
}

constexpr int LP_FIRST_TASK = 4096;   // entries per piece of a long row

__global__ __launch_bounds__(256) void k_lp_first(DGraph g, int32_t* __restrict__ lab_out,
                                                 int32_t* __restrict__ long_list, int32_t* __restrict__ long_base,
                                                 int32_t* __restrict__ counters, int32_t* __restrict__ task_row,
                                                 int32_t* __restrict__ task_idx, unsigned long long* pb) {
    const int64_t nsub = (int64_t)gridDim.x * (blockDim.x / LP_SUB);
    const int sl = threadIdx.x % LP_SUB;
    int64_t bytes = 0;
    for (int64_t v = (int64_t)blockIdx.x * (blockDim.x / LP_SUB) + threadIdx.x / LP_SUB; v < g.n; v += nsub) {
        const int32_t o = g.off[v], l = g.len[v];
        if (l > LP_SMALL) {
            // listed with its pieces; the 16 lanes write the task table
            const int32_t nt = (l + LP_FIRST_TASK - 1) / LP_FIRST_TASK;
            int32_t k = 0, t0 = 0;
            if (sl == 0) {
                k = atomicAdd(&counters[0], 1);
                t0 = atomicAdd(&counters[2], nt);
                long_list[k] = (int32_t)v;
                long_base[k] = t0;
            }
            k = __shfl(k, 0, LP_SUB);
            t0 = __shfl(t0, 0, LP_SUB);
            for (int32_t t = sl; t < nt; t += LP_SUB) { task_row[t0 + t] = k; task_idx[t0 + t] = t; }
            continue;
        }
        int64_t bw = 0;
        int32_t bx = INT32_MAX;
        int32_t j = sl;
        for (; j + 3 * LP_SUB < l; j += 4 * LP_SUB) {   // four independent loads in flight
            int32_t x[4];
            int64_t c[4];
            for (int u = 0; u < 4; u++) { x[u] = g.col[o + j + u * LP_SUB]; c[u] = g.w[o + j + u * LP_SUB]; }
            for (int u = 0; u < 4; u++) if (x[u] != (int32_t)v) lp_better(c[u], x[u], bw, bx);
        }
        for (; j < l; j += LP_SUB) {
            const int32_t x = g.col[o + j];
            if (x != (int32_t)v) lp_better(g.w[o + j], x, bw, bx);
        }
        for (int k = LP_SUB / 2; k > 0; k >>= 1) {
            const int64_t w2 = __shfl_xor(bw, k, LP_SUB);
            const int32_t x2 = __shfl_xor(bx, k, LP_SUB);
            if (w2 > bw || (w2 == bw && x2 < bx)) { bw = w2; bx = x2; }
        }
        if (sl == 0) {
            lab_out[v] = bx != INT32_MAX ? bx : (int32_t)v;
            bytes += 12 + 12 * (int64_t)l;   // off, len, label; col and w of each entry
        }
    }
    if (pb) prof_add(pb, bytes);
}

// one workgroup per piece of a long row: the piece's heaviest entry
__global__ __launch_bounds__(256) void k_lp_first_long(DGraph g, const int32_t* __restrict__ long_list,
                                                      const int32_t* __restrict__ counters,
                                                      const int32_t* __restrict__ task_row,
                                                      const int32_t* __restrict__ task_idx,
                                                      int64_t* __restrict__ part_w, int32_t* __restrict__ part_x) {
    __shared__ int64_t sw[256 / MC_WAVE];
    __shared__ int32_t sx[256 / MC_WAVE];
    const int32_t ntask = counters[2];
    for (int32_t i = blockIdx.x; i < ntask; i += gridDim.x) {
        const int32_t v = long_list[task_row[i]];
        const int32_t o = g.off[v], l = g.len[v];
        const int32_t j0 = task_idx[i] * LP_FIRST_TASK;
        const int32_t j1 = j0 + LP_FIRST_TASK < l ? j0 + LP_FIRST_TASK : l;
        int64_t bw = 0;
        int32_t bx = INT32_MAX;
        for (int32_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
            const int32_t x = g.col[o + j];
            if (x != v) lp_better(g.w[o + j], x, bw, bx);
        }
        for (int k = MC_WAVE / 2; k > 0; k >>= 1) {
            const int64_t w2 = __shfl_xor(bw, k, MC_WAVE);
            const int32_t x2 = __shfl_xor(bx, k, MC_WAVE);
            if (w2 > bw || (w2 == bw && x2 < bx)) { bw = w2; bx = x2; }
        }
        __syncthreads();
        if (lane_id() == 0) { sw[threadIdx.x / MC_WAVE] = bw; sx[threadIdx.x / MC_WAVE] = bx; }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int k = 1; k < 256 / MC_WAVE; k++)
                if (sw[k] > bw || (sw[k] == bw && sx[k] < bx)) { bw = sw[k]; bx = sx[k]; }
            part_w[i] = bw;
            part_x[i] = bx;
        }
    }
}

// one wavefront per long row: fold its pieces
__global__ __launch_bounds__(MC_WAVE) void k_lp_first_fold(DGraph g, int32_t* __restrict__ lab_out,
                                                          const int32_t* __restrict__ long_list,
                                                          const int32_t* __restrict__ long_base,
                                                          const int32_t* __restrict__ counters,
                                                          const int64_t* __restrict__ part_w,
                                                          const int32_t* __restrict__ part_x) {
    const int32_t nl = counters[0];
    for (int32_t k = blockIdx.x; k < nl; k += gridDim.x) {
        const int32_t v = long_list[k];
        const int32_t nt = (g.len[v] + LP_FIRST_TASK - 1) / LP_FIRST_TASK;
        int64_t bw = 0;
        int32_t bx = INT32_MAX;
        for (int32_t t = threadIdx.x; t < nt; t += MC_WAVE) {
            const int64_t w2 = part_w[long_base[k] + t];
            const int32_t x2 = part_x[long_base[k] + t];
            if (w2 > bw || (w2 == bw && x2 < bx)) { bw = w2; bx = x2; }
        }
        for (int d = MC_WAVE / 2; d > 0; d >>= 1) {
            const int64_t w2 = __shfl_xor(bw, d, MC_WAVE);
            const int32_t x2 = __shfl_xor(bx, d, MC_WAVE);
            if (w2 > bw || (w2 == bw && x2 < bx)) { bw = w2; bx = x2; }
        }
        if (threadIdx.x == 0) lab_out[v] = bx != INT32_MAX ? bx : v;
    }
}

// flag[l] = 1 for every label in use (flag zeroed before)
// flag[0] = 1 when some row's weight sum reaches 2^32 (one thread per row)
__global__ void k_lp_wide_rows(DGraph g, int32_t* __restrict__ flag) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t o = g.off[v], l = g.len[v];
        unsigned long long d = 0;
        for (int32_t j = 0; j < l && d < (1ULL << 32); j++) d += (unsigned long long)g.w[o + j];
        if (d >= (1ULL << 32)) flag[0] = 1;
    }
}

__global__ void k_label_used(const int32_t* __restrict__ lab, int32_t n, int32_t* __restrict__ flag) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        flag[lab[v]] = 1;
}

__global__ void k_label_rank(const int32_t* __restrict__ lab, const int32_t* __restrict__ rank, int32_t n,
                             int32_t* __restrict__ L, DevScalars* sc) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        L[v] = rank[lab[v]];
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->n2 = rank[n];
}

}  // namespace

void lp_ws_carve(Arena& a, int32_t n, int64_t cap, LpWS& w) {
    const size_t nlong = (size_t)std::min<int64_t>(n, cap / LP_SMALL + 1) + 64;
    w.long_list = a.take<int32_t>(nlong);
    w.long_base = a.take<int32_t>(nlong);
    w.long_lab = a.take<int32_t>(nlong);
    w.long_best = a.take<unsigned long long>(nlong);
    w.long_own = a.take<unsigned long long>(nlong);
    // tasks: at most cap / LP_TASK + one per long row
    const size_t ntask = (size_t)(cap / LP_TASK) + nlong;
    w.task_row = a.take<int32_t>(ntask);
    w.task_idx = a.take<int32_t>(ntask);
    w.counters = a.take<int32_t>(4);
    // chunk starts of either chunking (LPF_ROWW n / LPF_CHUNK >= n / LP_CHUNK)
    w.cg = a.take<int32_t>((size_t)((cap + (int64_t)LPF_ROWW * n) / LPF_CHUNK) + (size_t)((cap + n) / LP_CHUNK) + 4);
}

bool lp_round(const DGraph& g, const int32_t* lab_in, int32_t* lab_out, LpWS& w, ContractWS& cw, hipStream_t s,
              bool narrow) {
    const int32_t n = g.n;
    // row prefix (entries) of the current rows -> chunk starts
    k_row_len<<<grid_for(n, 256), 256, 0, s>>>(g.len, n, cw.mstart);
    MC_LAUNCHED("k_row_len");
    if (!scan_i32(cw.mstart, cw.mstart, n, cw.scan_tmp, s)) return false;
    if (!fill_i32(w.counters, 0, 4, s)) return false;
    if (narrow && n < (1 << LPF_LBITS) - 1) {
        // chunk keys run up to entries + LPF_ROWW rows <= cap + LPF_ROWW n
        const int64_t nchunks = (g.cap + (int64_t)LPF_ROWW * n) / LPF_CHUNK + 2;
        k_lpf_chunks<<<grid_for(nchunks + 1, 256), 256, 0, s>>>(cw.mstart, n, nchunks, w.cg);
        MC_LAUNCHED("k_lpf_chunks");
        prof_begin(PK_LP_SMALL, s);
        k_lp_flat<<<(unsigned)nchunks, LPF_T, 0, s>>>(g, lab_in, lab_out, w.cg, w.long_list, w.long_base, w.counters,
                                                      w.long_best, w.long_own, w.long_lab, w.task_row, w.task_idx,
                                                      prof_dev_bytes(PK_LP_SMALL));
        MC_LAUNCHED("k_lp_flat");
    } else {
    // chunk keys run up to (entries + rows) <= cap + n
    const int64_t nchunks = (g.cap + n) / LP_CHUNK + 2;
    k_lp_chunks<<<grid_for(nchunks + 1, 256), 256, 0, s>>>(cw.mstart, n, nchunks, w.cg);
    MC_LAUNCHED("k_lp_chunks");
    prof_begin(PK_LP_SMALL, s);
    k_lp_small<<<(unsigned)nchunks, LP_T, 0, s>>>(g, lab_in, lab_out, cw.mstart, w.cg, w.long_list, w.long_base,
                                                  w.counters, w.long_best, w.long_own, w.long_lab, w.task_row,
                                                  w.task_idx, prof_dev_bytes(PK_LP_SMALL));
    MC_LAUNCHED("k_lp_small");
    }
    prof_end(PK_LP_SMALL, s);
    const int tb = 2048;
    k_lp_long_clear<<<tb, LP_T, 0, s>>>(g, w.long_list, w.long_base, w.counters, w.task_row, w.task_idx, cw.tkey,
                                        cw.tval);
    MC_LAUNCHED("k_lp_long_clear");
    k_lp_long_insert<<<tb, LP_IT, 0, s>>>(g, lab_in, w.long_list, w.long_base, w.counters, w.task_row, w.task_idx,
                                         cw.tkey, cw.tval);
    MC_LAUNCHED("k_lp_long_insert");
    k_lp_long_max<<<tb, LP_T, 0, s>>>(g, lab_in, w.long_list, w.long_base, w.counters, w.task_row, w.task_idx,
                                      cw.tkey, cw.tval, w.long_best, w.long_own);
    MC_LAUNCHED("k_lp_long_max");
    k_lp_long_min<<<tb, LP_T, 0, s>>>(g, lab_in, w.long_list, w.long_base, w.counters, w.task_row, w.task_idx,
                                      cw.tkey, cw.tval, w.long_best, w.long_lab);
    MC_LAUNCHED("k_lp_long_min");
    k_lp_long_final<<<64, 256, 0, s>>>(lab_in, lab_out, w.long_list, w.counters, w.long_best, w.long_own,
                                       w.long_lab);
    MC_LAUNCHED("k_lp_long_final");
    return true;
}

bool lp_narrow(const DGraph& g, int32_t* flag_tmp, bool* narrow, hipStream_t s) {
    int32_t h = 0;
    if (!fill_i32(flag_tmp, 0, 1, s)) return false;
    k_lp_wide_rows<<<grid_for(g.n, 256), 256, 0, s>>>(g, flag_tmp);
    MC_LAUNCHED("k_lp_wide_rows");
    if (hipMemcpyAsync(&h, flag_tmp, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return false;
    *narrow = h == 0;
    return true;
}

bool lp_first(const DGraph& g, int32_t* lab_out, LpWS& w, ContractWS& cw, hipStream_t s) {
    if (!fill_i32(w.counters, 0, 4, s)) return false;
    prof_begin(PK_LP_FIRST, s);
    k_lp_first<<<grid_for((int64_t)g.n * LP_SUB, 256), 256, 0, s>>>(g, lab_out, w.long_list, w.long_base, w.counters,
                                                                   w.task_row, w.task_idx, prof_dev_bytes(PK_LP_FIRST));
    MC_LAUNCHED("k_lp_first");
    prof_end(PK_LP_FIRST, s);
    // piece partials go to the large-group table arrays (>= 2.5 cap slots,
    // more than the pieces)
    k_lp_first_long<<<2048, 256, 0, s>>>(g, w.long_list, w.counters, w.task_row, w.task_idx, cw.tval, cw.tkey);
    MC_LAUNCHED("k_lp_first_long");
    k_lp_first_fold<<<1024, MC_WAVE, 0, s>>>(g, lab_out, w.long_list, w.long_base, w.counters, cw.tval, cw.tkey);
    MC_LAUNCHED("k_lp_first_fold");
    return true;
}

bool lp_relabel(const int32_t* lab, int32_t n, int32_t* L, int32_t* flag_tmp, int32_t* scan_tmp, DevScalars* sc,
                hipStream_t s) {
    if (!fill_i32(flag_tmp, 0, (int64_t)n + 1, s)) return false;
    k_label_used<<<grid_for(n, 256), 256, 0, s>>>(lab, n, flag_tmp);
    MC_LAUNCHED("k_label_used");
    if (!scan_i32(flag_tmp, flag_tmp, n, scan_tmp, s)) return false;
    k_label_rank<<<grid_for(n, 256), 256, 0, s>>>(lab, flag_tmp, n, L, sc);
    MC_LAUNCHED("k_label_rank");
    return true;
}
