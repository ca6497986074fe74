// Graph contraction (paper, Section 2 "Basic Concepts" and Section 2.1
// "Parallel CAPFOREST and contraction"; Algorithm 2, contraction step).
//
// Given labels L: V -> [0, n2), vertex g of the result stands for the group
// {v : L[v] = g}; every entry v->x becomes g->L[x], loops (L[v] = L[x]) and
// zero weights vanish, entries between the same pair of groups add up. The
// degree of a collapsed vertex (the sum of its new row) is written at the
// same time; it is the capacity of the cut around the group.
//
// The merge is organised by contracted vertex, as the paper's accepted
// change 3 of the parallel session suggests, but in a GPU form:
//  1. counting sort of the vertices by label (atomics + scan): the members
//     of group g are perm[vstart[g] .. vstart[g+1]);
//  2. a scan of the member row lengths gives every group a private output
//     window [gstart[g], gstart[g+1]) as large as all rows it absorbs, so
//     new rows are written in place without a global offset pass (the
//     result is a padded CSR with off/len per row);
//  3. small groups (<= 512 entries) are packed into chunks of <= 1023
//     entries; one workgroup merges a chunk in an LDS hash table keyed by
//     (group, target) with 64-bit LDS atomics, then writes the rows;
//  4. large groups (hubs, big clusters) get a global hash table of about
//     2x their entries; one wavefront per member row inserts with global
//     CAS/atomic add, and 256-slot tiles are extracted in parallel.
// Streaming traffic per entry: 12 B read (col, w) + 4 B label gather +
// 12 B written per surviving entry.
#include "mc_internal.h"

namespace {

constexpr int CHUNK = 512;          // chunk span in (entry offset + GROUP_W group index)
constexpr int GROUP_W = 4;          // key units of a group: a chunk starts at most CHUNK / GROUP_W groups
constexpr int CHUNK_GROUPS = CHUNK / GROUP_W;
constexpr int SMALL_MAX = 512;      // larger groups take the global-table path
constexpr int HSLOTS = 1024;        // LDS hash slots per chunk (> the most entries a chunk holds)
constexpr int TILE_SLOTS = 256;     // global-table allocation and extraction unit
constexpr uint64_t EMPTY_KEY = ~0ULL;

// Counting sort of vertices by label. Contraction often sends a large part
// of the graph to one label (a giant group), and atomics on one address
// serialise, so each workgroup first combines its tile of GT vertices in an
// LDS table keyed by label and then issues one global atomic per distinct
// label of the tile.
constexpr int GT = 2048;            // vertices per workgroup tile
constexpr int GT_SLOTS = 4096;      // LDS table slots (load <= 1/2)
constexpr int GT_THREADS = 256;
constexpr int GT_PER = GT / GT_THREADS;

// insert label g into the tile table; returns its slot
__device__ __forceinline__ int gt_insert(int32_t* key, int32_t* cnt, int32_t g) {
    uint32_t h = hash32((uint32_t)g) & (GT_SLOTS - 1);
    for (;;) {
        const int32_t k = key[h];
        if (k == g) break;
        if (k == -1) {
            const int32_t old = atomicCAS(&key[h], -1, g);
            if (old == -1 || old == g) break;
        }
        h = (h + 1) & (GT_SLOTS - 1);
    }
    atomicAdd(&cnt[h], 1);
    return (int)h;
}

__global__ __launch_bounds__(GT_THREADS) void k_group_count(const int32_t* __restrict__ L, int32_t n,
                                                           int32_t* __restrict__ gcnt) {
    __shared__ int32_t key[GT_SLOTS], cnt[GT_SLOTS];
    const int64_t tiles = ((int64_t)n + GT - 1) / GT;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        for (int i = threadIdx.x; i < GT_SLOTS; i += GT_THREADS) { key[i] = -1; cnt[i] = 0; }
        __syncthreads();
        for (int k = 0; k < GT_PER; k++) {
            const int64_t u = t * GT + k * GT_THREADS + threadIdx.x;
            if (u < n && L[u] >= 0) gt_insert(key, cnt, L[u]);   // label -1: the vertex is dropped
        }
        __syncthreads();
        for (int i = threadIdx.x; i < GT_SLOTS; i += GT_THREADS)
            if (key[i] >= 0) atomicAdd(&gcnt[key[i]], cnt[i]);
        __syncthreads();
    }
}

// Same tiles: each distinct label of the tile reserves its members' places
// with one global atomic; members then take consecutive places in LDS.
__global__ __launch_bounds__(GT_THREADS) void k_group_scatter(const int32_t* __restrict__ L, int32_t n,
                                                             const int32_t* __restrict__ vstart,
                                                             int32_t* __restrict__ gcur, int32_t* __restrict__ perm) {
    __shared__ int32_t key[GT_SLOTS], cnt[GT_SLOTS];
    const int64_t tiles = ((int64_t)n + GT - 1) / GT;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        for (int i = threadIdx.x; i < GT_SLOTS; i += GT_THREADS) { key[i] = -1; cnt[i] = 0; }
        __syncthreads();
        int slot[GT_PER];
        for (int k = 0; k < GT_PER; k++) {
            const int64_t u = t * GT + k * GT_THREADS + threadIdx.x;
            slot[k] = u < n && L[u] >= 0 ? gt_insert(key, cnt, L[u]) : -1;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < GT_SLOTS; i += GT_THREADS) {
            const int32_t g = key[i];
            if (g >= 0) cnt[i] = vstart[g] + atomicAdd(&gcur[g], cnt[i]);
        }
        __syncthreads();
        for (int k = 0; k < GT_PER; k++) {
            if (slot[k] < 0) continue;
            const int64_t u = t * GT + k * GT_THREADS + threadIdx.x;
            perm[atomicAdd(&cnt[slot[k]], 1)] = (int32_t)u;
        }
        __syncthreads();
    }
}

// row length of every member in perm order; positions past the kept
// members (vertices dropped with label -1) get 0
__global__ void k_member_len(const int32_t* __restrict__ len, const int32_t* __restrict__ perm, int32_t n,
                             const int32_t* __restrict__ kept, int32_t* __restrict__ mlen) {
    const int64_t nk = kept ? *kept : n;
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < n; m += (int64_t)gridDim.x * blockDim.x)
        mlen[m] = m < nk ? len[perm ? perm[m] : m] : 0;
}

__global__ void k_group_start(const int32_t* __restrict__ vstart, const int32_t* __restrict__ mstart, int32_t n2,
                              int32_t* __restrict__ gstart) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g <= n2; g += (int64_t)gridDim.x * blockDim.x)
        gstart[g] = mstart[vstart[g]];
}

// Split groups into the chunk path and the large-group path; every group
// gets its output window start. Giant groups (at least a quarter of n2
// entries, so a table of twice their entries would be at least half as long
// as n2) accumulate into a dense array over all n2 targets instead of a hash
// table: no probing, a footprint of 8 n2 bytes, and the extraction is a
// stream over n2 values. The accumulator area is a fixed budget, so the
// number of dense groups is at most budget / n2 (and DENSE_MAX).
constexpr int DENSE_MAX = 1024;

// Groups of (SMALL_MAX, MID_MAX] entries and at most MID_MEM members (and
// the small groups of many members, below) are merged by one workgroup each,
// entirely in LDS: no global atomics, and the row is written in place.
// Larger groups take the tile path below.
constexpr int MID_MAX = 2048;
constexpr int MID_MEM = 1024;
constexpr int MID_T = 512;
// Groups of at most MID_HALF entries take a table of 2048 slots (32 KB of
// LDS per workgroup of eight waves, four workgroups per compute unit),
// larger ones 4096 slots (56 KB, two per compute unit): the merge of a group
// waits on its loads, and more waves in flight hide more of that. Both keep
// the table's load at most 1/2.
constexpr int MID_HALF = 1024;
// Small groups of more than MERGE_MANY members (and at most MID_MEM) are
// merged by the mid-group workgroups too: the chunk merge walks a group's
// members one after the other (a chain of dependent loads each), where a
// mid-group workgroup stages all of them at once and takes the entries flat.
constexpr int MERGE_MANY = 32;

__global__ void k_classify(const int32_t* __restrict__ gstart, const int32_t* __restrict__ vstart, int32_t n2,
                           int32_t nd_max, int32_t* __restrict__ tsize, int32_t* __restrict__ bigm,
                           int32_t* __restrict__ bcur, int32_t* __restrict__ dslot, int32_t* __restrict__ dinfo,
                           int32_t* __restrict__ mlist, int32_t* __restrict__ mcnt, int32_t* __restrict__ ssize,
                           DGraph dst) {
    const int64_t dense_min = n2 / 4;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n2; g += (int64_t)gridDim.x * blockDim.x) {
        int32_t s = gstart[g + 1] - gstart[g];
        dst.off[g] = gstart[g];
        dslot[g] = -1;
        const int32_t members = vstart ? vstart[g + 1] - vstart[g] : 1;
        const bool mid = members <= MID_MEM && (s > SMALL_MAX ? s <= MID_MAX : members > MERGE_MANY);
        ssize[g] = s <= SMALL_MAX && !mid ? s : 0;
        // groups of at most MID_HALF entries from the front of the list,
        // larger ones from the back; a wavefront reserves its places with one
        // atomic per list (two counters shared by every group serialise)
        const bool front = mid && s <= MID_HALF, back = mid && s > MID_HALF;
        const unsigned long long mfr = __ballot(front), mbk = __ballot(back);
        const unsigned long long below = (1ULL << lane_id()) - 1;
        const int lead_f = mfr ? __ffsll((long long)mfr) - 1 : 0;
        const int lead_b = mbk ? __ffsll((long long)mbk) - 1 : 0;
        int32_t base_f = 0, base_b = 0;
        if (mfr && lane_id() == lead_f) base_f = atomicAdd(&mcnt[0], __popcll(mfr));
        if (mbk && lane_id() == lead_b) base_b = atomicAdd(&mcnt[1], __popcll(mbk));
        base_f = __shfl(base_f, lead_f, MC_WAVE);
        base_b = __shfl(base_b, lead_b, MC_WAVE);
        if (mid) {
            if (front) mlist[base_f + __popcll(mfr & below)] = (int32_t)g;
            else mlist[n2 - (base_b + __popcll(mbk & below))] = (int32_t)g;
            tsize[g] = 0;
            bigm[g] = 0;
        } else if (s > SMALL_MAX) {
            int32_t d = -1;
            if (s >= dense_min && nd_max > 0) {
                d = atomicAdd(&dinfo[0], 1);
                if (d < nd_max) { dslot[g] = d; dinfo[1 + d] = (int32_t)g; } else d = -1;
            }
            const int64_t t = ((2 * (int64_t)s + TILE_SLOTS - 1) / TILE_SLOTS) * TILE_SLOTS;
            tsize[g] = d >= 0 ? 0 : (int32_t)t;
            bigm[g] = s;
            bcur[g] = 0;
            dst.len[g] = 0;
            dst.deg[g] = 0;
        } else {
            tsize[g] = 0;
            bigm[g] = 0;
        }
    }
}

// last index g in [0, n) with a[g] <= key (a non-decreasing, a[0] <= key)
__device__ __forceinline__ int32_t last_le(const int32_t* __restrict__ a, int32_t n, int64_t key) {
    int32_t lo = 0, hi = n;  // answer in [lo, hi)
    while (hi - lo > 1) {
        int32_t mid = lo + (hi - lo) / 2;
        if ((int64_t)a[mid] <= key) lo = mid; else hi = mid;
    }
    return lo;
}

// first g in [0, n2] with sstart[g] + GROUP_W g >= key
__device__ __forceinline__ int32_t first_key_ge(const int32_t* __restrict__ sstart, int32_t n2, int64_t key) {
    int32_t lo = 0, hi = n2 + 1;
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if ((int64_t)sstart[mid] + (int64_t)GROUP_W * mid >= key) hi = mid; else lo = mid + 1;
    }
    return lo;
}

constexpr int MERGE_THREADS = 256;
constexpr int SUB = 16;                              // lanes per group
constexpr int NSUB = MERGE_THREADS / SUB;

// first group of every chunk: cg[c] = first g with sstart[g] + GROUP_W g >= c CHUNK,
// sstart the prefix of the small groups' entry counts (larger groups count
// as empty, so no chunk is spent on their entries); one independent search
// per thread, so their latencies overlap
__global__ void k_chunk_start(const int32_t* __restrict__ sstart, int32_t n2, int64_t nchunks,
                              int32_t* __restrict__ cg) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= nchunks; c += (int64_t)gridDim.x * blockDim.x)
        cg[c] = first_key_ge(sstart, n2, c * CHUNK);
}

// One member row u of group g (chunk-local gl) into the chunk's LDS table,
// by the SUB lanes of a lane group: four entries per lane at a time, so their
// loads, then the labels of their targets, are in flight together.
__device__ __forceinline__ void merge_row(const DGraph& src, const int32_t* __restrict__ L, int32_t u, int32_t g,
                                          int gl, int sl, unsigned long long* hkey, long long* hval,
                                          int64_t& nin) {
    const int32_t o = src.off[u], l = src.len[u];
    if (sl == 0) nin += l;
    for (int32_t j0 = 0; j0 < l; j0 += 4 * SUB) {
        int32_t x[4], t[4];
        int64_t c[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int32_t j = j0 + q * SUB + sl;
            x[q] = j < l ? src.col[o + j] : 0;
            c[q] = j < l ? src.w[o + j] : 0;
        }
#pragma unroll
        for (int q = 0; q < 4; q++) t[q] = c[q] > 0 ? (L ? L[x[q]] : x[q]) : g;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            if (t[q] == g) continue;   // a loop, zero weight or no entry
            const unsigned long long key = ((unsigned long long)gl << 32) | (uint32_t)t[q];
            uint32_t h = hash32((uint32_t)t[q] ^ ((uint32_t)gl * 0x9E3779B1u)) & (HSLOTS - 1);
            for (;;) {
                unsigned long long k = hkey[h];
                if (k == key) break;
                if (k == EMPTY_KEY) {
                    unsigned long long old = atomicCAS(&hkey[h], EMPTY_KEY, key);
                    if (old == EMPTY_KEY || old == key) break;
                }
                h = (h + 1) & (HSLOTS - 1);
            }
            atomicAdd((unsigned long long*)&hval[h], (unsigned long long)c[q]);
        }
    }
}

// Algorithmic bytes (profiling): per input entry 12 B (col, w) plus 4 B for
// the label of its target; per output entry 12 B; per group 12 B (len, deg).
__global__ __launch_bounds__(MERGE_THREADS) void k_merge_small(DGraph src, const int32_t* __restrict__ L,
                                                              const int32_t* __restrict__ perm,
                                                              const int32_t* __restrict__ vstart,
                                                              const int32_t* __restrict__ gstart, int32_t n2,
                                                              const int32_t* __restrict__ cg, DGraph dst,
                                                              unsigned long long* pb) {
    __shared__ unsigned long long hkey[HSLOTS];
    __shared__ long long hval[HSLOTS];
    __shared__ int32_t gst[CHUNK_GROUPS + 1];
    __shared__ int32_t gvs[CHUNK_GROUPS + 1];
    __shared__ int32_t gcur[CHUNK_GROUPS];
    __shared__ long long gdeg[CHUNK_GROUPS];
    __shared__ int32_t mpre[NSUB + 1];   // few-group chunks: prefix of the small groups' member counts

    const int tid = threadIdx.x;
    const int32_t g_lo = cg[blockIdx.x];
    const int32_t g_hi = cg[blockIdx.x + 1] < n2 ? cg[blockIdx.x + 1] : n2;
    if (g_lo >= n2 || g_lo >= g_hi) return;
    int64_t nin = 0, nout = 0, ngrp = 0;
    const int32_t ng = g_hi - g_lo;
    for (int i = tid; i < HSLOTS; i += MERGE_THREADS) { hkey[i] = EMPTY_KEY; hval[i] = 0; }
    for (int i = tid; i <= ng; i += MERGE_THREADS) {
        gst[i] = gstart[g_lo + i];
        gvs[i] = vstart ? vstart[g_lo + i] : g_lo + i;
    }
    for (int i = tid; i < ng; i += MERGE_THREADS) { gcur[i] = 0; gdeg[i] = 0; }
    __syncthreads();

    // the groups merged here: at most SMALL_MAX entries, and not the many-
    // member ones the mid-group workgroups take (as k_classify splits them)
    auto here = [&](int gl) {
        const int32_t mc = gvs[gl + 1] - gvs[gl];
        return gst[gl + 1] - gst[gl] <= SMALL_MAX && !(mc > MERGE_MANY && mc <= MID_MEM);
    };
    const int sg = tid / SUB, sl = tid % SUB;
    if (ng >= NSUB) {
        // many groups: one lane group per group, its members in turn
        for (int gl = sg; gl < ng; gl += NSUB) {
            if (!here(gl)) continue;
            for (int32_t m = gvs[gl]; m < gvs[gl + 1]; m++)
                merge_row(src, L, perm ? perm[m] : m, g_lo + gl, gl, sl, hkey, hval, nin);
        }
    } else {
        // a few groups (large ones, each with many members): the members of
        // the small groups NSUB at a time whatever their group, so every
        // lane group stays busy
        if (tid == 0) {
            int32_t run = 0;
            for (int gl = 0; gl < ng; gl++) {
                mpre[gl] = run;
                if (here(gl)) run += gvs[gl + 1] - gvs[gl];
            }
            mpre[ng] = run;
        }
        __syncthreads();
        for (int32_t k = sg; k < mpre[ng]; k += NSUB) {
            int gl = 0;   // the last group with mpre[gl] <= k (it has members)
            while (gl + 1 < ng && mpre[gl + 1] <= k) gl++;
            const int32_t m = gvs[gl] + (k - mpre[gl]);
            merge_row(src, L, perm ? perm[m] : m, g_lo + gl, gl, sl, hkey, hval, nin);
        }
    }
    __syncthreads();
    for (int i = tid; i < HSLOTS; i += MERGE_THREADS) {
        unsigned long long k = hkey[i];
        if (k == EMPTY_KEY) continue;
        const int gl = (int)(k >> 32);
        const int32_t t = (int32_t)(k & 0xFFFFFFFFu);
        const int64_t s = hval[i];
        const int32_t pos = atomicAdd(&gcur[gl], 1);
        dst.col[gst[gl] + pos] = t;
        dst.w[gst[gl] + pos] = s;
        atomicAdd((unsigned long long*)&gdeg[gl], (unsigned long long)s);
        nout++;
    }
    __syncthreads();
    for (int gl = tid; gl < ng; gl += MERGE_THREADS) {
        if (!here(gl)) continue;
        dst.len[g_lo + gl] = gcur[gl];
        dst.deg[g_lo + gl] = gdeg[gl];
        ngrp++;
    }
    if (pb) prof_add(pb, nin * (L ? 16 : 12) + nout * 12 + ngrp * 12);
}

// A mid group's place in the list and sizes.
struct MidMeta {
    int32_t g, m0, mc, gs, s;
};
__device__ __forceinline__ MidMeta mid_meta(int32_t g, const int32_t* __restrict__ vstart,
                                            const int32_t* __restrict__ gstart) {
    MidMeta m{g, 0, 0, 0, 0};
    if (g < 0) return m;
    m.m0 = vstart ? vstart[g] : g;
    m.mc = vstart ? vstart[g + 1] - m.m0 : 1;
    m.gs = gstart[g];
    m.s = gstart[g + 1] - m.gs;
    return m;
}

// One workgroup per mid group, looping over the list. The merge of a group
// is a chain of dependent loads (list entry, group bounds, member rows,
// entries, target labels), so the loop is software-pipelined: while group A
// merges its entries, the member offsets of the next group B are loaded
// into registers, the bounds of the group C after it and the list entry of
// the one after that, so each group waits for two dependent loads (entries,
// then labels) instead of six.
template <int MID_SLOTS>
__global__ __launch_bounds__(MID_T) void k_mid_merge(DGraph src, const int32_t* __restrict__ L,
                                                    const int32_t* __restrict__ perm,
                                                    const int32_t* __restrict__ vstart,
                                                    const int32_t* __restrict__ mstart,
                                                    const int32_t* __restrict__ gstart,
                                                    const int32_t* __restrict__ mlist,
                                                    const int32_t* __restrict__ mcnt, int32_t n2, DGraph dst,
                                                    unsigned long long* pb) {
    constexpr int PER = MID_MEM / MID_T;   // members staged per thread
    __shared__ int32_t tk[MID_SLOTS];
    __shared__ long long tv[MID_SLOTS];
    __shared__ int32_t wm[MID_MEM + 1];   // group-relative entry offset of each member
    __shared__ int32_t wo[MID_MEM];       // row offset of each member
    __shared__ int32_t s_cnt;
    __shared__ long long s_deg;
    const bool front = MID_SLOTS < 2 * MID_MAX;   // the list's front holds the groups of at most MID_HALF entries
    const int32_t cnt = mcnt[front ? 0 : 1];
    const int tid = threadIdx.x;
    const int32_t G = (int32_t)gridDim.x;
    auto list_at = [&](int32_t i) -> int32_t { return i < cnt ? mlist[front ? i : n2 - i] : -1; };
    // the members of group m into registers: entry offset and row offset
    auto stage = [&](const MidMeta& m, int32_t* rw, int32_t* ro) {
        int32_t p[PER];
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int32_t k = q * MID_T + tid;
            rw[q] = k < m.mc ? mstart[m.m0 + k] - m.gs : 0;
            p[q] = k < m.mc ? (perm ? perm[m.m0 + k] : m.m0 + k) : 0;
        }
#pragma unroll
        for (int q = 0; q < PER; q++) ro[q] = q * MID_T + tid < m.mc ? src.off[p[q]] : 0;
    };
    int64_t bytes = 0;
    int32_t i = blockIdx.x;
    if (i >= cnt) return;
    for (int k = tid; k < MID_SLOTS; k += MID_T) { tk[k] = -1; tv[k] = 0; }
    MidMeta A = mid_meta(list_at(i), vstart, gstart);
    int32_t aw[PER], ao[PER];
    stage(A, aw, ao);
    MidMeta B = mid_meta(list_at(i + G), vstart, gstart);
    int32_t c_g = list_at(i + 2 * G);
    for (;;) {
        // A's members into LDS (the previous group's readers passed the
        // barrier that ended its sweep)
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int32_t k = q * MID_T + tid;
            if (k < A.mc) { wm[k] = aw[q]; wo[k] = ao[q]; }
        }
        if (tid == 0) { wm[A.mc] = A.s; s_cnt = 0; s_deg = 0; }
        __syncthreads();
        // loads of the groups to come, issued before A's entries so that
        // their latencies overlap
        const MidMeta C = mid_meta(c_g, vstart, gstart);
        const int32_t d_g = list_at(i + 3 * G);
        int32_t bw[PER], bo[PER];
        stage(B, bw, bo);
        const int32_t g = A.g;
        for (int32_t e0 = 0; e0 < A.s; e0 += 4 * MID_T) {
            int32_t x[4], t[4];
            int64_t c[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int32_t e = e0 + q * MID_T + tid;
                x[q] = 0;
                c[q] = 0;
                if (e >= A.s) continue;
                int32_t lo = 0, hi = A.mc;   // the member holding entry e
                while (hi - lo > 1) { const int32_t mid = (lo + hi) >> 1; if (wm[mid] <= e) lo = mid; else hi = mid; }
                x[q] = src.col[wo[lo] + (e - wm[lo])];
                c[q] = src.w[wo[lo] + (e - wm[lo])];
            }
#pragma unroll
            for (int q = 0; q < 4; q++) t[q] = c[q] > 0 ? (L ? L[x[q]] : x[q]) : g;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                if (t[q] == g) continue;   // a loop, zero weight or no entry
                uint32_t h = hash32((uint32_t)t[q]) & (MID_SLOTS - 1);
                for (;;) {
                    const int32_t k = tk[h];
                    if (k == t[q]) break;
                    if (k == -1) {
                        const int32_t old = atomicCAS(&tk[h], -1, t[q]);
                        if (old == -1 || old == t[q]) break;
                    }
                    h = (h + 1) & (MID_SLOTS - 1);
                }
                atomicAdd((unsigned long long*)&tv[h], (unsigned long long)c[q]);
            }
        }
        __syncthreads();
        // sweep: the merged row out, the table cleared for the next group
        for (int k = tid; k < MID_SLOTS; k += MID_T) {
            const int32_t key = tk[k];
            if (key < 0) continue;
            const long long val = tv[k];
            tk[k] = -1;
            tv[k] = 0;
            const int32_t pos = atomicAdd(&s_cnt, 1);
            dst.col[A.gs + pos] = key;
            dst.w[A.gs + pos] = val;
            atomicAdd((unsigned long long*)&s_deg, (unsigned long long)val);
        }
        __syncthreads();
        if (tid == 0) {
            dst.len[g] = s_cnt;
            dst.deg[g] = s_deg;
            // col, w (and the label of each target) in; col, w out; off, len, deg
            bytes += (int64_t)A.s * (L ? 16 : 12) + (int64_t)s_cnt * 12 + 12 * A.mc;
        }
        i += G;
        if (i >= cnt) break;
        A = B;
#pragma unroll
        for (int q = 0; q < PER; q++) { aw[q] = bw[q]; ao[q] = bo[q]; }
        B = C;
        c_g = d_g;
    }
    if (pb) prof_add(pb, bytes);
}

__global__ void k_big_clear(const int32_t* __restrict__ total_p, int32_t* __restrict__ tkey,
                            int64_t* __restrict__ tval) {
    const int64_t total = *total_p;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        tkey[i] = -1;
        tval[i] = 0;
    }
}

// Large groups: their entries form one flattened space (bebase = prefix
// of the entry counts of large groups). A workgroup takes a tile of
// BIG_TILE entries, combines equal (group, target) pairs in an LDS hash, and
// adds each distinct pair once to the group's global table, so a target hit
// by many members costs one global atomic per tile rather than per entry.
constexpr int BIG_TILE = 4096;
constexpr int BIG_HSLOTS = 2 * BIG_TILE;
constexpr int BIG_T = BIG_TILE / 4;      // threads: four entries each per segment pass
constexpr int BIG_WIN = 1024;            // members whose row offsets a segment stages in LDS

// group and first member of every tile's first entry, searched for all
// tiles at once so the searches' latencies overlap
__global__ void k_big_tiles(const int32_t* __restrict__ vstart, const int32_t* __restrict__ mstart,
                            const int32_t* __restrict__ gstart, const int32_t* __restrict__ bebase, int32_t n2,
                            int32_t* __restrict__ tinfo) {
    const int64_t ntiles = ((int64_t)bebase[n2] + BIG_TILE - 1) / BIG_TILE;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = t * BIG_TILE;
        const int32_t g = last_le(bebase, n2, e);
        const int32_t m0 = vstart ? vstart[g] : g;
        const int32_t mc = vstart ? vstart[g + 1] - m0 : 1;
        tinfo[2 * t] = g;
        tinfo[2 * t + 1] = m0 + last_le(mstart + m0, mc, gstart[g] + (int32_t)(e - bebase[g]));
    }
}

__global__ __launch_bounds__(BIG_T) void k_big_insert(DGraph src, const int32_t* __restrict__ L,
                                                   const int32_t* __restrict__ perm,
                                                   const int32_t* __restrict__ vstart,
                                                   const int32_t* __restrict__ mstart,
                                                   const int32_t* __restrict__ gstart,
                                                   const int32_t* __restrict__ bebase,
                                                   const int32_t* __restrict__ tbase, int32_t n2,
                                                   int32_t* __restrict__ tkey, int64_t* __restrict__ tval,
                                                   const int32_t* __restrict__ dslot, int64_t* __restrict__ dense,
                                                   const int32_t* __restrict__ tinfo, DGraph dst,
                                                   unsigned long long* pb) {
    constexpr int PER = BIG_TILE / BIG_T;   // entries per thread and segment pass
    constexpr int FL = BIG_HSLOTS / BIG_T;  // table slots per thread in the flush
    __shared__ unsigned long long hkey[BIG_HSLOTS];
    __shared__ long long hval[BIG_HSLOTS];
    __shared__ int32_t wm[BIG_WIN + 2];      // member-space start of each member in the window
    __shared__ int32_t wo[BIG_WIN + 1];      // row offset of each member in the window
    __shared__ int32_t info[4];              // g, first member, member count in window, g's group end
    const int64_t total = bebase[n2];
    const int64_t ntiles = (total + BIG_TILE - 1) / BIG_TILE;
    int64_t nin = 0;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        for (int i = threadIdx.x; i < BIG_HSLOTS; i += blockDim.x) { hkey[i] = EMPTY_KEY; hval[i] = 0; }
        const int64_t e0 = tile * BIG_TILE;
        const int64_t e1 = e0 + BIG_TILE < total ? e0 + BIG_TILE : total;
        // a tile may straddle groups; handle it one group segment at a time
        int64_t e = e0;
        int32_t gprev = -1;
        while (e < e1) {
            __syncthreads();
            if (threadIdx.x < MC_WAVE) {
                // the tile's first group and member were found beforehand; a
                // later segment starts a large group at its first entry: the
                // next large group after the previous one, looked for by the
                // whole wavefront 64 groups at a time (small groups in
                // between own no entries of this space)
                int32_t g = -1;
                if (e == e0) {
                    g = tinfo[2 * tile];
                } else {
                    int32_t base = gprev + 1;
                    for (int it = 0; it < 8 && g < 0; it++, base += MC_WAVE) {
                        const int32_t gg = base + (int32_t)lane_id();
                        const unsigned long long m = __ballot(gg < n2 && (int64_t)bebase[gg + 1] > e);
                        if (m) g = base + __ffsll((long long)m) - 1;
                    }
                    if (g < 0) g = last_le(bebase, n2, e);
                }
                if (threadIdx.x == 0) {
                    const int32_t m0 = vstart ? vstart[g] : g;
                    const int32_t mc = vstart ? vstart[g + 1] - m0 : 1;
                    const int32_t mf = e == e0 ? tinfo[2 * tile + 1] : m0;
                    info[0] = g;
                    info[1] = mf;
                    info[2] = (m0 + mc) - mf;            // members from mf to the group's end
                    info[3] = bebase[g + 1];
                }
            }
            __syncthreads();
            const int32_t g = info[0], mf = info[1];
            gprev = g;
            const int32_t wc = info[2] < BIG_WIN + 1 ? info[2] : BIG_WIN + 1;
            const int64_t seg_end = (int64_t)info[3] < e1 ? (int64_t)info[3] : e1;
            for (int i = threadIdx.x; i <= wc; i += blockDim.x) {
                wm[i] = mstart[mf + i];
                if (i < wc) wo[i] = src.off[perm ? perm[mf + i] : mf + i];
            }
            __syncthreads();
            const int32_t gbase = gstart[g] - bebase[g];
            // each thread's entries of the segment, their loads issued
            // together: row offset (LDS), entry, label of its target
            int32_t x[PER];
            int64_t c[PER];
#pragma unroll
            for (int q = 0; q < PER; q++) {
                const int64_t f = e + threadIdx.x + q * BIG_T;
                c[q] = 0;
                x[q] = 0;
                if (f >= seg_end) continue;
                nin++;
                const int32_t ge = gbase + (int32_t)f;
                int32_t o, j;
                if (ge < wm[wc]) {
                    int32_t lo = 0, hi = wc;
                    while (hi - lo > 1) { int32_t mid = (lo + hi) >> 1; if (wm[mid] <= ge) lo = mid; else hi = mid; }
                    o = wo[lo];
                    j = ge - wm[lo];
                } else {
                    // rows shorter than one entry cannot occur in a contracted
                    // graph; search HBM if a window is ever too short
                    const int32_t m0 = vstart ? vstart[g] : g;
                    const int32_t mc = vstart ? vstart[g + 1] - m0 : 1;
                    const int32_t k = m0 + last_le(mstart + m0, mc, ge);
                    o = src.off[perm ? perm[k] : k];
                    j = ge - mstart[k];
                }
                x[q] = src.col[o + j];
                c[q] = src.w[o + j];
            }
            int32_t t[PER];
#pragma unroll
            for (int q = 0; q < PER; q++) t[q] = c[q] > 0 ? (L ? L[x[q]] : x[q]) : g;
#pragma unroll
            for (int q = 0; q < PER; q++) {
                if (t[q] == g) continue;   // loop, zero weight or no entry
                const unsigned long long key = ((unsigned long long)(uint32_t)g << 32) | (uint32_t)t[q];
                uint32_t h = hash32((uint32_t)t[q] ^ hash32((uint32_t)g)) & (BIG_HSLOTS - 1);
                for (;;) {
                    unsigned long long kk = hkey[h];
                    if (kk == key) break;
                    if (kk == EMPTY_KEY) {
                        unsigned long long old = atomicCAS(&hkey[h], EMPTY_KEY, key);
                        if (old == EMPTY_KEY || old == key) break;
                    }
                    h = (h + 1) & (BIG_HSLOTS - 1);
                }
                atomicAdd((unsigned long long*)&hval[h], (unsigned long long)c[q]);
            }
            e = seg_end;
        }
        __syncthreads();
        // flush: each thread's table slots go out together; a probe is one
        // compare-and-swap that claims an empty slot or finds the key, and
        // all of a thread's pending probes are in flight at once
        int32_t fg[FL], ft[FL], fb[FL], fs[FL];
        uint32_t fh[FL];
        long long fv[FL];
        bool pend[FL];
#pragma unroll
        for (int q = 0; q < FL; q++) {
            const unsigned long long k = hkey[threadIdx.x + q * BIG_T];
            pend[q] = k != EMPTY_KEY;
            fg[q] = (int32_t)(k >> 32);
            ft[q] = (int32_t)(k & 0xFFFFFFFFu);
            fv[q] = hval[threadIdx.x + q * BIG_T];
        }
#pragma unroll
        for (int q = 0; q < FL; q++) {
            fs[q] = 0;
            fb[q] = 0;
            fh[q] = 0;
            if (!pend[q]) continue;
            const int32_t d = dslot[fg[q]];
            if (d >= 0) {
                atomic_add_i64(&dense[(int64_t)d * n2 + ft[q]], fv[q]);
                pend[q] = false;
                continue;
            }
            fb[q] = tbase[fg[q]];
            fs[q] = tbase[fg[q] + 1] - fb[q];
            fh[q] = (uint32_t)(((uint64_t)hash32((uint32_t)ft[q]) * (uint32_t)fs[q]) >> 32);
        }
        for (;;) {
            bool any = false;
            int32_t old[FL];
#pragma unroll
            for (int q = 0; q < FL; q++)
                if (pend[q]) old[q] = atomicCAS(&tkey[fb[q] + fh[q]], -1, ft[q]);
#pragma unroll
            for (int q = 0; q < FL; q++) {
                if (!pend[q]) continue;
                if (old[q] == -1 || old[q] == ft[q]) {
                    atomic_add_i64(&tval[fb[q] + fh[q]], fv[q]);
                    pend[q] = false;
                } else {
                    if (++fh[q] == (uint32_t)fs[q]) fh[q] = 0;
                    any = true;
                }
            }
            if (!any) break;
        }
        __syncthreads();
    }
    if (pb) prof_add(pb, nin * (L ? 16 : 12));
}

// group of every 256-slot table tile (tables are whole tiles), searched for
// all tiles at once so the searches' latencies overlap
__global__ void k_big_xtiles(const int32_t* __restrict__ tbase, int32_t n2, int32_t* __restrict__ xg) {
    const int64_t ntiles = tbase[n2] / TILE_SLOTS;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += (int64_t)gridDim.x * blockDim.x)
        xg[t] = last_le(tbase, n2, t * TILE_SLOTS);
}

// One wavefront emits the valid slots of a unit of group g (PERL slots per
// lane): a wave prefix sum places them, and one atomic per unit reserves
// their room in the row (one more adds their weight to the degree). The
// callers spread the units of one group over time, since atomics on one
// address serialise.
template <int PERL>
__device__ __forceinline__ void wave_emit(int32_t g, const bool (&take)[PERL], const int32_t (&key)[PERL],
                                          const int64_t (&val)[PERL], int32_t gs, int32_t* __restrict__ bcur,
                                          DGraph& dst) {
    const int lane = lane_id();
    int32_t cnt = 0;
    int64_t sum = 0;
#pragma unroll
    for (int q = 0; q < PERL; q++) { cnt += take[q] ? 1 : 0; sum += take[q] ? val[q] : 0; }
    int32_t incl = cnt;
    for (int d = 1; d < MC_WAVE; d <<= 1) {
        const int32_t y = __shfl_up(incl, d, MC_WAVE);
        if (lane >= d) incl += y;
    }
    const int32_t total = __shfl(incl, MC_WAVE - 1, MC_WAVE);
    if (total == 0) return;
    const int64_t wsum = wave_sum_i64(sum);
    int32_t base = 0;
    if (lane == 0) {
        base = atomicAdd(&bcur[g], total);
        atomic_add_i64(&dst.deg[g], wsum);
    }
    int32_t pos = gs + __shfl(base, 0, MC_WAVE) + incl - cnt;
#pragma unroll
    for (int q = 0; q < PERL; q++) {
        if (!take[q]) continue;
        dst.col[pos] = key[q];
        dst.w[pos] = val[q];
        pos++;
    }
}

constexpr int EX_T = 256;   // threads of the extraction kernels: four waves, one unit each
static_assert(TILE_SLOTS == 4 * MC_WAVE, "a table tile is one wave's unit");

__global__ __launch_bounds__(EX_T) void k_big_extract(const int32_t* __restrict__ tbase,
                                                      const int32_t* __restrict__ gstart, int32_t n2,
                                                      const int32_t* __restrict__ xg,
                                                      const int32_t* __restrict__ tkey,
                                                      const int64_t* __restrict__ tval,
                                                      int32_t* __restrict__ bcur, DGraph dst) {
    const int64_t ntiles = tbase[n2] / TILE_SLOTS;
    const int64_t wid = (int64_t)blockIdx.x * (EX_T / MC_WAVE) + threadIdx.x / MC_WAVE;
    const int64_t nw = (int64_t)gridDim.x * (EX_T / MC_WAVE);
    // tiles in the order u K mod ntiles (a permutation when K and ntiles
    // are coprime), so that waves running together serve different groups
    const int64_t K = ntiles % 1000003 ? 1000003 : 1;
    for (int64_t u = wid; u < ntiles; u += nw) {
        const int64_t t = (u * K) % ntiles;
        const int64_t base = t * TILE_SLOTS + lane_id();
        const int32_t g = xg[t];
        bool take[4];
        int32_t key[4];
        int64_t val[4];
#pragma unroll
        for (int q = 0; q < 4; q++) key[q] = tkey[base + q * MC_WAVE];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            take[q] = key[q] >= 0;
            val[q] = take[q] ? tval[base + q * MC_WAVE] : 0;
        }
        wave_emit<4>(g, take, key, val, gstart[g], bcur, dst);
    }
}

// the dense accumulators the giant groups of this contraction use, zeroed
// once their count is known (no earlier reset needed)
__global__ void k_dense_clear(const int32_t* __restrict__ dinfo, int32_t nd_max, int32_t n2,
                              int64_t* __restrict__ dense) {
    const int32_t nd = dinfo[0] < nd_max ? dinfo[0] : nd_max;
    const int64_t total = (int64_t)nd * n2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
        dense[i] = 0;
}

// dense accumulators of the giant groups: stream over n2 targets and emit
// the non-zero ones
__global__ __launch_bounds__(EX_T) void k_dense_extract(const int32_t* __restrict__ dinfo, int32_t nd_max,
                                                        const int32_t* __restrict__ gstart, int32_t n2,
                                                        const int64_t* __restrict__ dense, int32_t* __restrict__ bcur,
                                                        DGraph dst) {
    constexpr int PERL = 16;                       // a unit is 1024 targets
    constexpr int UNIT = PERL * MC_WAVE;
    const int32_t nd = dinfo[0] < nd_max ? dinfo[0] : nd_max;
    const int64_t per = ((int64_t)n2 + UNIT - 1) / UNIT;   // units per accumulator
    const int64_t wid = (int64_t)blockIdx.x * (EX_T / MC_WAVE) + threadIdx.x / MC_WAVE;
    const int64_t nw = (int64_t)gridDim.x * (EX_T / MC_WAVE);
    // unit u belongs to accumulator u mod nd: waves running together serve
    // different groups
    for (int64_t u = wid; u < (int64_t)nd * per; u += nw) {
        const int32_t d = (int32_t)(u % nd);
        const int32_t t0 = (int32_t)(u / nd) * UNIT + lane_id();
        const int32_t g = dinfo[1 + d];
        const int64_t* acc = dense + (int64_t)d * n2;
        bool take[PERL];
        int32_t key[PERL];
        int64_t val[PERL];
#pragma unroll
        for (int q = 0; q < PERL; q++) {
            key[q] = t0 + q * MC_WAVE;
            val[q] = key[q] < n2 ? acc[key[q]] : 0;
        }
#pragma unroll
        for (int q = 0; q < PERL; q++) take[q] = val[q] != 0;
        wave_emit<PERL>(g, take, key, val, gstart[g], bcur, dst);
    }
}

__global__ void k_big_finalize(const int32_t* __restrict__ bebase, int32_t n2, const int32_t* __restrict__ bcur,
                               DGraph dst) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n2; g += (int64_t)gridDim.x * blockDim.x)
        if (bebase[g + 1] > bebase[g]) dst.len[g] = bcur[g];
}

// minimum degree, ties to the smallest vertex, the entry count and the
// maximum degree: per-block partials, then one block folds them
__global__ __launch_bounds__(256) void k_min_deg_blocks(const int64_t* __restrict__ deg,
                                                       const int32_t* __restrict__ len, int32_t n,
                                                       int64_t* __restrict__ rv, int32_t* __restrict__ ri,
                                                       int64_t* __restrict__ rm, int64_t* __restrict__ rd) {
    __shared__ int64_t sv[4], sm[4], sd[4];
    __shared__ int32_t si[4];
    int64_t best = 0, m = 0, dmax = 0;
    int32_t bid = -1;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int64_t d = deg[v];
        m += len[v];
        dmax = d > dmax ? d : dmax;
        if (bid < 0 || d < best) { best = d; bid = (int32_t)v; }
    }
    wave_argmin(best, bid);
    m = wave_sum_i64(m);
    dmax = wave_max_i64(dmax);
    if (lane_id() == 0) {
        const int wv = threadIdx.x / MC_WAVE;
        sv[wv] = best; si[wv] = bid; sm[wv] = m; sd[wv] = dmax;
    }
    __syncthreads();
    if (threadIdx.x < MC_WAVE) {
        int64_t b = threadIdx.x < 4 ? sv[threadIdx.x] : 0;
        int32_t i = threadIdx.x < 4 ? si[threadIdx.x] : -1;
        wave_argmin(b, i);
        if (threadIdx.x == 0) {
            rv[blockIdx.x] = b; ri[blockIdx.x] = i;
            rm[blockIdx.x] = sm[0] + sm[1] + sm[2] + sm[3];
            const int64_t a = sd[0] > sd[1] ? sd[0] : sd[1], b = sd[2] > sd[3] ? sd[2] : sd[3];
            rd[blockIdx.x] = a > b ? a : b;
        }
    }
}

__global__ __launch_bounds__(64) void k_min_deg_final(const int64_t* __restrict__ rv, const int32_t* __restrict__ ri,
                                                     const int64_t* __restrict__ rm, const int64_t* __restrict__ rd,
                                                     int nblocks, DevScalars* sc) {
    int64_t best = 0, m = 0, dmax = 0;
    int32_t bid = -1;
    for (int i = threadIdx.x; i < nblocks; i += MC_WAVE) {
        int32_t id = ri[i];
        m += rm[i];
        dmax = rd[i] > dmax ? rd[i] : dmax;
        if (id >= 0 && (bid < 0 || rv[i] < best || (rv[i] == best && id < bid))) { best = rv[i]; bid = id; }
    }
    wave_argmin(best, bid);
    m = wave_sum_i64(m);
    dmax = wave_max_i64(dmax);
    if (threadIdx.x == 0) { sc->dmin = best; sc->dmin_arg = bid; sc->m2 = m; sc->dmax = dmax; }
}

inline int grid_for(int64_t count, int threads, int cap = 8192) {
    int64_t b = (count + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

}  // namespace

void contract_ws_carve(Arena& a, int32_t n, int64_t cap, ContractWS& ws, bool sort) {
    ws.sorted = sort;
    if (sort) sort_ws_carve(a, n, cap, ws.sw);
    ws.gcnt = a.take<int32_t>((size_t)n + 2);
    ws.vstart = ws.gcnt;
    ws.gcur = a.take<int32_t>((size_t)n + 1);
    ws.perm = a.take<int32_t>((size_t)n + 1);
    ws.mstart = a.take<int32_t>((size_t)n + 2);
    ws.gstart = a.take<int32_t>((size_t)n + 2);
    ws.tsize = a.take<int32_t>((size_t)n + 2);
    ws.bigm = a.take<int32_t>((size_t)n + 2);
    ws.bcur = a.take<int32_t>((size_t)n + 1);
    // large-group tables: sum over groups of round_up(2 s, 256) with s > 512
    // is at most 2 cap + 256 cap / 513 < 2.5 cap
    size_t slots = (size_t)(cap * 5 / 2) + 4 * TILE_SLOTS;
    ws.tkey = a.take<int32_t>(slots);
    ws.tval = a.take<int64_t>(slots);
    ws.dslot = a.take<int32_t>((size_t)n + 1);
    ws.dinfo = a.take<int32_t>(1 + DENSE_MAX);
    // accumulator budget: the entries' weight array at most, 512 MB at most,
    // and never below four accumulators of n + 1
    const int64_t lim = cap < ((int64_t)1 << 26) ? cap : ((int64_t)1 << 26);
    ws.dense_elems = lim > 4 * ((int64_t)n + 1) ? lim : 4 * ((int64_t)n + 1);
    ws.dense = a.take<int64_t>((size_t)ws.dense_elems);
    ws.scan_tmp = a.take<int32_t>(scan_tmp_elems((int64_t)n + 2) + 16);
    ws.red_val = a.take<int64_t>(1024);
    ws.red_id = a.take<int32_t>(1024);
    ws.red_m = a.take<int64_t>(1024);
    ws.red_d = a.take<int64_t>(1024);
    ws.cg = a.take<int32_t>((size_t)((cap + (int64_t)GROUP_W * n) / CHUNK) + 4);
    ws.tinfo = a.take<int32_t>(2 * ((size_t)(cap / BIG_TILE) + 2));
    ws.xg = a.take<int32_t>(slots / TILE_SLOTS + 8);
    ws.mlist = a.take<int32_t>((size_t)n + 1);
    ws.sstart = a.take<int32_t>((size_t)n + 2);
    ws.mcnt = a.take<int32_t>(4);
}


bool min_degree(const DGraph& g, ContractWS& ws, DevScalars* sc, hipStream_t s) {
    int nb = grid_for(g.n, 256, 1024);
    k_min_deg_blocks<<<nb, 256, 0, s>>>(g.deg, g.len, g.n, ws.red_val, ws.red_id, ws.red_m, ws.red_d);
    MC_LAUNCHED("k_min_deg_blocks");
    k_min_deg_final<<<1, 64, 0, s>>>(ws.red_val, ws.red_id, ws.red_m, ws.red_d, nb, sc);
    MC_LAUNCHED("k_min_deg_final");
    return true;
}

bool contract(const DGraph& src, const int32_t* L, int32_t n2, DGraph& dst, ContractWS& ws, DevScalars* sc,
              hipStream_t s) {
    if (ws.sorted) return contract_sorted(src, L, n2, dst, ws, sc, s);
    const int32_t n = src.n;
    dst.n = n2;
    const int32_t* perm = nullptr;
    const int32_t* vstart = nullptr;
    if (L) {
        if (!fill_i32(ws.gcnt, 0, (int64_t)n2 + 1, s)) return false;
        if (!fill_i32(ws.gcur, 0, n2, s)) return false;
        const int gtiles = grid_for(n, GT, 4096);
        prof_begin(PK_GROUP_COUNT, s);
        k_group_count<<<gtiles, GT_THREADS, 0, s>>>(L, n, ws.gcnt);
        MC_LAUNCHED("k_group_count");
        prof_end(PK_GROUP_COUNT, s);
        prof_host_bytes(PK_GROUP_COUNT, 4.0 * n + 4.0 * n2);   // labels in, counts out
        if (!scan_i32(ws.gcnt, ws.vstart, n2, ws.scan_tmp, s)) return false;
        prof_begin(PK_GROUP_SCATTER, s);
        k_group_scatter<<<gtiles, GT_THREADS, 0, s>>>(L, n, ws.vstart, ws.gcur, ws.perm);
        MC_LAUNCHED("k_group_scatter");
        prof_end(PK_GROUP_SCATTER, s);
        prof_host_bytes(PK_GROUP_SCATTER, 8.0 * n + 4.0 * n2);  // labels in, perm out, group starts in
        perm = ws.perm;
        vstart = ws.vstart;
    }
    k_member_len<<<grid_for(n, 256), 256, 0, s>>>(src.len, perm, n, vstart ? vstart + n2 : nullptr, ws.mstart);
    MC_LAUNCHED("k_member_len");
    if (!scan_i32(ws.mstart, ws.mstart, n, ws.scan_tmp, s)) return false;
    const int32_t* gstart = ws.mstart;
    if (L) {
        k_group_start<<<grid_for((int64_t)n2 + 1, 256), 256, 0, s>>>(vstart, ws.mstart, n2, ws.gstart);
        MC_LAUNCHED("k_group_start");
        gstart = ws.gstart;
    }
    const int64_t ndm = ws.dense_elems / (n2 > 0 ? n2 : 1);
    const int32_t nd_max = (int32_t)(ndm < DENSE_MAX ? ndm : DENSE_MAX);
    if (!fill_i32(ws.dinfo, 0, 1, s) || !fill_i32(ws.mcnt, 0, 2, s)) return false;
    k_classify<<<grid_for(n2, 256), 256, 0, s>>>(gstart, vstart, n2, nd_max, ws.tsize, ws.bigm, ws.bcur, ws.dslot,
                                                 ws.dinfo, ws.mlist, ws.mcnt, ws.sstart, dst);
    MC_LAUNCHED("k_classify");
    if (nd_max > 0) {
        k_dense_clear<<<grid_for((int64_t)nd_max * n2, 256, 4096), 256, 0, s>>>(ws.dinfo, nd_max, n2, ws.dense);
        MC_LAUNCHED("k_dense_clear");
    }
    if (!scan_i32(ws.tsize, ws.tsize, n2, ws.scan_tmp, s)) return false;  // -> tbase
    if (!scan_i32(ws.bigm, ws.bigm, n2, ws.scan_tmp, s)) return false;    // -> bebase
    if (!scan_i32(ws.sstart, ws.sstart, n2, ws.scan_tmp, s)) return false;  // small-group entry prefix
    // at most this many chunks hold small groups; the rest of the grid finds
    // no group and returns
    const int64_t chunks = (src.cap + (int64_t)GROUP_W * n2) / CHUNK + 2;
    k_chunk_start<<<grid_for(chunks + 1, 256), 256, 0, s>>>(ws.sstart, n2, chunks, ws.cg);
    MC_LAUNCHED("k_chunk_start");
    prof_begin(PK_MERGE_SMALL, s);
    k_merge_small<<<(unsigned)chunks, MERGE_THREADS, 0, s>>>(src, L, perm, vstart, gstart, n2, ws.cg, dst,
                                                             prof_dev_bytes(PK_MERGE_SMALL));
    MC_LAUNCHED("k_merge_small");
    prof_end(PK_MERGE_SMALL, s);
    prof_begin(PK_MID_MERGE, s);
    k_mid_merge<2 * MID_HALF><<<256 * 4, MID_T, 0, s>>>(src, L, perm, vstart, ws.mstart, gstart, ws.mlist, ws.mcnt,
                                                        n2, dst, prof_dev_bytes(PK_MID_MERGE));
    MC_LAUNCHED("k_mid_merge");
    k_mid_merge<2 * MID_MAX><<<256 * 2, MID_T, 0, s>>>(src, L, perm, vstart, ws.mstart, gstart, ws.mlist, ws.mcnt,
                                                       n2, dst, prof_dev_bytes(PK_MID_MERGE));
    MC_LAUNCHED("k_mid_merge");
    prof_end(PK_MID_MERGE, s);
    k_big_clear<<<2048, 256, 0, s>>>(ws.tsize + n2, ws.tkey, ws.tval);
    MC_LAUNCHED("k_big_clear");
    k_big_tiles<<<grid_for(src.cap / BIG_TILE + 1, 256), 256, 0, s>>>(vstart, ws.mstart, gstart, ws.bigm, n2,
                                                                      ws.tinfo);
    MC_LAUNCHED("k_big_tiles");
    prof_begin(PK_BIG_INSERT, s);
    k_big_insert<<<4096 * 256 / BIG_T, BIG_T, 0, s>>>(src, L, perm, vstart, ws.mstart, gstart, ws.bigm, ws.tsize, n2, ws.tkey,
                                      ws.tval, ws.dslot, ws.dense, ws.tinfo, dst, prof_dev_bytes(PK_BIG_INSERT));
    MC_LAUNCHED("k_big_insert");
    prof_end(PK_BIG_INSERT, s);
    k_big_xtiles<<<grid_for((src.cap * 5 / 2) / TILE_SLOTS + 8, 256), 256, 0, s>>>(ws.tsize, n2, ws.xg);
    MC_LAUNCHED("k_big_xtiles");
    k_big_extract<<<4096, EX_T, 0, s>>>(ws.tsize, gstart, n2, ws.xg, ws.tkey, ws.tval, ws.bcur, dst);
    MC_LAUNCHED("k_big_extract");
    k_dense_extract<<<grid_for((int64_t)nd_max * n2, 16 * EX_T, 4096), EX_T, 0, s>>>(ws.dinfo, nd_max, gstart, n2, ws.dense,
                                                                              ws.bcur, dst);
    MC_LAUNCHED("k_dense_extract");
    k_big_finalize<<<grid_for(n2, 256), 256, 0, s>>>(ws.bigm, n2, ws.bcur, dst);
    MC_LAUNCHED("k_big_finalize");
    return min_degree(dst, ws, sc, s);
}
