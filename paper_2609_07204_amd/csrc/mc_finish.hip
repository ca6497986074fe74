// Device-resident exact rounds for small graphs (paper, Algorithm 2; the
// regime of Section 4 where rounds contract little, which needs the round
// loop on the device) with CAPFOREST passes whose priority queue lives in
// LDS (Section 2.1 "Bounded priority queues").
//
// One workgroup takes one graph of at most FIN_N vertices and runs every
// remaining round of Algorithm 2 in one launch, with no host round trip:
//  - a complete CAPFOREST pass (Algorithm 1, one pass, private state) run by
//    one wavefront: one vertex is popped at a time and its row is scanned by
//    the 64 lanes together; scanning x adds c(x) - 2 r(x) to alpha, which
//    lowers lambda-hat while the scanned set is a proper subset; an edge to
//    an unscanned y whose r(y) crosses lambda-hat is marked (union-find in
//    LDS);
//  - canonical relabelling of the marked components and contraction: the
//    groups are merged by four wavefronts, each with a dense accumulator over
//    the new vertices in LDS, into the other of two scratch buffers;
//  - the collapsed degrees bound lambda-hat (Section 2.1 "Overall
//    algorithm"),
// until at most two vertices remain. The queue holds the keys min(r, lam),
// integers in [0, lam]:
//  - buckets (lam < FQB): one bucket per attainable key, each a LIFO list of
//    nodes in an LDS pool; a key increase pushes a new node and leaves the
//    old one behind (it is skipped when popped), so pushes from many lanes
//    need only LDS atomics; a full pool is rebuilt from the queued vertices;
//  - binary heap (otherwise): ordered by (key, smallest id), updated by
//    lane 0 after each row chunk; when lam drops the keys change and the
//    heap is rebuilt. This order is exactly the sequential pass's (largest
//    key, then smallest id), so a heap pass is bit-exact against it.
// The graph's rows stay in global memory (the input graph's window, then
// two scratch buffers); everything per vertex is in LDS.
#include "mc_internal.h"

namespace {

constexpr int FT = 1024;                 // threads of a finisher workgroup
constexpr int FMW = 4;                   // wavefronts that merge groups
constexpr int FQB = 2048;                // bucket heads: buckets while lam < FQB
constexpr int FPOOL = 2048;              // bucket nodes before a rebuild

enum : uint8_t { F_NEW = 0, F_QUEUED = 1, F_SCANNED = 2 };

struct FinLds {
    int32_t off[FIN_N], len[FIN_N];      // rows of the current graph (positions in its buffer)
    int64_t deg[FIN_N];
    int64_t r[FIN_N];
    int32_t parent[FIN_N];
    int32_t vstart[FIN_N + 1];
    int32_t gstart[FIN_N + 1];
    int32_t bhead[FQB];
    int32_t pool_nx[FPOOL];
    int16_t pool_v[FPOOL];
    int16_t order[FIN_N];
    int16_t heap[FIN_N], hpos[FIN_N];
    int16_t fmap[FIN_N];                 // entry vertex -> current vertex
    int16_t lab[FIN_N];                  // canonical labels of the round
    int16_t perm[FIN_N];                 // current vertices grouped by label
    uint8_t st[FIN_N];
    uint8_t bestf[FIN_N];                // side over the entry vertices of the best cut found here
    int64_t acc[FMW][FIN_N];
    int16_t tch[FMW][FIN_N];
    int32_t ntch[FMW];
    int64_t red64[FT / MC_WAVE];
    int32_t red32[FT / MC_WAVE];
    int32_t gnext;
    int32_t n2;
};

// ------------------------------------------------------------ union-find
__device__ __forceinline__ int32_t lf_find(int32_t* par, int32_t x) {
    int32_t p = __hip_atomic_load(&par[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    while (p != x) {
        const int32_t gp = __hip_atomic_load(&par[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (gp == p) return p;
        __hip_atomic_store(&par[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        x = p;
        p = gp;
    }
    return x;
}
// smaller root wins, so roots are the smallest vertex of their component
__device__ __forceinline__ bool lf_union(int32_t* par, int32_t a, int32_t b) {
    int32_t ra = lf_find(par, a), rb = lf_find(par, b);
    while (ra != rb) {
        if (ra > rb) { const int32_t t = ra; ra = rb; rb = t; }
        const int32_t old = atomicCAS(&par[rb], rb, ra);
        if (old == rb) return true;
        rb = lf_find(par, old);
        ra = lf_find(par, ra);
    }
    return false;
}

// ------------------------------------------------------------ heap queue
// max-heap on (min(r, lam), smallest id); single-threaded (lane 0)
__device__ __forceinline__ bool h_before(const FinLds& S, int32_t a, int32_t b, int64_t lam) {
    const int64_t ka = S.r[a] < lam ? S.r[a] : lam, kb = S.r[b] < lam ? S.r[b] : lam;
    return ka > kb || (ka == kb && a < b);
}
__device__ void h_up(FinLds& S, int32_t i, int64_t lam) {
    const int32_t v = S.heap[i];
    while (i > 0) {
        const int32_t p = (i - 1) >> 1;
        const int32_t u = S.heap[p];
        if (!h_before(S, v, u, lam)) break;
        S.heap[i] = (int16_t)u;
        S.hpos[u] = (int16_t)i;
        i = p;
    }
    S.heap[i] = (int16_t)v;
    S.hpos[v] = (int16_t)i;
}
__device__ void h_down(FinLds& S, int32_t i, int32_t hn, int64_t lam) {
    const int32_t v = S.heap[i];
    for (;;) {
        int32_t c = 2 * i + 1;
        if (c >= hn) break;
        if (c + 1 < hn && h_before(S, S.heap[c + 1], S.heap[c], lam)) c++;
        const int32_t u = S.heap[c];
        if (!h_before(S, u, v, lam)) break;
        S.heap[i] = (int16_t)u;
        S.hpos[u] = (int16_t)i;
        i = c;
    }
    S.heap[i] = (int16_t)v;
    S.hpos[v] = (int16_t)i;
}

// ------------------------------------------------------------ bucket queue
__device__ __forceinline__ void b_push(FinLds& S, int32_t* pool_n, int32_t* maxk, int32_t v, int32_t k,
                                       bool* overflow) {
    const int32_t node = atomicAdd(pool_n, 1);
    if (node >= FPOOL) { *overflow = true; return; }
    S.pool_v[node] = (int16_t)v;
    S.pool_nx[node] = atomicExch(&S.bhead[k], node);
    atomicMax(maxk, k);
}

// One complete CAPFOREST pass over the current graph (n vertices, rows in
// col/w at S.off/S.len, target t of an entry is col - cbase) by wavefront 0,
// from start.
// Marks go to S.parent. Returns (uniform over the wave) the bound after the
// pass in lam, the smallest proper-prefix alpha and its length, the scanned
// count and the marks.
struct PassOut {
    int64_t lam, best_alpha;
    int32_t best_len, nscan;
    int32_t marks;
};

__device__ PassOut fin_pass(FinLds& S, int32_t n, const int32_t* __restrict__ col, const int64_t* __restrict__ w,
                            int32_t cbase, int32_t start, int64_t lam, bool heap_mode, int32_t* scal) {
    // scal: [0] pool count, [1] max bucket, [2] overflow flag (LDS scalars)
    const int lane = lane_id();
    for (int32_t v = lane; v < n; v += MC_WAVE) { S.st[v] = F_NEW; S.r[v] = 0; }
    if (!heap_mode)
        for (int32_t k = lane; k < FQB; k += MC_WAVE) S.bhead[k] = -1;
    wave_sync();
    int32_t hn = 0;                 // heap size (lane 0's copy is the one used)
    if (lane == 0) {
        S.st[start] = F_QUEUED;
        if (heap_mode) {
            S.heap[0] = (int16_t)start;
            S.hpos[start] = 0;
            hn = 1;
        } else {
            scal[0] = 0;
            scal[1] = 0;
            scal[2] = 0;
            bool of = false;
            b_push(S, &scal[0], &scal[1], start, 0, &of);
        }
    }
    wave_sync();
    PassOut o;
    o.lam = lam;
    o.best_alpha = -1;
    o.best_len = 0;
    o.nscan = 0;
    o.marks = 0;
    int64_t alpha = 0;
    int32_t marks = 0;
    for (;;) {
        // ---- pop (lane 0), broadcast
        int32_t x = -1;
        if (lane == 0) {
            if (heap_mode) {
                if (hn > 0) {
                    x = S.heap[0];
                    hn--;
                    if (hn > 0) {
                        S.heap[0] = S.heap[hn];
                        S.hpos[S.heap[0]] = 0;
                        h_down(S, 0, hn, lam);
                    }
                }
            } else {
                // highest non-empty bucket; nodes left behind by key
                // increases (or scans) are skipped; buckets at or above lam
                // all hold the largest key
                int32_t k = scal[1];
                for (;;) {
                    if (k < 0) break;
                    const int32_t node = S.bhead[k];
                    if (node < 0) { k--; continue; }
                    S.bhead[k] = S.pool_nx[node];
                    const int32_t y = S.pool_v[node];
                    if (S.st[y] != F_QUEUED) continue;
                    const int64_t ky = S.r[y] < lam ? S.r[y] : lam;
                    const int64_t kb = (int64_t)k < lam ? (int64_t)k : lam;
                    if (ky != kb) continue;      // a node of an older, smaller key
                    x = y;
                    break;
                }
                scal[1] = k < 0 ? 0 : k;
            }
            if (x >= 0) {
                S.st[x] = F_SCANNED;
                S.order[o.nscan] = (int16_t)x;
            }
        }
        x = __shfl(x, 0, MC_WAVE);
        wave_sync();
        if (x < 0) break;
        // ---- alpha and the bound (every lane keeps the same copy)
        const int64_t rx = S.r[x];
        o.nscan++;
        alpha += S.deg[x] - 2 * rx;
        const int64_t lam_before = lam;
        if (o.nscan < n) {
            if (o.best_alpha < 0 || alpha < o.best_alpha) { o.best_alpha = alpha; o.best_len = o.nscan; }
            if (alpha < lam) lam = alpha;
        }
        if (heap_mode && lam < lam_before && lane == 0 && hn > 1) {
            // keys min(r, lam) changed: heapify again
            for (int32_t i = hn / 2 - 1; i >= 0; i--) h_down(S, i, hn, lam);
        }
        wave_sync();
        // ---- scan x's row, 64 entries at a time
        const int32_t ox = S.off[x], lx = S.len[x];
        for (int32_t j0 = 0; j0 < lx; j0 += MC_WAVE) {
            const int32_t j = j0 + lane;
            int32_t y = -1;
            bool fresh = false, raise = false;
            int32_t newkey = 0;
            int64_t nw = 0;
            if (j < lx) {
                y = col[ox + j] - cbase;
                const int64_t c = w[ox + j];
                const uint8_t sy = S.st[y];
                if (sy == F_SCANNED) {
                    y = -1;
                } else {
                    const int64_t old = S.r[y];
                    nw = old + c;
                    if (old < lam && lam <= nw && lf_union(S.parent, x, y)) marks++;
                    const int64_t kold = old < lam ? old : lam, knew = nw < lam ? nw : lam;
                    fresh = sy == F_NEW;
                    raise = !fresh && knew > kold;
                    newkey = (int32_t)(knew < (int64_t)(FQB - 1) ? knew : (int64_t)(FQB - 1));
                    // targets of one row are distinct; in the heap, a key
                    // that changes is written together with its sift-up
                    if (!heap_mode || !(fresh || raise)) S.r[y] = nw;
                    if (fresh) S.st[y] = F_QUEUED;
                }
            }
            wave_sync();
            if (!heap_mode) {
                if (fresh || raise) {
                    bool of = false;
                    b_push(S, &scal[0], &scal[1], y, newkey, &of);
                    if (of) scal[2] = 1;
                }
                wave_sync();
                if (scal[2]) {
                    // pool full: rebuild the buckets from the queued vertices
                    for (int32_t k = lane; k < FQB; k += MC_WAVE) S.bhead[k] = -1;
                    if (lane == 0) { scal[0] = 0; scal[1] = 0; scal[2] = 0; }
                    wave_sync();
                    for (int32_t v = lane; v < n; v += MC_WAVE) {
                        if (S.st[v] != F_QUEUED) continue;
                        const int64_t kv = S.r[v] < lam ? S.r[v] : lam;
                        bool of = false;
                        b_push(S, &scal[0], &scal[1], v, (int32_t)kv, &of);
                    }
                    wave_sync();
                }
            } else {
                // lane 0 applies the chunk's key changes one at a time, each
                // r update followed by its sift-up, so the heap is valid
                // after every step (raising several keys first and sifting
                // afterwards can leave a raised child below a smaller key)
                const unsigned long long m = __ballot(fresh || raise);
                unsigned long long mm = m;
                while (mm) {
                    const int k = __ffsll((long long)mm) - 1;
                    mm &= mm - 1;
                    const int32_t yk = __shfl(y, k, MC_WAVE);
                    const bool fk = __shfl(fresh ? 1 : 0, k, MC_WAVE) != 0;
                    const int64_t nk = __shfl(nw, k, MC_WAVE);
                    if (lane == 0) {
                        S.r[yk] = nk;
                        if (fk) {
                            S.heap[hn] = (int16_t)yk;
                            S.hpos[yk] = (int16_t)hn;
                            hn++;
                            h_up(S, hn - 1, lam);
                        } else {
                            h_up(S, S.hpos[yk], lam);
                        }
                    }
                }
                wave_sync();
            }
        }
    }
    // marks summed over the wave
    for (int d = 32; d > 0; d >>= 1) marks += __shfl_xor(marks, d, MC_WAVE);
    o.lam = lam;
    o.marks = marks;
    return o;
}

template <int NT>
__device__ int32_t block_sum_i32(int32_t v, int32_t* red) {
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, MC_WAVE);
    __syncthreads();
    if (lane_id() == 0) red[threadIdx.x / MC_WAVE] = v;
    __syncthreads();
    int32_t t = 0;
    for (int k = 0; k < NT / MC_WAVE; k++) t += red[k];
    return t;
}

// exclusive scan of a[0..n) into out[0..n] (out[n] = total), whole block;
// a and out may alias. n <= FIN_N.
__device__ void block_scan_lds(const int32_t* a, int32_t* out, int32_t n, FinLds& S) {
    constexpr int PER = FIN_N / FT > 0 ? FIN_N / FT : 1;
    int32_t loc[PER];
    int32_t sum = 0;
    const int32_t b0 = threadIdx.x * PER;
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int32_t i = b0 + q;
        loc[q] = i < n ? a[i] : 0;
        sum += loc[q];
    }
    // inclusive scan of the per-thread sums over the block
    int32_t incl = sum;
    for (int d = 1; d < MC_WAVE; d <<= 1) {
        const int32_t t = __shfl_up(incl, d, MC_WAVE);
        if (lane_id() >= d) incl += t;
    }
    __syncthreads();
    if (lane_id() == MC_WAVE - 1) S.red32[threadIdx.x / MC_WAVE] = incl;
    __syncthreads();
    int32_t pre = 0, tot = 0;
    for (int k = 0; k < FT / MC_WAVE; k++) {
        const int32_t t = S.red32[k];
        if (k < (int)(threadIdx.x / MC_WAVE)) pre += t;
        tot += t;
    }
    int32_t run = pre + incl - sum;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int32_t i = b0 + q;
        if (i < n) out[i] = run;
        run += loc[q];
    }
    if (threadIdx.x == 0) out[n] = tot;
    __syncthreads();
}

}  // namespace

// All remaining rounds of graph k by one workgroup (see the file comment).
static __device__ __forceinline__ void finish_one(const FinishArgs& a, int32_t k, FinLds& S, int32_t* scal, int64_t* sc64) {
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / MC_WAVE;
    const int32_t vb = a.gvoff ? a.gvoff[k] : 0;
    const int32_t n0 = a.gvoff ? a.gvoff[k + 1] - vb : a.g.n;
    int64_t lam = a.lam_in[k];
    if (n0 > FIN_N) {
        if (tid == 0) atomicCAS(a.err, 0, 1);
        return;
    }
    // entry graph: rows of vertices vb.. in g; its entries start at ebase
    const int32_t ebase = a.xwindow && n0 > 0 ? a.g.off[vb] : 0;
    for (int32_t v = tid; v < n0; v += FT) {
        S.off[v] = a.g.off[vb + v];
        S.len[v] = a.g.len[vb + v];
        S.deg[v] = a.g.deg[vb + v];
        S.fmap[v] = (int16_t)v;
        S.bestf[v] = 0;
    }
    __syncthreads();
    const int32_t* col = a.g.col;
    const int64_t* w = a.g.w;
    int32_t cbase = vb;                 // targets in g are ids of the union graph
    int32_t buf = 0;                    // scratch buffer the next contraction writes
    int32_t n = n0;
    bool dropped = false;
    int32_t rounds = 0, err = 0;
    // every round marks an edge or lowers the bound
    const int32_t max_rounds = 4 * n0 + 16;
    while (n > 2 && lam > 0) {
        if (rounds >= max_rounds) { err = 2; break; }
        for (int32_t v = tid; v < n; v += FT) S.parent[v] = v;
        __syncthreads();
        // ---- one complete CAPFOREST pass (wavefront 0)
        const uint64_t h = splitmix64(a.seed ^ splitmix64(((uint64_t)(uint32_t)rounds << 32) ^ (uint64_t)(uint32_t)k));
        const int32_t start = (int32_t)(((h >> 32) * (uint64_t)n) >> 32);
        // buckets need one bucket per attainable key, so a bound of FQB or
        // more always takes the heap
        const bool heap_mode = a.qmode == 2 || lam >= FQB;
        const int64_t lam_prev = lam;
        if (wid == 0) {
            const PassOut po = fin_pass(S, n, col, w, cbase, start, lam, heap_mode, scal);
            if (lane == 0) {
                sc64[0] = po.lam;
                scal[4] = po.best_len;
            }
        }
        __syncthreads();
        const int64_t lam_pass = sc64[0];
        const int32_t best_len = scal[4];
        rounds++;
        if (lam_pass < lam_prev) {
            // the best proper prefix of the pass is the new side
            for (int32_t v = tid; v < n; v += FT) S.lab[v] = 0;
            __syncthreads();
            for (int32_t i = tid; i < best_len; i += FT) S.lab[S.order[i]] = 1;
            __syncthreads();
            for (int32_t u = tid; u < n0; u += FT) S.bestf[u] = (uint8_t)S.lab[S.fmap[u]];
            lam = lam_pass;
            dropped = true;
        }
        // ---- canonical labels of the marked components (roots are the
        // smallest vertex of their component)
        for (int32_t v = tid; v < n; v += FT) {
            int32_t r0 = S.parent[v];
            while (S.parent[r0] != r0) r0 = S.parent[r0];
            S.vstart[v] = r0 == v ? 1 : 0;
            S.gstart[v] = r0;
        }
        __syncthreads();
        block_scan_lds(S.vstart, S.vstart, n, S);
        const int32_t n2 = S.vstart[n];
        for (int32_t v = tid; v < n; v += FT) S.lab[v] = (int16_t)S.vstart[S.gstart[v]];
        __syncthreads();
        if (n2 == n) {
            if (lam < lam_prev) continue;   // the pass lowered the bound instead: pass again
            err = 3;                        // a complete pass at a fixed bound marks an edge
            break;
        }
        // ---- group the vertices by label (counting sort in LDS); output
        // windows from the members' row lengths
        for (int32_t g = tid; g <= n2; g += FT) { S.vstart[g] = 0; S.gstart[g] = 0; }
        __syncthreads();
        for (int32_t v = tid; v < n; v += FT) {
            const int32_t g = S.lab[v];
            atomicAdd(&S.vstart[g], 1);
            atomicAdd(&S.gstart[g], S.len[v]);
        }
        __syncthreads();
        block_scan_lds(S.vstart, S.vstart, n2, S);
        block_scan_lds(S.gstart, S.gstart, n2, S);
        for (int32_t g = tid; g < n2; g += FT) S.parent[g] = S.vstart[g];   // fill cursors
        __syncthreads();
        for (int32_t v = tid; v < n; v += FT) S.perm[atomicAdd(&S.parent[S.lab[v]], 1)] = (int16_t)v;
        for (int32_t i = tid; i < FMW * n2; i += FT) S.acc[i / n2][i % n2] = 0;
        if (tid == 0) S.gnext = 0;
        __syncthreads();
        // ---- merge: FMW wavefronts take groups in turn; each sums its
        // group's entries by new target in its dense accumulator
        int32_t* ocol = a.xcol[buf];
        int64_t* ow = a.xw[buf];
        if (wid < FMW) {
            int64_t* acc = S.acc[wid];
            int16_t* tch = S.tch[wid];
            for (;;) {
                int32_t g = 0;
                if (lane == 0) {
                    g = atomicAdd(&S.gnext, 1);
                    S.ntch[wid] = 0;
                }
                g = __shfl(g, 0, MC_WAVE);
                wave_sync();
                if (g >= n2) break;
                for (int32_t m = S.vstart[g]; m < S.vstart[g + 1]; m++) {
                    const int32_t v = S.perm[m];
                    const int32_t ov = S.off[v], lv = S.len[v];
                    for (int32_t j = lane; j < lv; j += MC_WAVE) {
                        const int32_t t = S.lab[col[ov + j] - cbase];
                        if (t == g) continue;    // inside the group
                        const int64_t c = w[ov + j];
                        const unsigned long long old = atomicAdd((unsigned long long*)&acc[t], (unsigned long long)c);
                        if (old == 0) tch[atomicAdd(&S.ntch[wid], 1)] = (int16_t)t;
                    }
                    wave_sync();
                }
                const int32_t nt = S.ntch[wid];
                const int32_t gs = ebase + S.gstart[g];
                int64_t dsum = 0;
                for (int32_t i = lane; i < nt; i += MC_WAVE) {
                    const int32_t t = tch[i];
                    const int64_t c = acc[t];
                    acc[t] = 0;
                    ocol[gs + i] = t;
                    ow[gs + i] = c;
                    dsum += c;
                }
                dsum = wave_sum_i64(dsum);
                wave_sync();
                if (lane == 0) {
                    // the new row: start, length, degree (r[] is free until
                    // the next pass); only this wavefront touches group g
                    S.parent[g] = gs;
                    S.gstart[g] = nt;
                    S.r[g] = dsum;
                }
                wave_sync();
            }
        }
        __syncthreads();
        for (int32_t g = tid; g < n2; g += FT) {
            S.off[g] = S.parent[g];
            S.len[g] = S.gstart[g];
            S.deg[g] = S.r[g];
        }
        for (int32_t u = tid; u < n0; u += FT) S.fmap[u] = S.lab[S.fmap[u]];
        __syncthreads();
        col = ocol;
        w = ow;
        cbase = 0;
        buf ^= 1;
        n = n2;
        // ---- collapsed degrees bound lambda while two or more vertices remain
        if (n >= 2) {
            int64_t best = INT64_MAX;
            int32_t bid = -1;
            for (int32_t v = tid; v < n; v += FT)
                if (bid < 0 || S.deg[v] < best) { best = S.deg[v]; bid = v; }
            wave_argmin(best, bid);
            __syncthreads();
            if (lane == 0) { S.red64[wid] = best; S.red32[wid] = bid; }
            __syncthreads();
            best = INT64_MAX;
            bid = -1;
            for (int q = 0; q < FT / MC_WAVE; q++) {
                const int32_t i2 = S.red32[q];
                const int64_t v2 = S.red64[q];
                if (i2 >= 0 && (bid < 0 || v2 < best || (v2 == best && i2 < bid))) { best = v2; bid = i2; }
            }
            if (best < lam) {
                for (int32_t u = tid; u < n0; u += FT) S.bestf[u] = S.fmap[u] == bid ? 1 : 0;
                lam = best;
                dropped = true;
            }
            __syncthreads();
        }
    }
    // results
    if (tid == 0) {
        a.lam_out[k] = lam;
        a.dropped[k] = dropped ? 1 : 0;
        if (a.rounds) a.rounds[k] = rounds;
        if (err) atomicCAS(a.err, 0, err);
    }
    if (dropped)
        for (int32_t u = tid; u < n0; u += FT) a.fside[vb + u] = S.bestf[u];
}

// One persistent launch over a work queue: each workgroup takes the next
// graph of the list (an atomic ticket) until the list is used up, so a
// launch of as many workgroups as fit the device serves any number of
// graphs, and a workgroup that drew small graphs takes more of them.
__global__ __launch_bounds__(FT) void k_finish(FinishArgs a, int32_t count) {
    __shared__ FinLds S;
    __shared__ int32_t scal[8];
    __shared__ int64_t sc64[4];
    __shared__ int32_t ticket;
    for (;;) {
        if (threadIdx.x == 0) ticket = atomicAdd(a.qnext, 1);
        __syncthreads();
        const int32_t i = ticket;
        __syncthreads();
        if (i >= count) break;
        finish_one(a, a.glist ? a.glist[i] : i, S, scal, sc64);
        __syncthreads();
    }
}

// One pass of the finisher's CAPFOREST on its own (parity and measurement):
// graph g (n <= FIN_N, rows at off/len, local targets), from `start` at
// bound lam, with the queue of qmode (1 buckets, 2 heap). Writes the marks
// as a union-find forest to parent[n] (roots smallest), the scan order and
// its length, the bound after the pass (lam_io), the smallest proper-prefix
// alpha (INT64_MAX if none) and its prefix length.
__global__ __launch_bounds__(FT) void k_fin_pass(DGraph g, int32_t start, int32_t qmode, int64_t* lam_io,
                                                int64_t* best_alpha, int32_t* parent, int32_t* order,
                                                int32_t* nscan_out, int32_t* best_len) {
    __shared__ FinLds S;
    __shared__ int32_t scal[8];
    const int32_t n = g.n;
    const int tid = threadIdx.x;
    for (int32_t v = tid; v < n; v += FT) {
        S.off[v] = g.off[v];
        S.len[v] = g.len[v];
        S.deg[v] = g.deg[v];
        S.parent[v] = v;
    }
    __syncthreads();
    if (tid < MC_WAVE) {
        const PassOut po = fin_pass(S, n, g.col, g.w, 0, start, lam_io[0], qmode == 2 || lam_io[0] >= FQB, scal);
        if (tid == 0) {
            lam_io[0] = po.lam;
            best_alpha[0] = po.best_alpha < 0 ? INT64_MAX : po.best_alpha;
            nscan_out[0] = po.nscan;
            best_len[0] = po.best_len;
            scal[6] = po.nscan;
        }
    }
    __syncthreads();
    const int32_t nscan = scal[6];
    for (int32_t v = tid; v < n; v += FT) {
        parent[v] = S.parent[v];
        order[v] = v < nscan ? S.order[v] : -1;
    }
}

bool finish_graphs(const FinishArgs& a, int32_t count, int32_t cus, hipStream_t s) {
    if (count <= 0) return true;
    // one workgroup per compute unit at most (the LDS holds one)
    const int32_t grid = count < cus ? count : cus;
    k_finish<<<grid, FT, 0, s>>>(a, count);
    MC_LAUNCHED("k_finish");
    return true;
}

bool finish_pass(const DGraph& g, int32_t start, int32_t qmode, int64_t* lam_io, int64_t* best_alpha,
                 int32_t* parent, int32_t* order, int32_t* nscan, int32_t* best_len, hipStream_t s) {
    if (g.n > FIN_N) return false;
    k_fin_pass<<<1, FT, 0, s>>>(g, start, qmode, lam_io, best_alpha, parent, order, nscan, best_len);
    MC_LAUNCHED("k_fin_pass");
    return true;
}
