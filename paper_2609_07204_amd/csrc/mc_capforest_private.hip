// CAPFOREST with private passes and capped batches (paper, Section 2.1,
// "Bounded priority queues" and "Parallel CAPFOREST"; Algorithm 1).
//
// Keys are bounded by lam: once r(y) >= lam the key of y is lam, the largest
// key there is, and no later scan can raise another vertex above it. So all
// queued vertices with capped keys may be scanned in any order, one after
// the other; this kernel scans such a set as one batch with a whole
// workgroup. The marks of the batch are the marks of one sequential order:
// for a target y, the batch member whose atomic add moves r(y) across lam
// is the one that would cross it if the members that added to y before it
// had been scanned first. Edges inside a batch only change r of vertices
// already capped, so they are skipped for marks and their weight is taken
// out of alpha (alpha grows by sum(c(x) - 2 r(x)) - 2 w(edges inside)).
// When no key is capped, the single vertex with the largest key (smallest
// id on ties) is scanned.
//
// Passes do not share a visited array (the private mode of the paper's
// parallel session, item 1): a pass's traversal is never cut by another
// pass, which on power-law graphs is what lets vertices reach lam at all.
// Every pass is one workgroup with dense per-pass state in HBM
// (st, r, capped FIFO, touched list, queue list, scan order), which has no
// capacity limit, so hubs are scanned like any other vertex. State is
// cleared through the touched list at the end of the pass.
#include "mc_internal.h"

namespace {

// Threads per pass: a single solve's few passes take 1024 threads each; in
// instance mode (one pass per graph of a batch, most of them small) a pass
// takes 256 by default, so four times as many passes are resident at once
// (64 to 1024 on request).
constexpr int PT_SOLVE = 1024;
constexpr int PT_INST = 256;

enum : int32_t { S_NEW = 0, S_QUEUED = 1, S_SCANNED = 2, S_BATCH = 3 };

constexpr int L2_MAX = 8192;   // level-2 entries (n <= 32 M vertices)
// passes of at most L1_LDS * 64 vertices keep their level-1 index in LDS
// (16 KB), which takes a global round trip off the refresh and the
// selection of every single pop
constexpr int L1_LDS = 2048;
constexpr int DL_LDS = 128;    // dirty blocks whose ids are also kept in LDS

// level-1 entry b of the pass: in LDS (ls) or in HBM (lg)
__device__ __forceinline__ int64_t l1_get(const int64_t* lg, const long long* ls, int32_t b) {
    if (ls) return ls[b];
    return __hip_atomic_load(&lg[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void l1_set(int64_t* lg, long long* ls, int32_t b, int64_t v) {
    if (ls) ls[b] = v;
    else __hip_atomic_store(&lg[b], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void l1_max(int64_t* lg, long long* ls, int32_t b, int64_t v) {
    if (ls) atomicMax(&ls[b], (long long)v);
    else atomicMax((long long*)&lg[b], (long long)v);
}

template <int PT>
struct PassLds {
    static constexpr int PW = PT / MC_WAVE;
    int32_t head, tail, tn, dn, single_x, one_valid;
    int64_t one_part, one_intra;
    int32_t bx[PT];
    int32_t boff[PT + 1];
    int64_t red64[PW];
    int32_t redi[PW];
    int32_t scan32[PW];
    uint32_t l2dirty[L2_MAX / 32];
    int32_t dl[DL_LDS];
};

__device__ __forceinline__ int32_t ld32(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t ld64(const int64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// exclusive scan over the block; every thread gets the total
template <int PT>
__device__ int32_t block_scan(int32_t v, int32_t& total, PassLds<PT>& L) {
    constexpr int PW = PT / MC_WAVE;
    const int lane = lane_id(), wid = threadIdx.x / MC_WAVE;
    int32_t incl = v;
    for (int o = 1; o < MC_WAVE; o <<= 1) {
        int32_t y = __shfl_up(incl, o, MC_WAVE);
        if (lane >= o) incl += y;
    }
    __syncthreads();
    if (lane == MC_WAVE - 1) L.scan32[wid] = incl;
    __syncthreads();
    int32_t pre = 0, tot = 0;
    for (int k = 0; k < PW; k++) {
        int32_t t = L.scan32[k];
        if (k < wid) pre += t;
        tot += t;
    }
    total = tot;
    return pre + incl - v;
}

template <int PT>
__device__ int64_t block_sum(int64_t v, PassLds<PT>& L) {
    constexpr int PW = PT / MC_WAVE;
    v = wave_sum_i64(v);
    __syncthreads();
    if (lane_id() == 0) L.red64[threadIdx.x / MC_WAVE] = v;
    __syncthreads();
    int64_t t = 0;
    for (int k = 0; k < PW; k++) t += L.red64[k];
    return t;
}

// (key desc, id asc) maximum over the block; id < 0 means empty
template <int PT>
__device__ void block_argmax(int64_t& key, int32_t& id, PassLds<PT>& L) {
    constexpr int PW = PT / MC_WAVE;
    int32_t aux = 0;
    wave_argmax(key, id, aux);
    __syncthreads();
    if (lane_id() == 0) { L.red64[threadIdx.x / MC_WAVE] = key; L.redi[threadIdx.x / MC_WAVE] = id; }
    __syncthreads();
    key = -1;
    id = -1;
    for (int k = 0; k < PW; k++) {
        int32_t i2 = L.redi[k];
        int64_t k2 = L.red64[k];
        if (i2 >= 0 && (id < 0 || k2 > key || (k2 == key && i2 < id))) { key = k2; id = i2; }
    }
}

__device__ __forceinline__ int32_t last_le_lds(const int32_t* a, int32_t n, int32_t key) {
    int32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        int32_t mid = (lo + hi) >> 1;
        if (a[mid] <= key) lo = mid; else hi = mid;
    }
    return lo;
}

template <int PT>
__device__ __forceinline__ void mark_dirty(uint32_t* dbits, int32_t* dlist, int32_t b, PassLds<PT>& L) {
    const uint32_t bit = 1u << (b & 31);
    if (!(atomicOr(&dbits[b >> 5], bit) & bit)) {
        const int32_t k = atomicAdd(&L.dn, 1);
        dlist[k] = b;
        if (k < DL_LDS) L.dl[k] = b;   // the refresh reads these from LDS
    }
}

// Per-pass priority index over the queued vertices outside the capped FIFO:
// l1[b] bounds the largest r over block b (64 consecutive ids) from above,
// l2[g] (LDS) the largest l1 over group g (64 blocks). Raising r below lam
// raises l1/l2 by atomic max; a vertex that leaves this set (capped into the
// FIFO, or scanned) marks its block dirty, and dirty blocks are recomputed
// right before the next single pop, which is then exact: largest r, then
// smallest block and id.
template <int PT>
__global__ __launch_bounds__(PT) void k_capforest_private(PrivateArgs a) {
    constexpr int PW = PT / MC_WAVE;
    extern __shared__ long long l2[];
    __shared__ PassLds<PT> L;
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / MC_WAVE;
    const int p = blockIdx.x;
    // the pass's vertices are [base, base + n); st and r are indexed by
    // vertex id, the per-pass lists and the index by position in the range
    int32_t base = 0, n = a.g.n;
    int32_t *st, *fifo, *tl, *order, *dlist;
    int64_t *r, *l1;
    uint32_t* dbits;
    if (a.pvoff) {
        base = a.pvoff[p];
        n = a.pvoff[p + 1] - base;
        if (n < 3 || (a.prun && !a.prun[p])) {
            if (tid == 0) {
                a.nscan[p] = 0;
                a.alpha[p] = INT64_MAX;
                a.alpha_len[p] = 0;
                a.lam_out[p] = a.plam[p];
                if (a.steps) a.steps[p] = 0;
                if (a.pmarks) a.pmarks[p] = 0;
            }
            return;
        }
        st = a.st;
        r = a.r;
        fifo = a.fifo + base;
        tl = a.touched + base;
        order = a.order + base;
        l1 = a.l1 + (base >> 6) + p;
        dlist = a.dlist + (base >> 6) + p;
        dbits = a.dbits + (base >> 11) + 2 * p;
    } else {
        st = a.st + (int64_t)p * a.stride;
        r = a.r + (int64_t)p * a.stride;
        fifo = a.fifo + (int64_t)p * a.stride;
        tl = a.touched + (int64_t)p * a.stride;
        order = a.order + (int64_t)p * a.stride;
        l1 = a.l1 + (int64_t)p * a.stride1;
        dlist = a.dlist + (int64_t)p * a.stride1;
        dbits = a.dbits + (int64_t)p * (a.stride1 / 32 + 1);
    }
    const int32_t nb1 = (n + 63) / 64;
    const int32_t nb2 = (nb1 + 63) / 64;
    long long* l1s = a.l1_at > 0 ? l2 + a.l1_at : nullptr;   // uniform

    for (int32_t b = tid; b < nb1; b += PT) l1_set(l1, l1s, b, -1);
    for (int32_t b = tid; b <= nb1 / 32; b += PT) dbits[b] = 0;
    for (int32_t g = tid; g < nb2; g += PT) l2[g] = -1;
    for (int32_t g = tid; g < L2_MAX / 32; g += PT) L.l2dirty[g] = 0;
    int64_t lam = a.plam ? a.plam[p] : *a.lam;
    if (tid == 0) {
        int32_t s = a.start;
        if (s < 0) {
            uint64_t h = splitmix64(a.seed ^ splitmix64(((uint64_t)(uint32_t)a.round << 32) | (uint32_t)p));
            s = base + (int32_t)(((h >> 32) * (uint64_t)n) >> 32);
        }
        st[s] = S_QUEUED;
        tl[0] = s;
        L.head = 0;
        L.tail = 0;
        L.tn = 1;
        L.dn = 0;
        L.single_x = s;
    }
    __threadfence_block();
    __syncthreads();

    int64_t alpha = 0, best_alpha = INT64_MAX;
    int32_t best_len = 0, nscan = 0, steps = 0;
    unsigned long long marks = 0;
    bool first = true;
    int64_t d_single = 0, d_pop_clk = 0, d_batch_clk = 0, d_entries = 0, d_maxb = 0;

    for (;;) {
        __syncthreads();
        if (a.len_cap > 0 && nscan >= a.len_cap) break;
        const int64_t t_pop0 = wall_clock64();
        const int32_t head = L.head, tail = L.tail;
        int32_t B;
        const int32_t* src = nullptr;
        bool from_lds = false;
        if (head < tail) {
            // capped vertices may be scanned in any order, so a batch cut at
            // the pass's remaining budget is a prefix of a valid pass
            B = tail - head;
            if (a.len_cap > 0 && B > a.len_cap - nscan) B = a.len_cap - nscan;
            src = fifo + head;
        } else if (first) {
            B = 1;
            from_lds = true;
            first = false;
        } else {
            // refresh dirty blocks (one wavefront per block)
            const int32_t dn = L.dn;
            for (int32_t i = wid; i < dn; i += PW) {
                const int32_t b = i < DL_LDS ? L.dl[i] : dlist[i];
                const int32_t lv = b * 64 + lane;
                // every queued vertex counts: one whose r reached a lowered
                // bound has the largest key and must stay findable
                int64_t val = -1;
                if (lv < n && ld32(&st[base + lv]) == S_QUEUED) val = ld64(&r[base + lv]);
                for (int o = 32; o > 0; o >>= 1) { int64_t t = __shfl_xor(val, o, MC_WAVE); val = t > val ? t : val; }
                if (lane == 0) {
                    l1_set(l1, l1s, b, val);
                    atomicAnd(&dbits[b >> 5], ~(1u << (b & 31)));
                    atomicOr(&L.l2dirty[b >> 11], 1u << ((b >> 6) & 31));
                }
            }
            __threadfence_block();
            __syncthreads();
            // refresh dirty groups of level 2
            for (int32_t g = wid; g < nb2; g += PW) {
                if (!(L.l2dirty[g >> 5] & (1u << (g & 31)))) continue;
                const int32_t b = g * 64 + lane;
                int64_t val = b < nb1 ? l1_get(l1, l1s, b) : -1;
                for (int o = 32; o > 0; o >>= 1) { int64_t t = __shfl_xor(val, o, MC_WAVE); val = t > val ? t : val; }
                if (lane == 0) l2[g] = val;
            }
            __syncthreads();
            for (int32_t g = tid; g < L2_MAX / 32; g += PT) L.l2dirty[g] = 0;
            if (tid == 0) L.dn = 0;
            // exact pop through the two levels
            int64_t bk = -1;
            int32_t bg = -1;
            for (int32_t g = tid; g < nb2; g += PT) {
                const int64_t v = l2[g];
                if (v >= 0 && (bg < 0 || v > bk)) { bk = v; bg = g; }
            }
            block_argmax(bk, bg, L);
            if (bg < 0) break;          // queue empty (uniform)
            if (wid == 0) {
                const int32_t b = bg * 64 + lane;
                int64_t v1 = b < nb1 ? l1_get(l1, l1s, b) : -1;
                int32_t bb = v1 >= 0 ? b : -1;
                int32_t aux = 0;
                wave_argmax(v1, bb, aux);
                int32_t x = -1;
                int64_t rx = -1;
                if (bb >= 0) {
                    const int32_t lv = bb * 64 + lane;
                    if (lv < n && ld32(&st[base + lv]) == S_QUEUED) { rx = ld64(&r[base + lv]); x = base + lv; }
                }
                wave_argmax(rx, x, aux);
                if (lane == 0) L.single_x = x;
            }
            __syncthreads();
            if (L.single_x < 0) break;  // index and state disagree: stop the pass
            B = 1;
            from_lds = true;
            d_single++;
        }
        // a single pop has passed a barrier since head and tail were read
        if (!from_lds) __syncthreads();
        if (tid == 0 && !from_lds) L.head = head + B;
        steps++;
        const int64_t t_b0 = wall_clock64();
        d_pop_clk += t_b0 - t_pop0;
        d_maxb = B > d_maxb ? B : d_maxb;
        for (int32_t c0 = 0; c0 < B; c0 += PT) {
            const int32_t cnt = (B - c0) < PT ? (B - c0) : PT;
            if (cnt == 1) {
                // one vertex (a single pop, or a batch of one): thread 0 sets
                // it up, with two barriers in place of the scans and sums a
                // batch needs; most pops of a sparse, lightly weighted graph
                // take this path
                int32_t x1 = -1;
                if (tid == 0) {
                    x1 = from_lds ? L.single_x : src[c0];
                    // the vertex's state, length, degree and r in one round trip
                    const int32_t s1 = ld32(&st[x1]);
                    int32_t e1 = a.g.len[x1];
                    int64_t p1 = a.g.deg[x1] - 2 * ld64(&r[x1]);
                    if (s1 == S_QUEUED) {
                        st[x1] = S_BATCH;
                        order[nscan] = x1;
                        mark_dirty(dbits, dlist, (x1 - base) >> 6, L);
                    } else {
                        x1 = -1;
                        e1 = 0;
                        p1 = 0;
                    }
                    L.bx[0] = x1 < 0 ? 0 : x1;
                    L.boff[0] = 0;
                    L.boff[1] = e1;
                    L.one_valid = x1 >= 0 ? 1 : 0;
                    L.one_part = p1;
                    L.one_intra = 0;
                }
                __syncthreads();
                __threadfence_block();
                const int32_t E = L.boff[1];
                const int32_t xs = L.bx[0];
                int64_t intra = 0;
                if (E > 0) {
                    const int32_t o = a.g.off[xs];
                    for (int32_t j = tid; j < E; j += PT) {
                        const int32_t y = a.g.col[o + j];
                        const int64_t c = a.g.w[o + j];
                        const int32_t sy = ld32(&st[y]);
                        if (sy == S_BATCH) { intra += c; continue; }
                        if (sy == S_SCANNED) continue;
                        if (sy == S_NEW) {
                            if (atomicCAS(&st[y], S_NEW, S_QUEUED) == S_NEW) tl[atomicAdd(&L.tn, 1)] = y;
                        }
                        const int64_t old = atomic_add_i64(&r[y], c);
                        const int64_t nw = old + c;
                        if (old < lam && lam <= nw) {
                            if (uf_union(a.parent, xs, y)) marks++;
                            fifo[atomicAdd(&L.tail, 1)] = y;
                            mark_dirty(dbits, dlist, (y - base) >> 6, L);
                        } else if (nw < lam) {
                            l1_max(l1, l1s, (y - base) >> 6, nw);
                            atomicMax(&l2[(y - base) >> 12], (long long)nw);
                        }
                    }
                }
                if (intra) atomicAdd((unsigned long long*)&L.one_intra, (unsigned long long)intra);
                d_entries += E;
                __syncthreads();
                if (x1 >= 0) st[x1] = S_SCANNED;
                __threadfence_block();
                const int32_t nvalid = L.one_valid;
                nscan += nvalid;
                alpha += L.one_part - L.one_intra;
                if (nscan < n) {
                    if (alpha < best_alpha) { best_alpha = alpha; best_len = nscan; }
                    if (alpha < lam) lam = alpha;
                }
                continue;
            }
            int32_t dl = 0;
            int64_t part = 0;
            int32_t x = -1;
            if (tid < cnt) {
                x = from_lds ? L.single_x : src[c0 + tid];
                // every entry is queued by construction; anything else is
                // left out rather than scanned twice
                if (ld32(&st[x]) != S_QUEUED) x = -1;
            }
            int32_t nvalid;
            const int32_t opos = block_scan(x >= 0 ? 1 : 0, nvalid, L);
            if (tid < cnt) {
                L.bx[tid] = x < 0 ? 0 : x;
                if (x >= 0) {
                    st[x] = S_BATCH;
                    dl = a.g.len[x];
                    part = a.g.deg[x] - 2 * ld64(&r[x]);
                    order[nscan + opos] = x;
                    mark_dirty(dbits, dlist, (x - base) >> 6, L);
                }
            }
            int32_t E;
            const int32_t eo = block_scan(dl, E, L);
            if (tid < cnt) L.boff[tid] = eo;
            if (tid == 0) L.boff[cnt] = E;
            const int64_t P = block_sum(part, L);
            __syncthreads();
            __threadfence_block();
            int64_t intra = 0;
            for (int32_t e = tid; e < E; e += PT) {
                const int32_t k = last_le_lds(L.boff, cnt, e);
                const int32_t xs = L.bx[k];
                const int32_t j = e - L.boff[k];
                const int32_t o = a.g.off[xs];
                const int32_t y = a.g.col[o + j];
                const int64_t c = a.g.w[o + j];
                const int32_t sy = ld32(&st[y]);
                if (sy == S_BATCH) { intra += c; continue; }
                if (sy == S_SCANNED) continue;
                if (sy == S_NEW) {
                    if (atomicCAS(&st[y], S_NEW, S_QUEUED) == S_NEW) tl[atomicAdd(&L.tn, 1)] = y;
                }
                const int64_t old = atomic_add_i64(&r[y], c);
                const int64_t nw = old + c;
                if (old < lam && lam <= nw) {
                    if (uf_union(a.parent, xs, y)) marks++;
                    fifo[atomicAdd(&L.tail, 1)] = y;
                    mark_dirty(dbits, dlist, (y - base) >> 6, L);
                } else if (nw < lam) {
                    l1_max(l1, l1s, (y - base) >> 6, nw);
                    atomicMax(&l2[(y - base) >> 12], (long long)nw);
                }
            }
            const int64_t I = block_sum(intra, L);
            d_entries += E;
            __syncthreads();
            if (x >= 0) st[x] = S_SCANNED;
            __threadfence_block();
            nscan += nvalid;
            alpha += P - I;
            if (nscan < n) {
                if (alpha < best_alpha) { best_alpha = alpha; best_len = nscan; }
                if (alpha < lam) lam = alpha;
            }
        }
        d_batch_clk += wall_clock64() - t_b0;
    }
    __syncthreads();
    if (a.diag && tid == 0) {
        int64_t* d = a.diag + (int64_t)p * 8;
        d[0] = steps; d[1] = d_single; d[2] = L.tn; d[3] = d_entries;
        d[4] = d_pop_clk; d[5] = d_batch_clk; d[6] = nscan; d[7] = d_maxb;
    }
    // leave st and r all-zero for the next launch
    const int32_t tn = L.tn;
    for (int32_t i = tid; i < tn; i += PT) {
        const int32_t v = tl[i];
        st[v] = S_NEW;
        r[v] = 0;
    }
    marks = (unsigned long long)wave_sum_i64((int64_t)marks);
    if (lane == 0 && marks) atomicAdd(a.marks, marks);
    if (a.pmarks) {
        __shared__ unsigned long long s_marks;
        if (tid == 0) s_marks = 0;
        __syncthreads();
        if (lane == 0 && marks) atomicAdd(&s_marks, marks);
        __syncthreads();
        if (tid == 0) a.pmarks[p] = s_marks;
    }
    if (tid == 0) {
        a.nscan[p] = nscan;
        a.alpha[p] = best_alpha;
        a.alpha_len[p] = best_len;
        a.lam_out[p] = lam;
        if (a.steps) a.steps[p] = steps;
    }
}

__global__ void k_private_reset(int32_t* st, int64_t* r, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        st[i] = 0;
        r[i] = 0;
    }
}

}  // namespace

static bool launch_private(const PrivateArgs& a, int32_t threads, size_t lds, hipStream_t s) {
    switch (threads) {
        case 64: k_capforest_private<64><<<a.passes, 64, lds, s>>>(a); break;
        case 128: k_capforest_private<128><<<a.passes, 128, lds, s>>>(a); break;
        case 256: k_capforest_private<256><<<a.passes, 256, lds, s>>>(a); break;
        case 512: k_capforest_private<512><<<a.passes, 512, lds, s>>>(a); break;
        case 1024: k_capforest_private<1024><<<a.passes, 1024, lds, s>>>(a); break;
        default:
            mc_hip_ok(hipErrorInvalidValue, "capforest_private: unsupported pass workgroup size");
            return false;
    }
    MC_LAUNCHED("k_capforest_private");
    return true;
}

bool capforest_private(const PrivateArgs& a, hipStream_t s, int32_t max_pass_n) {
    if (a.passes <= 0) return true;
    if (a.pvoff) {
        // instance mode: the index of the largest range sets the LDS size
        const int32_t nb2 = ((max_pass_n + 63) / 64 + 63) / 64;
        if (nb2 > L2_MAX) {
            mc_hip_ok(hipErrorInvalidValue, "capforest_private: instance too large for the pass index");
            return false;
        }
        const int32_t nb1 = (max_pass_n + 63) / 64;
        PrivateArgs b = a;
        b.l1_at = nb1 <= L1_LDS ? (nb2 > 0 ? nb2 : 1) : 0;
        const size_t lds = (size_t)((nb2 > 0 ? nb2 : 1) + (b.l1_at ? nb1 : 0)) * sizeof(long long);
        return launch_private(b, a.threads > 0 ? a.threads : PT_INST, lds, s);
    }
    if (a.g.n > a.stride) {
        mc_hip_ok(hipErrorInvalidValue, "capforest_private: per-pass stride smaller than n");
        return false;
    }
    const int32_t nb2 = ((a.g.n + 63) / 64 + 63) / 64;
    if (nb2 > L2_MAX || (int64_t)a.g.n / 64 + 1 > a.stride1) {
        mc_hip_ok(hipErrorInvalidValue, "capforest_private: graph too large for the pass index");
        return false;
    }
    const int32_t nb1 = (a.g.n + 63) / 64;
    PrivateArgs b = a;
    b.l1_at = nb1 <= L1_LDS ? nb2 : 0;
    return launch_private(b, a.threads > 0 ? a.threads : PT_SOLVE, (size_t)(nb2 + (b.l1_at ? nb1 : 0)) * sizeof(long long), s);
}

bool capforest_private_reset(const PrivateArgs& a, hipStream_t s) {
    const int64_t count = a.region > 0 ? a.region : (int64_t)a.passes * a.stride;
    k_private_reset<<<4096, 256, 0, s>>>(a.st, a.r, count);
    MC_LAUNCHED("k_private_reset");
    return true;
}
