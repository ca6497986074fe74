// CAPFOREST with private passes, run level-synchronously over the whole GPU
// (paper, Section 2.1 and Algorithm 1; same pass semantics as
// mc_capforest_private.hip, where each pass is one workgroup).
//
// Every pass advances in steps. A step scans one batch per pass: all
// queued vertices with capped keys (cut at the pass's remaining budget), or,
// when there are none, the single queued vertex with the largest key. The
// work of a step is split into launches so that all compute units work on
// the edges of all passes at once:
//   k_cfs_popscan all workgroups: for passes with no capped vertex queued,
//                the largest key over the pass's vertex words, in parts;
//   k_cfs_plan   one workgroup per pass: pick the batch (capped FIFO slice,
//                or the single vertex the parts agree on), mark it, prefix
//                of the batch's row lengths, sum of c(x) - 2 r(x);
//   k_cfs_tiles  one workgroup: cut every pass's entries into 1024-entry
//                tiles, and count the passes still running;
//   k_cfs_edges  all workgroups, one tile at a time: one 64-bit atomic add
//                per entry raises r and reports the target's state; marks
//                and the capped FIFO follow from it;
//   k_cfs_hubfix targets of high degree (hubs) are not updated entry by
//                entry: atomics on one address serialise, and a hub can
//                receive thousands of entries in one step. Their entries
//                go to HUB_SLOTS partial sums per hub instead, together
//                with the heaviest entry; this launch folds them into r;
//   k_cfs_finish one workgroup per pass: batch becomes scanned, alpha and
//                the bound are updated.
// Within a batch the entries may be applied in any order (all batch
// vertices are scanned together), so a hub's step total may be applied at
// once: if it lifts r from below lam to at least lam, the heaviest entry of
// the step is one that crosses lam in some order of the entries (put the
// others first until the remaining gap is at most its weight, which no
// other entry exceeds), and its edge is contracted as Algorithm 1 does.
// The host issues steps and reads the running-pass count every few steps.
#include <algorithm>

#include <vector>

#include "mc_internal.h"

namespace {

constexpr int T = 1024;           // threads of the per-pass kernels
constexpr int TW = T / MC_WAVE;
constexpr int ETILE = 1024;       // entries per edge tile
constexpr int ET = 256;           // threads of the edge kernel

// Per-pass vertex word: r in the low 62 bits (every r is below the total
// weight, < 2^62), the state in the top two: 00 new (r = 0) or queued
// (r > 0), 11 in the current batch, 10 scanned. One 64-bit atomic add per
// entry then both raises r and reports the state it found.
constexpr unsigned long long SCAN_BIT = 1ULL << 63;
constexpr unsigned long long BATCH_BIT = 1ULL << 62;
constexpr unsigned long long R_MASK = BATCH_BIT - 1;

__device__ __forceinline__ bool is_queued(unsigned long long wv) { return (wv >> 62) == 0 && (wv & R_MASK) > 0; }

__device__ __forceinline__ unsigned long long ldw(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct Red {
    int64_t v64[TW];
    int32_t v32[TW];
    int32_t s32[TW];
};

__device__ int32_t bscan(int32_t v, int32_t& total, Red& R) {
    const int lane = lane_id(), wid = threadIdx.x / MC_WAVE;
    int32_t incl = v;
    for (int o = 1; o < MC_WAVE; o <<= 1) {
        int32_t y = __shfl_up(incl, o, MC_WAVE);
        if (lane >= o) incl += y;
    }
    __syncthreads();
    if (lane == MC_WAVE - 1) R.s32[wid] = incl;
    __syncthreads();
    int32_t pre = 0, tot = 0;
    for (int k = 0; k < TW; k++) { int32_t t = R.s32[k]; if (k < wid) pre += t; tot += t; }
    total = tot;
    return pre + incl - v;
}

__device__ int64_t bsum(int64_t v, Red& R) {
    v = wave_sum_i64(v);
    __syncthreads();
    if (lane_id() == 0) R.v64[threadIdx.x / MC_WAVE] = v;
    __syncthreads();
    int64_t t = 0;
    for (int k = 0; k < TW; k++) t += R.v64[k];
    return t;
}

__device__ void bargmax(int64_t& key, int32_t& id, Red& R) {
    int32_t aux = 0;
    wave_argmax(key, id, aux);
    __syncthreads();
    if (lane_id() == 0) { R.v64[threadIdx.x / MC_WAVE] = key; R.v32[threadIdx.x / MC_WAVE] = id; }
    __syncthreads();
    key = -1;
    id = -1;
    for (int k = 0; k < TW; k++) {
        const int32_t i2 = R.v32[k];
        const int64_t k2 = R.v64[k];
        if (i2 >= 0 && (id < 0 || k2 > key || (k2 == key && i2 < id))) { key = k2; id = i2; }
    }
}

struct PassView {
    int32_t *fifo, *tl, *order, *bpre, *single;
    unsigned long long* rw;
    unsigned long long* hacc;   // [max_hubs * HUB_SLOTS * 2] (sum, heaviest entry)
    StepCtl* ctl;
};

// heaviest entry key: weight (saturated at 2^31 - 1) above the source vertex
constexpr unsigned long long HUB_WSAT = 0x7FFFFFFFULL;
__device__ __forceinline__ unsigned long long hub_key(int64_t c, int32_t x) {
    const unsigned long long cw = (unsigned long long)c < HUB_WSAT ? (unsigned long long)c : HUB_WSAT;
    return (cw << 32) | (uint32_t)x;
}

__device__ __forceinline__ PassView view(const StepArgs& a, int p) {
    const PrivateArgs& v = a.pv;
    PassView w;
    w.rw = reinterpret_cast<unsigned long long*>(v.r + (int64_t)p * v.stride);
    w.fifo = v.fifo + (int64_t)p * v.stride;
    w.tl = v.touched + (int64_t)p * v.stride;
    w.order = v.order + (int64_t)p * v.stride;
    w.bpre = a.bpre + (int64_t)p * (a.bcap + 1);
    w.single = a.single + p;
    w.ctl = a.ctl + p;
    w.hacc = a.hacc + (size_t)p * a.max_hubs * HUB_SLOTS * 2;
    return w;
}

// hub index of every vertex with at least HUB_LEN entries (else -1); the
// hub's partial sums start at zero
__global__ __launch_bounds__(256) void k_cfs_hubs(StepArgs a) {
    const int32_t n = a.pv.g.n;
    const int64_t top = ((int64_t)n + MC_WAVE - 1) / MC_WAVE * MC_WAVE;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < top; v += (int64_t)gridDim.x * blockDim.x) {
        const bool hub = v < n && a.pv.g.len[v] >= HUB_LEN;
        const unsigned long long m = __ballot(hub);
        int32_t base = 0;
        const int lead = m ? __ffsll((long long)m) - 1 : 0;
        if (m && lane_id() == lead) base = atomicAdd(a.nhub, __popcll(m));
        base = __shfl(base, lead, MC_WAVE);
        if (v < n) {
            int32_t h = -1;
            if (hub) {
                h = base + __popcll(m & ((1ULL << lane_id()) - 1));
                if (h >= a.max_hubs) h = -1;   // cannot happen: max_hubs >= entries / HUB_LEN
                else {
                    a.hv[h] = (int32_t)v;
                    for (int32_t p = 0; p < a.pv.passes; p++) {
                        unsigned long long* hs = a.hacc + ((size_t)p * a.max_hubs + h) * HUB_SLOTS * 2;
                        for (int k = 0; k < 2 * HUB_SLOTS; k++) hs[k] = 0;
                    }
                }
            }
            a.hid[v] = h;
        }
    }
}

__global__ __launch_bounds__(T) void k_cfs_init(StepArgs a) {
    const int p = blockIdx.x;
    PassView w = view(a, p);
    const int32_t n = a.pv.g.n;
    if (threadIdx.x == 0) {
        int32_t s = a.pv.start;
        if (s < 0) {
            uint64_t h = splitmix64(a.pv.seed ^ splitmix64(((uint64_t)(uint32_t)a.pv.round << 32) | (uint32_t)p));
            s = (int32_t)(((h >> 32) * (uint64_t)n) >> 32);
        }
        StepCtl c{};
        c.lam = *a.pv.lam;
        c.best_alpha = INT64_MAX;
        c.single_pending = 1;
        *w.single = s;
        *w.ctl = c;
    }
    if (threadIdx.x < SPREAD) {
        unsigned long long* sp = a.spread + ((size_t)p * SPREAD + threadIdx.x) * SPREAD_STRIDE;
        sp[0] = 0;
        sp[1] = 0;
    }
}

constexpr int POP_BLOCKS = 512;
constexpr int POP_T = 256;

__device__ __forceinline__ bool wants_pop(const StepCtl& c, int32_t cap) {
    return !c.done && !c.single_pending && c.head >= c.tail && !(cap > 0 && c.nscan >= cap);
}

// largest (r, smallest id) over the queued vertices of every pass that will
// need a single pop; one partial per workgroup and pass
__global__ __launch_bounds__(POP_T) void k_cfs_popscan(StepArgs a) {
    __shared__ int64_t sk[POP_T / MC_WAVE];
    __shared__ int32_t si[POP_T / MC_WAVE];
    const int32_t n = a.pv.g.n;
    for (int32_t p = 0; p < a.pv.passes; p++) {
        const StepCtl& c = a.ctl[p];
        if (!wants_pop(c, a.pv.len_cap)) continue;   // uniform per launch
        const unsigned long long* rw = reinterpret_cast<const unsigned long long*>(a.pv.r + (int64_t)p * a.pv.stride);
        int64_t bk = -1;
        int32_t bv = -1;
        for (int64_t v = (int64_t)blockIdx.x * POP_T + threadIdx.x; v < n; v += (int64_t)gridDim.x * POP_T) {
            const unsigned long long wv = rw[v];
            if (is_queued(wv)) {
                const int64_t r = (int64_t)(wv & R_MASK);
                if (bv < 0 || r > bk) { bk = r; bv = (int32_t)v; }
            }
        }
        int32_t aux = 0;
        wave_argmax(bk, bv, aux);
        __syncthreads();
        if (lane_id() == 0) { sk[threadIdx.x / MC_WAVE] = bk; si[threadIdx.x / MC_WAVE] = bv; }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int k = 1; k < POP_T / MC_WAVE; k++)
                if (si[k] >= 0 && (bv < 0 || sk[k] > bk || (sk[k] == bk && si[k] < bv))) { bk = sk[k]; bv = si[k]; }
            a.popk[(int64_t)p * POP_BLOCKS + blockIdx.x] = bk;
            a.popv[(int64_t)p * POP_BLOCKS + blockIdx.x] = bv;
        }
    }
}

// pick the batch of every running pass
__global__ __launch_bounds__(T) void k_cfs_plan(StepArgs a) {
    __shared__ Red R;
    __shared__ int32_t s_x;
    const int p = blockIdx.x, tid = threadIdx.x;
    PassView w = view(a, p);
    StepCtl& c = *w.ctl;
    const int32_t cap = a.pv.len_cap;
    if (c.done) return;                          // uniform: read by every thread
    if (cap > 0 && c.nscan >= cap) {
        __syncthreads();
        if (tid == 0) { c.done = 1; c.bcount = 0; c.E = 0; }
        return;
    }
    int32_t B = 0;
    bool single = false;
    if (c.single_pending) {
        single = true;
        B = 1;
    } else if (c.head < c.tail) {
        // capped vertices may be scanned in any order, so a batch cut at
        // the pass's remaining budget is a prefix of a valid pass
        B = c.tail - c.head;
        if (cap > 0 && B > cap - c.nscan) B = cap - c.nscan;
        if (B > a.bcap) B = a.bcap;
    } else {
        // the largest key, from the parts of k_cfs_popscan. A truncated pass
        // stops here, at a valid prefix, after max_singles single pops in a
        // row (each costs a whole-GPU step); single pops up to there are
        // what lets a weighted graph's pass reach its first capped vertices
        const int32_t streak = c.streak;
        if (a.max_singles > 0 && streak >= a.max_singles) {
            __syncthreads();
            if (tid == 0) { c.done = 1; c.bcount = 0; c.E = 0; }
            return;
        }
        int64_t bk = -1;
        int32_t bv = -1;
        for (int32_t i = tid; i < POP_BLOCKS; i += T) {
            const int64_t k2 = a.popk[(int64_t)p * POP_BLOCKS + i];
            const int32_t v2 = a.popv[(int64_t)p * POP_BLOCKS + i];
            if (v2 >= 0 && (bv < 0 || k2 > bk || (k2 == bk && v2 < bv))) { bk = k2; bv = v2; }
        }
        bargmax(bk, bv, R);
        if (tid == 0) s_x = bv;
        __syncthreads();
        if (s_x < 0) {
            if (tid == 0) { c.done = 1; c.bcount = 0; c.E = 0; }
            return;
        }
        if (tid == 0) { *w.single = s_x; c.singles++; c.streak++; }
        single = true;
        B = 1;
    }
    __syncthreads();
    if (tid == 0 && !single) c.streak = 0;
    // mark the batch, prefix of row lengths, sum of c(x) - 2 r(x)
    const int32_t* src = single ? w.single : w.fifo + c.head;
    int32_t run = 0;
    int64_t part = 0;
    for (int32_t c0 = 0; c0 < B; c0 += T) {
        const int32_t i = c0 + tid;
        int32_t dl = 0;
        if (i < B) {
            const int32_t x = src[i];
            // every batch entry is queued (or the start vertex) by
            // construction; anything else gets an empty range
            const unsigned long long wv = ldw(&w.rw[x]);
            if ((wv >> 62) == 0) {
                atomicOr(&w.rw[x], SCAN_BIT | BATCH_BIT);
                dl = a.pv.g.len[x];
                part += a.pv.g.deg[x] - 2 * (int64_t)(wv & R_MASK);
            }
        }
        int32_t tot;
        const int32_t ex = bscan(dl, tot, R);
        if (i < B) w.bpre[i] = run + ex;
        run += tot;
    }
    part = bsum(part, R);
    if (tid == 0) {
        w.bpre[B] = run;
        c.bcount = B;
        c.bsingle = single ? 1 : 0;
        c.E = run;
        c.entries += run;
        if (B > c.maxbatch) c.maxbatch = B;
        c.part = part;
        c.intra = 0;
        if (!single) c.head += B;
        c.single_pending = 0;
    }
}

// tiles of every pass's batch entries
__global__ __launch_bounds__(T) void k_cfs_tiles(StepArgs a) {
    __shared__ Red R;
    const int32_t P = a.pv.passes;
    int32_t run = 0, active = 0;
    for (int32_t c0 = 0; c0 < P; c0 += T) {
        const int32_t p = c0 + threadIdx.x;
        int32_t nt = 0;
        if (p < P) {
            const StepCtl& c = a.ctl[p];
            if (!c.done) { nt = (c.E + ETILE - 1) / ETILE; active++; }
        }
        int32_t tot;
        const int32_t ex = bscan(nt, tot, R);
        if (p < P) a.ptile[p] = run + ex;
        run += tot;
    }
    active = (int32_t)bsum(active, R);
    if (threadIdx.x == 0) {
        a.ptile[P] = run;
        *a.running = active;
    }
}

__device__ __forceinline__ int32_t last_le(const int32_t* x, int32_t n, int32_t key) {
    int32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (x[mid] <= key) lo = mid; else hi = mid;
    }
    return lo;
}

static_assert(SPREAD == MC_WAVE, "k_cfs_finish folds one spread slot per lane");

// pass and first batch vertex of every edge tile, searched for all tiles
// at once so the searches' latencies overlap
__global__ __launch_bounds__(256) void k_cfs_tileinfo(StepArgs a) {
    const int32_t P = a.pv.passes;
    const int32_t ntiles = a.ptile[P];
    for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += gridDim.x * blockDim.x) {
        const int32_t p = last_le(a.ptile, P, t);
        const int32_t e0 = (t - a.ptile[p]) * ETILE;
        const int32_t* bpre = a.bpre + (int64_t)p * (a.bcap + 1);
        a.tinfo[2 * (int64_t)t] = p;
        a.tinfo[2 * (int64_t)t + 1] = last_le(bpre, a.ctl[p].bcount, e0);
    }
}

// process the entries of all batches, one 1024-entry tile per workgroup
// pass. Newly capped targets are staged in LDS and appended to the pass's
// FIFO with one counter atomic per tile.
__global__ __launch_bounds__(ET) void k_cfs_edges(StepArgs a) {
    __shared__ int32_t win[ETILE + 2];
    __shared__ int32_t s_cross[ETILE];
    __shared__ int32_t s_nc, s_base;
    __shared__ long long s_intra[ET / MC_WAVE];
    __shared__ unsigned long long s_marks[ET / MC_WAVE];
    const int32_t P = a.pv.passes;
    const int32_t ntiles = a.ptile[P];
    const unsigned hslot = (blockIdx.x * (ET / MC_WAVE) + threadIdx.x / MC_WAVE) % HUB_SLOTS;
    for (int32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int32_t p = a.tinfo[2 * (int64_t)t], k0 = a.tinfo[2 * (int64_t)t + 1];
        const int32_t e0 = (t - a.ptile[p]) * ETILE;
        PassView w = view(a, p);
        const StepCtl& c = *w.ctl;
        const int32_t rest = c.bcount - k0;      // batch vertices from k0 on
        const int32_t wc = rest < ETILE + 1 ? rest : ETILE + 1;
        __syncthreads();
        for (int i = threadIdx.x; i <= wc; i += ET) win[i] = w.bpre[k0 + i];
        if (threadIdx.x == 0) s_nc = 0;
        __syncthreads();
        const int32_t e1 = e0 + ETILE < c.E ? e0 + ETILE : c.E;
        const int64_t lam = c.lam;
        const int32_t* src = c.bsingle ? w.single : w.fifo + (c.head - c.bcount);
        int64_t intra = 0;
        unsigned long long marks = 0;
        for (int32_t e = e0 + (int32_t)threadIdx.x; e < e1; e += ET) {
            int32_t k, j;
            if (e < win[wc]) {
                int32_t lo = 0, hi = wc;
                while (hi - lo > 1) { const int32_t mid = (lo + hi) >> 1; if (win[mid] <= e) lo = mid; else hi = mid; }
                k = k0 + lo;
                j = e - win[lo];
            } else {
                k = last_le(w.bpre, c.bcount, e);
                j = e - w.bpre[k];
            }
            const int32_t xs = src[k];
            const int32_t o = a.pv.g.off[xs];
            const int32_t y = a.pv.g.col[o + j];
            const int64_t cw = a.pv.g.w[o + j];
            const int32_t h = a.hid[y];
            if (h >= 0) {
                // hub: its state bits do not change during this launch
                const unsigned long long sv = ldw(&w.rw[y]);
                if (sv & SCAN_BIT) {
                    if (sv & BATCH_BIT) intra += cw;
                } else {
                    unsigned long long* hs = w.hacc + ((size_t)h * HUB_SLOTS + hslot) * 2;
                    atomicAdd(&hs[0], (unsigned long long)cw);
                    atomicMax(&hs[1], hub_key(cw, xs));
                }
            } else {
                const unsigned long long ow = atomicAdd(&w.rw[y], (unsigned long long)cw);
                if (ow & SCAN_BIT) {
                    if (ow & BATCH_BIT) intra += cw;
                } else {
                    const int64_t old = (int64_t)(ow & R_MASK);
                    if (old < lam && lam <= old + cw) {
                        if (uf_union(a.pv.parent, xs, y)) marks++;
                        s_cross[atomicAdd(&s_nc, 1)] = y;
                    }
                }
            }
        }
        intra = wave_sum_i64(intra);
        marks = (unsigned long long)wave_sum_i64((int64_t)marks);
        if (lane_id() == 0) { s_intra[threadIdx.x / MC_WAVE] = intra; s_marks[threadIdx.x / MC_WAVE] = marks; }
        __syncthreads();
        if (threadIdx.x == 0) {
            long long si = 0;
            unsigned long long sm = 0;
            for (int k = 0; k < ET / MC_WAVE; k++) { si += s_intra[k]; sm += s_marks[k]; }
            unsigned long long* sp = a.spread + ((size_t)p * SPREAD + blockIdx.x % SPREAD) * SPREAD_STRIDE;
            if (si) atomicAdd(&sp[0], (unsigned long long)si);
            if (sm) atomicAdd(&sp[1], sm);
            s_base = s_nc ? atomicAdd(&w.ctl->tail, s_nc) : 0;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < s_nc; i += ET) w.fifo[s_base + i] = s_cross[i];
    }
}

// fold every hub's partial sums of the step into its r (one wavefront per
// hub and pass; the hub's word has no other writer during this launch)
__global__ __launch_bounds__(256) void k_cfs_hubfix(StepArgs a) {
    static_assert(HUB_SLOTS <= MC_WAVE, "one lane per partial sum");
    const int32_t nh = *a.nhub;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / MC_WAVE);
    const int lane = lane_id();
    for (int64_t t = (int64_t)blockIdx.x * (blockDim.x / MC_WAVE) + threadIdx.x / MC_WAVE;
         t < (int64_t)nh * a.pv.passes; t += nwaves) {
        const int32_t p = (int32_t)(t / nh), h = (int32_t)(t % nh);
        PassView w = view(a, p);
        StepCtl& c = *w.ctl;
        if (c.done) continue;                     // uniform over the wavefront
        unsigned long long* hs = w.hacc + (size_t)h * HUB_SLOTS * 2;
        int64_t sum = 0;
        unsigned long long best = 0;
        if (lane < HUB_SLOTS) {
            sum = (int64_t)hs[2 * lane];
            best = hs[2 * lane + 1];
            if (sum) { hs[2 * lane] = 0; hs[2 * lane + 1] = 0; }
        }
        sum = wave_sum_i64(sum);
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long b2 = __shfl_xor(best, o, MC_WAVE);
            best = b2 > best ? b2 : best;
        }
        if (lane == 0 && sum > 0) {
            const int32_t y = a.hv[h];
            const unsigned long long ow = w.rw[y];
            w.rw[y] = ow + (unsigned long long)sum;
            const int64_t old = (int64_t)(ow & R_MASK);
            if (old < c.lam && c.lam <= old + sum) {
                // the heaviest entry crosses lam in some order of the step's
                // entries (only when its weight is exact, below saturation)
                if ((best >> 32) < HUB_WSAT && uf_union(a.pv.parent, (int32_t)(best & 0xFFFFFFFFu), y)) {
                    unsigned long long* sp = a.spread + ((size_t)p * SPREAD + h % SPREAD) * SPREAD_STRIDE;
                    atomicAdd(&sp[1], 1ULL);
                }
                w.fifo[atomicAdd(&c.tail, 1)] = y;
            }
        }
    }
}

// the batch becomes scanned; alpha and the bound of the pass move on
__global__ __launch_bounds__(T) void k_cfs_finish(StepArgs a) {
    __shared__ Red R;
    const int p = blockIdx.x, tid = threadIdx.x;
    PassView w = view(a, p);
    StepCtl& c = *w.ctl;
    if (c.done) return;
    const int32_t B = c.bcount;
    const int32_t* src = c.bsingle ? w.single : w.fifo + (c.head - B);
    const int32_t base = c.nscan;
    int32_t run = 0;
    for (int32_t c0 = 0; c0 < B; c0 += T) {
        const int32_t i = c0 + tid;
        bool ok = false;
        int32_t x = -1;
        if (i < B) {
            x = src[i];
            ok = (ldw(&w.rw[x]) >> 62) == 3;
        }
        int32_t tot;
        const int32_t ex = bscan(ok ? 1 : 0, tot, R);
        if (ok) {
            atomicAnd(&w.rw[x], ~BATCH_BIT);
            w.order[base + run + ex] = x;
        }
        run += tot;
    }
    // fold the step's spread partial sums (intra-batch weight, marks)
    __shared__ unsigned long long s_sum[2];
    if (tid < MC_WAVE) {
        unsigned long long* sp = a.spread + ((size_t)p * SPREAD + tid) * SPREAD_STRIDE;
        const int64_t si = wave_sum_i64((int64_t)sp[0]);
        const int64_t sm = wave_sum_i64((int64_t)sp[1]);
        sp[0] = 0;
        sp[1] = 0;
        if (tid == 0) { s_sum[0] = (unsigned long long)si; s_sum[1] = (unsigned long long)sm; }
    }
    __syncthreads();
    if (tid == 0) {
        const int32_t n = a.pv.g.n;
        c.intra = (int64_t)s_sum[0];
        if (s_sum[1]) { c.marks += s_sum[1]; atomicAdd(a.pv.marks, s_sum[1]); }
        c.nscan = base + run;
        c.alpha += c.part - c.intra;
        if (c.nscan < n) {
            if (c.alpha < c.best_alpha) { c.best_alpha = c.alpha; c.best_len = c.nscan; }
            if (c.alpha < c.lam) c.lam = c.alpha;
        }
        c.steps++;
    }
}

// leave the vertex words zero (many workgroups per pass); publish results
constexpr int END_SPLIT = 64;

__global__ __launch_bounds__(T) void k_cfs_end(StepArgs a) {
    const int p = blockIdx.x / END_SPLIT, part = blockIdx.x % END_SPLIT;
    PassView w = view(a, p);
    const StepCtl& c = *w.ctl;
    for (int32_t i = part * T + threadIdx.x; i < a.pv.g.n; i += END_SPLIT * T) w.rw[i] = 0;
    if (part == 0 && threadIdx.x == 0) {
        a.pv.nscan[p] = c.nscan;
        a.pv.alpha[p] = c.best_alpha;
        a.pv.alpha_len[p] = c.best_len;
        a.pv.lam_out[p] = c.lam;
        if (a.pv.steps) a.pv.steps[p] = c.steps;
        if (a.pv.diag) {
            int64_t* d = a.pv.diag + (int64_t)p * 8;
            d[0] = c.steps; d[1] = c.singles; d[2] = 0; d[3] = c.entries;
            d[4] = 0; d[5] = 0; d[6] = c.nscan; d[7] = c.maxbatch;
        }
        // algorithmic bytes of the pass's edge launches (profiling): 12 B
        // per scanned entry (col, w), 5 B per scanned vertex
        if (a.prof) atomicAdd(a.prof + (size_t)(p % PROF_LANES) * PROF_STRIDE,
                              (unsigned long long)(12 * c.entries + 5 * (int64_t)c.nscan));
    }
}

}  // namespace

// the kernels of one whole-GPU step
static bool launch_step(const StepArgs& a, int hub_blocks, int tile_blocks, bool timed, hipStream_t s) {
    k_cfs_popscan<<<POP_BLOCKS, POP_T, 0, s>>>(a);
    MC_LAUNCHED("k_cfs_popscan");
    k_cfs_plan<<<a.pv.passes, T, 0, s>>>(a);
    MC_LAUNCHED("k_cfs_plan");
    k_cfs_tiles<<<1, T, 0, s>>>(a);
    MC_LAUNCHED("k_cfs_tiles");
    k_cfs_tileinfo<<<tile_blocks, 256, 0, s>>>(a);
    MC_LAUNCHED("k_cfs_tileinfo");
    if (timed) prof_begin(PK_CFS_EDGES, s);
    k_cfs_edges<<<4096, ET, 0, s>>>(a);
    MC_LAUNCHED("k_cfs_edges");
    if (timed) prof_end(PK_CFS_EDGES, s);
    k_cfs_hubfix<<<hub_blocks, 256, 0, s>>>(a);
    MC_LAUNCHED("k_cfs_hubfix");
    k_cfs_finish<<<a.pv.passes, T, 0, s>>>(a);
    MC_LAUNCHED("k_cfs_finish");
    return true;
}

bool capforest_steps(StepArgs& a, int32_t* running_host, hipStream_t s, hipStream_t cap) {
    const int32_t P = a.pv.passes;
    if (P <= 0) return true;
    if (a.pv.g.n > a.pv.stride) {
        mc_hip_ok(hipErrorInvalidValue, "capforest_steps: per-pass arrays too small");
        return false;
    }
    a.prof = prof_dev_bytes(PK_CFS_EDGES);
    if (!fill_i32(a.nhub, 0, 1, s)) return false;
    k_cfs_hubs<<<std::max(1, std::min<int>((a.pv.g.n + 255) / 256, 8192)), 256, 0, s>>>(a);
    MC_LAUNCHED("k_cfs_hubs");
    // enough wavefronts for every (pass, hub) pair of a typical graph in one
    // sweep; the kernel strides over the rest
    const int hub_blocks = std::max(1, std::min<int>((int)(((int64_t)P * a.max_hubs + 3) / 4), 2048));
    const int tile_blocks = std::max(1, std::min<int>((int)((a.max_tiles + 255) / 256), 1024));
    k_cfs_init<<<P, T, 0, s>>>(a);
    MC_LAUNCHED("k_cfs_init");
    // Steps run in groups of `poll` between two reads of the running flag
    // (a finished pass leaves later steps with nothing to do). A group's
    // launches take the same arguments every time (the state is on the
    // device), so with kernel timing off it is captured once as a HIP graph
    // and replayed: one graph launch instead of 7 * poll kernel launches.
    const int poll = 4;
    const bool timed = a.prof != nullptr;
    hipGraphExec_t exec = nullptr;
    if (cap && !timed) {
        hipGraph_t graph = nullptr;
        bool ok = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
        for (int k = 0; ok && k < poll; k++) ok = launch_step(a, hub_blocks, tile_blocks, false, cap);
        ok = hipStreamEndCapture(cap, &graph) == hipSuccess && ok;
        if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
        if (!ok) {
            // no graph: the eager launches below (clear the capture's error)
            exec = nullptr;
            (void)hipGetLastError();
        }
    }
    a.steps_run = 0;
    for (int32_t step = 0;; step += poll) {
        a.steps_run = step + poll;
        if (exec) {
            if (hipGraphLaunch(exec, s) != hipSuccess) {
                (void)hipGraphExecDestroy(exec);
                return mc_hip_ok(hipErrorUnknown, "capforest_steps: graph launch failed");
            }
        } else {
            for (int k = 0; k < poll; k++)
                if (!launch_step(a, hub_blocks, tile_blocks, timed, s)) return false;
        }
        bool fail = hipMemcpyAsync(running_host, a.running, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess;
        if (fail || *running_host == 0 || step > 4 * (int64_t)a.pv.g.n + 64) {
            if (exec) (void)hipGraphExecDestroy(exec);
            if (fail) return mc_hip_ok(hipErrorUnknown, "capforest_steps: poll failed");
            if (*running_host == 0) break;
            mc_hip_ok(hipErrorUnknown, "capforest_steps: no progress");
            return false;
        }
    }
    // the passes' scan counts, for the caller's choice of a complete pass
    std::vector<StepCtl> ctl((size_t)P);
    MC_HIP(hipMemcpyAsync(ctl.data(), a.ctl, sizeof(StepCtl) * (size_t)P, hipMemcpyDeviceToHost, s));
    k_cfs_end<<<P * END_SPLIT, T, 0, s>>>(a);
    MC_LAUNCHED("k_cfs_end");
    MC_HIP(hipStreamSynchronize(s));
    a.scans_run = 0;
    for (const StepCtl& c : ctl) a.scans_run += c.nscan;
    return true;
}
