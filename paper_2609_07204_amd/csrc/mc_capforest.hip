// CAPFOREST (paper, Section 2.1 and Algorithm 1 "Parallel CAPFOREST").
//
// A pass grows a scanned set S from a start vertex, always scanning the
// queued vertex y with the largest key min(r(y), lam), where r(y) is the
// weight between y and S (bounded priorities, Section 2.1). Scanning x adds
// c(x) - 2 r(x) to alpha, the capacity of the cut (S, V\S), which bounds
// lambda while S is a proper subset. Each edge e = {x,y} to an unscanned y
// with r(y) < lam <= r(y) + c(e) is contractible (its endpoints have
// connectivity at least lam), so x and y are unioned.
//
// k_capforest_passes: many passes at once, one wavefront per pass. Per-pass
// state (r, queue membership) lives in an LDS hash of CF_HC vertices; the
// 64 lanes scan x's row together (coalesced 12 B/entry loads) and update r
// with LDS operations. With `shared`, the passes share one visited array:
// a pass that pops a vertex already claimed by another pass blacklists it
// (Algorithm 1, T and B). A pass also blacklists a vertex whose row would
// overflow its hash and stops when its length cap is reached. Leaving out
// vertices in either way keeps every mark valid: the argument for a mark
// only involves S and the marked vertex (keys compared in S's order), and
// stopping early just ends the pass at a prefix.
//
// k_capforest_complete: the sequential CAPFOREST of Algorithm 2's fallback.
// One wavefront, no capacity limit: r and queue state are dense arrays in
// HBM, and an exact pop (largest key, smallest id on ties) uses a
// two-level maximum over 64-vertex blocks (level 1 in HBM, level 2 in LDS).
#include "mc_internal.h"

namespace {

constexpr int CF_FILL = CF_HC * 3 / 4;   // touched vertices allowed per pass
constexpr int64_t NO_ALPHA = INT64_MAX;

__device__ __forceinline__ int64_t ld64(const int64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t pick_start(const CapforestArgs& a, int p) {
    const int32_t n = a.g.n;
    if (a.start >= 0) return a.start;
    int32_t s = 0;
    for (int attempt = 0; attempt < 4; attempt++) {
        uint64_t h = splitmix64(a.seed ^ splitmix64(((uint64_t)(uint32_t)a.tag << 32) ^ (uint64_t)p * 8 + attempt));
        s = (int32_t)(((h >> 32) * (uint64_t)n) >> 32);
        if (!a.shared || ld_acq(&a.claim[s]) != a.tag) break;
    }
    return s;
}

__global__ __launch_bounds__(MC_WAVE) void k_capforest_passes(CapforestArgs a) {
    __shared__ int32_t hkey[CF_HC];
    __shared__ int64_t hr[CF_HC];
    __shared__ uint8_t hst[CF_HC];       // 0 queued, 1 scanned, 2 blacklisted
    __shared__ int16_t qlist[CF_HC];     // queued slots
    __shared__ int32_t s_qn, s_used;

    const int p = blockIdx.x;
    const int lane = threadIdx.x;
    const int32_t n = a.g.n;
    for (int i = lane; i < CF_HC; i += MC_WAVE) hkey[i] = -1;
    int64_t lam = *a.lam;
    __syncthreads();
    if (lane == 0) {
        const int32_t s = pick_start(a, p);
        uint32_t h = hash32((uint32_t)s) & (CF_HC - 1);
        hkey[h] = s;
        hr[h] = 0;
        hst[h] = 0;
        qlist[0] = (int16_t)h;
        s_qn = 1;
        s_used = 1;
    }
    __syncthreads();

    int64_t alpha = 0, best_alpha = NO_ALPHA;
    int32_t best_len = 0, nscan = 0;
    unsigned long long marks = 0;
    int32_t* order = a.order + (int64_t)p * CF_HC;

    int32_t pops = 0;
    for (;;) {
        const int32_t qn = s_qn;
        if (qn == 0 || (a.len_cap > 0 && nscan >= a.len_cap)) break;
        // a vertex another pass scanned, or whose row no longer fits, is
        // blacklisted without a scan; pop_cap bounds those pops too
        if (a.pop_cap > 0 && pops++ >= a.pop_cap) break;
        // pop: largest min(r, lam), then smallest vertex id
        int64_t bk = -1;
        int32_t bv = -1, bq = -1;
        for (int32_t i = lane; i < qn; i += MC_WAVE) {
            const int sl = qlist[i];
            const int32_t v = hkey[sl];
            const int64_t r = hr[sl];
            const int64_t k = r < lam ? r : lam;
            if (bv < 0 || k > bk || (k == bk && v < bv)) { bk = k; bv = v; bq = i; }
        }
        wave_argmax(bk, bv, bq);
        const int32_t x = bv;
        const int sx = qlist[bq];
        __syncthreads();
        if (lane == 0) { qlist[bq] = qlist[qn - 1]; s_qn = qn - 1; }
        const int64_t rx = hr[sx];
        const int32_t ox = a.g.off[x], lx = a.g.len[x];
        const int64_t dx = a.g.deg[x];
        bool ok = s_used + lx <= CF_FILL;
        if (ok && a.shared) {
            int32_t old = 0;
            if (lane == 0) old = atomicExch(&a.claim[x], a.tag);
            ok = __shfl(old, 0, MC_WAVE) != a.tag;
        }
        if (!ok) {
            if (lane == 0) hst[sx] = 2;
            __syncthreads();
            continue;
        }
        if (lane == 0) { hst[sx] = 1; order[nscan] = x; }
        alpha += dx - 2 * rx;
        nscan++;
        if (nscan < n) {
            if (alpha < best_alpha) { best_alpha = alpha; best_len = nscan; }
            if (alpha < lam) lam = alpha;
        }
        __syncthreads();
        for (int32_t j = lane; j < lx; j += MC_WAVE) {
            const int32_t y = a.g.col[ox + j];
            const int64_t c = a.g.w[ox + j];
            uint32_t h = hash32((uint32_t)y) & (CF_HC - 1);
            bool fresh = false;
            for (;;) {
                const int32_t k = hkey[h];
                if (k == y) break;
                if (k == -1) {
                    const int32_t old = atomicCAS(&hkey[h], -1, y);
                    if (old == -1) { fresh = true; break; }
                    if (old == y) break;
                }
                h = (h + 1) & (CF_HC - 1);
            }
            int64_t r = 0;
            if (fresh) {
                hst[h] = 0;
                const int32_t qi = atomicAdd(&s_qn, 1);
                qlist[qi] = (int16_t)h;
                atomicAdd(&s_used, 1);
            } else {
                if (hst[h] != 0) continue;
                r = hr[h];
            }
            if (r < lam && lam <= r + c && uf_union(a.parent, x, y)) marks++;
            hr[h] = r + c;
        }
        __syncthreads();
    }
    marks = (unsigned long long)wave_sum_i64((int64_t)marks);
    if (lane == 0) {
        a.nscan[p] = nscan;
        a.alpha[p] = best_alpha;
        a.alpha_len[p] = best_len;
        a.lam_out[p] = lam;
        if (marks) atomicAdd(a.marks, marks);
    }
}

__global__ __launch_bounds__(MC_WAVE) void k_capforest_reduce(const int64_t* alpha, const int32_t* alen, int passes,
                                                              DevScalars* sc) {
    int64_t best = 0;
    int32_t bp = -1;
    for (int p = threadIdx.x; p < passes; p += MC_WAVE) {
        const int64_t v = alpha[p];
        if (v != NO_ALPHA && (bp < 0 || v < best)) { best = v; bp = p; }
    }
    wave_argmin(best, bp);
    if (threadIdx.x == 0) {
        sc->best_alpha = bp >= 0 ? best : NO_ALPHA;
        sc->best_pass = bp;
        sc->best_len = bp >= 0 ? alen[bp] : 0;
    }
}

__global__ __launch_bounds__(MC_WAVE) void k_capforest_complete(CompleteArgs a) {
    extern __shared__ long long l2[];
    const int lane = threadIdx.x;
    const int32_t n = a.g.n;
    const int32_t nb1 = (n + 63) / 64;
    const int32_t nb2 = (nb1 + 63) / 64;
    const int32_t TQ = a.tag * 4 + 1, TS = a.tag * 4 + 2;
    for (int i = lane; i < nb2; i += MC_WAVE) l2[i] = -1;
    int64_t lam = *a.lam;
    __syncthreads();
    if (lane == 0) {
        const int32_t s = a.start;
        a.r[s] = 0;
        a.st[s] = TQ;
        atomicMax((long long*)&a.l1[s >> 6], 0LL);
        l2[s >> 12] = 0;
    }
    __threadfence();
    __syncthreads();

    int64_t alpha = 0, best_alpha = NO_ALPHA;
    int32_t best_len = 0, nscan = 0, queued = 1;
    unsigned long long marks = 0;
    while (queued > 0) {
        // level 2: K = min(max r over the queue, lam)
        int64_t m = -1;
        for (int i = lane; i < nb2; i += MC_WAVE) m = l2[i] > m ? l2[i] : m;
        for (int o = 32; o > 0; o >>= 1) { int64_t t = __shfl_xor(m, o, MC_WAVE); m = t > m ? t : m; }
        if (m < 0) break;
        const int64_t K = m < lam ? m : lam;
        // first level-2 group holding a vertex with r >= K
        int32_t g2 = INT32_MAX;
        for (int i = lane; i < nb2; i += MC_WAVE)
            if (l2[i] >= K) { g2 = i; break; }
        for (int o = 32; o > 0; o >>= 1) { int32_t t = __shfl_xor(g2, o, MC_WAVE); g2 = t < g2 ? t : g2; }
        // the two index levels always agree with the queue; stop rather than
        // index out of range if they ever did not
        if (g2 >= nb2) { if (lane == 0) a.nscan[0] = -1; return; }
        // first level-1 block in that group
        const int32_t b1i = g2 * 64 + lane;
        const int64_t v1 = b1i < nb1 ? ld64(&a.l1[b1i]) : -1;
        const unsigned long long hit1 = __ballot(v1 >= K);
        if (hit1 == 0) { if (lane == 0) a.nscan[0] = -1; return; }
        const int32_t b1 = g2 * 64 + (int32_t)__ffsll((long long)hit1) - 1;
        // the vertex: first queued vertex of the block with r >= K
        const int32_t xv = b1 * 64 + lane;
        const int32_t sv = xv < n ? ld_acq(&a.st[xv]) : 0;
        const int64_t rv = sv == TQ ? ld64(&a.r[xv]) : -1;
        const unsigned long long hit0 = __ballot(sv == TQ && rv >= K);
        if (hit0 == 0) { if (lane == 0) a.nscan[0] = -1; return; }
        const int xl = (int)__ffsll((long long)hit0) - 1;
        const int32_t x = b1 * 64 + xl;
        const int64_t rx = __shfl(rv, xl, MC_WAVE);
        // remove x and refresh both levels
        int64_t nb = (sv == TQ && lane != xl) ? rv : -1;
        for (int o = 32; o > 0; o >>= 1) { int64_t t = __shfl_xor(nb, o, MC_WAVE); nb = t > nb ? t : nb; }
        int64_t n2v = (b1i < nb1) ? (b1i == b1 ? nb : v1) : -1;
        for (int o = 32; o > 0; o >>= 1) { int64_t t = __shfl_xor(n2v, o, MC_WAVE); n2v = t > n2v ? t : n2v; }
        if (lane == 0) {
            a.st[x] = TS;
            __hip_atomic_store(&a.l1[b1], nb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            l2[g2] = n2v;
            a.order[nscan] = x;
        }
        queued--;
        const int32_t ox = a.g.off[x], lx = a.g.len[x];
        alpha += a.g.deg[x] - 2 * rx;
        nscan++;
        if (nscan < n) {
            if (alpha < best_alpha) { best_alpha = alpha; best_len = nscan; }
            if (alpha < lam) lam = alpha;
        }
        __threadfence();
        __syncthreads();
        int32_t added = 0;
        for (int32_t j = lane; j < lx; j += MC_WAVE) {
            const int32_t y = a.g.col[ox + j];
            const int64_t c = a.g.w[ox + j];
            const int32_t sy = ld_acq(&a.st[y]);
            if (sy == TS) continue;
            int64_t r = 0;
            if (sy == TQ) r = ld64(&a.r[y]);
            else { a.st[y] = TQ; added++; }
            if (r < lam && lam <= r + c && uf_union(a.parent, x, y)) marks++;
            const int64_t rn = r + c;
            __hip_atomic_store(&a.r[y], rn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            atomicMax((long long*)&a.l1[y >> 6], (long long)rn);
            atomicMax(&l2[y >> 12], (long long)rn);
        }
        queued += wave_sum_i32(added);
        __threadfence();
        __syncthreads();
    }
    marks = (unsigned long long)wave_sum_i64((int64_t)marks);
    if (lane == 0) {
        a.nscan[0] = nscan;
        a.alpha[0] = best_alpha;
        a.alpha_len[0] = best_len;
        a.lam_out[0] = lam;
        if (marks) atomicAdd(a.marks, marks);
    }
}

}  // namespace

bool capforest_passes(const CapforestArgs& a, hipStream_t s) {
    if (a.passes <= 0) return true;
    k_capforest_passes<<<a.passes, MC_WAVE, 0, s>>>(a);
    MC_LAUNCHED("k_capforest_passes");
    return true;
}

bool capforest_reduce(const CapforestArgs& a, DevScalars* sc, hipStream_t s) {
    k_capforest_reduce<<<1, MC_WAVE, 0, s>>>(a.alpha, a.alpha_len, a.passes, sc);
    MC_LAUNCHED("k_capforest_reduce");
    return true;
}

bool capforest_complete(const CompleteArgs& a, hipStream_t s) {
    const int32_t nb1 = (a.g.n + 63) / 64;
    const int32_t nb2 = (nb1 + 63) / 64;
    const size_t lds = (size_t)nb2 * sizeof(long long);
    if (lds > 64 * 1024) {
        mc_hip_ok(hipErrorInvalidValue, "capforest_complete: graph too large for the level-2 index");
        return false;
    }
    if (!fill_i64(a.l1, -1, nb1, s) || !fill_i32(a.st, 0, a.g.n, s)) return false;
    k_capforest_complete<<<1, MC_WAVE, lds, s>>>(a);
    MC_LAUNCHED("k_capforest_complete");
    return true;
}
