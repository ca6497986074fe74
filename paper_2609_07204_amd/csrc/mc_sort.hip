// Contraction by sorting: the edge merge of a contraction (paper, Section 2:
// contracting a set of vertices sums the weights of parallel edges and
// drops loops; Section 2.1 "Parallel CAPFOREST and contraction") as a radix
// sort of the contracted entries followed by a segmented reduction, the
// alternative to the hash merge of mc_contract.hip (options.contract_mode).
//
//  1. emit: every entry (u, x, w) with w > 0 whose ends land in different
//     groups becomes a key a * 2^bits + b (a = L[u], b = L[x], bits enough
//     for n2 + 1 values) with its weight; rows are cut into pieces of at
//     most 1024 entries and every wavefront takes an equal range of pieces;
//     a first pass counts each wavefront's entries, a prefix over the
//     wavefronts places them, and a second pass writes them (exact, in row
//     order, no atomics);
//  2. an LSD radix sort of the keys with their weights, 8 bits per pass,
//     over the 2 bits of the keys only; each pass takes a histogram per
//     4096-item tile, one prefix over (digit, tile), and a stable scatter
//     that ranks equal digits inside a wavefront with ballots;
//  3. the runs of equal keys are the contracted entries: a prefix over the
//     run heads numbers them, a wavefront-level segmented sum adds their
//     weights (one atomic per run and wavefront), each row's first and last
//     run set its offset and length, and the same segmented sum keyed by
//     row gives the degrees.
// Rows come out sorted by target. The result is the same padded CSR as the
// hash merge's (the parity tests compare both to the oracle).
#include "mc_internal.h"

namespace {

constexpr int RS_T = 256;                      // threads of the sort kernels
constexpr int RS_ITEMS = 16;                   // items per thread and tile
constexpr int RS_TILE = RS_T * RS_ITEMS;       // 4096
constexpr int RS_RADIX = 256;                  // 8-bit digits
constexpr int EM_T = 256;                      // threads of the emit kernels
constexpr int EM_WAVES = EM_T / MC_WAVE;
static_assert(RS_T == RS_RADIX, "one thread per digit in the sort kernels");

inline int grid_for(int64_t count, int threads, int cap = 8192) {
    int64_t b = (count + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

__device__ __forceinline__ uint64_t lanes_below() {
    const int lane = lane_id();
    return lane == 0 ? 0ULL : (~0ULL >> (64 - lane));
}

// Units of the emit passes: each row of a kept vertex is cut into pieces of
// at most EM_PIECE entries; ucnt[v] = pieces of row v (exclusive prefix ->
// the first unit of the row).
constexpr int EM_PIECE = 1024;
__global__ void k_sort_units(DGraph src, const int32_t* __restrict__ L, int32_t* __restrict__ ucnt) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < src.n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = L ? L[v] : (int32_t)v;
        const int32_t l = a >= 0 ? src.len[v] : 0;
        ucnt[v] = (l + EM_PIECE - 1) / EM_PIECE;
    }
}

// One traversal for both emit passes: wavefront w takes a contiguous range
// of units (a long row is spread over several wavefronts), 64 entries per
// step. With okey == nullptr it only counts (cnt[w]); otherwise it writes
// its entries from base[w] on, in the same order.
__global__ __launch_bounds__(EM_T) void k_sort_emit(DGraph src, const int32_t* __restrict__ L, int32_t bits,
                                                  const int32_t* __restrict__ ustart, int32_t* __restrict__ cnt,
                                                  const int32_t* __restrict__ base, uint64_t* __restrict__ okey,
                                                  int64_t* __restrict__ oval) {
    const int lane = lane_id();
    const int64_t nw = (int64_t)gridDim.x * EM_WAVES;
    const int64_t wid = (int64_t)blockIdx.x * EM_WAVES + threadIdx.x / MC_WAVE;
    const int64_t units = ustart[src.n];
    const int64_t per = (units + nw - 1) / nw;
    const int64_t u0 = wid * per, u1 = u0 + per < units ? u0 + per : units;
    int32_t pos = okey ? base[wid] : 0;
    if (u0 < u1) {
        // the row of the first unit: the last v with ustart[v] <= u0 (rows
        // without units have ustart[v] == ustart[v + 1])
        int32_t lo = 0, hi = src.n;
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (ustart[mid] <= u0) lo = mid; else hi = mid;
        }
        int32_t v = lo;
        for (int64_t u = u0; u < u1; u++) {
            while (ustart[v + 1] <= u) v++;
            const int32_t a = L ? L[v] : v;
            const int32_t o = src.off[v], l = src.len[v];
            const int32_t j0 = (int32_t)(u - ustart[v]) * EM_PIECE;
            const int32_t j1 = j0 + EM_PIECE < l ? j0 + EM_PIECE : l;
            for (int32_t jb = j0; jb < j1; jb += MC_WAVE) {
                const int32_t j = jb + lane;
                bool e = false;
                uint64_t k = 0;
                int64_t w = 0;
                if (j < j1) {
                    const int32_t x = src.col[o + j];
                    w = src.w[o + j];
                    const int32_t b = L ? L[x] : x;
                    e = w > 0 && b >= 0 && b != a;
                    k = ((uint64_t)(uint32_t)a << bits) | (uint32_t)b;
                }
                const uint64_t m = __ballot(e);
                if (okey && e) {
                    const int32_t at = pos + __popcll(m & lanes_below());
                    okey[at] = k;
                    oval[at] = w;
                }
                pos += __popcll(m);
            }
        }
    }
    if (!okey && lane == 0) cnt[wid] = pos;
}

// per-tile histogram of one digit: hist[d * ntiles + tile]
__global__ __launch_bounds__(RS_T) void k_rs_hist(const uint64_t* __restrict__ key, int64_t m, int shift,
                                                int32_t ntiles, int32_t* __restrict__ hist) {
    __shared__ int32_t h[RS_T / MC_WAVE][RS_RADIX];
    const int tid = threadIdx.x, wv = tid / MC_WAVE;
    for (int w = 0; w < RS_T / MC_WAVE; w++) h[w][tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll 4
    for (int r = 0; r < RS_ITEMS; r++) {
        const int64_t i = base + (int64_t)r * RS_T + tid;
        if (i < m) atomicAdd(&h[wv][(int)((key[i] >> shift) & (RS_RADIX - 1))], 1);
    }
    __syncthreads();
    int32_t s = 0;
    for (int w = 0; w < RS_T / MC_WAVE; w++) s += h[w][tid];
    hist[(int64_t)tid * ntiles + blockIdx.x] = s;
}

// stable scatter of one tile: its items in index order (round r, then
// thread), each placed at its digit's offset for this tile plus its rank
// among the equal digits before it
__global__ __launch_bounds__(RS_T) void k_rs_scatter(const uint64_t* __restrict__ kin, const int64_t* __restrict__ vin,
                                                   uint64_t* __restrict__ kout, int64_t* __restrict__ vout, int64_t m,
                                                   int shift, int32_t ntiles, const int32_t* __restrict__ offs) {
    __shared__ int32_t run[RS_RADIX];
    __shared__ int32_t wc[RS_T / MC_WAVE][RS_RADIX];
    const int tid = threadIdx.x, wv = tid / MC_WAVE;
    run[tid] = offs[(int64_t)tid * ntiles + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; r++) {
        const int64_t i = base + (int64_t)r * RS_T + tid;
        const bool valid = i < m;
        const uint64_t k = valid ? kin[i] : 0;
        const int64_t v = valid ? vin[i] : 0;
        const int d = (int)((k >> shift) & (RS_RADIX - 1));
        for (int w = 0; w < RS_T / MC_WAVE; w++) wc[w][tid] = 0;
        __syncthreads();
        // lanes of this wavefront with the same digit
        uint64_t eq = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; bit++) {
            const uint64_t b = __ballot(valid && ((d >> bit) & 1));
            eq &= ((d >> bit) & 1) ? b : ~b;
        }
        const int rank = __popcll(eq & lanes_below());
        if (valid && rank == 0) wc[wv][d] = __popcll(eq);
        __syncthreads();
        if (valid) {
            int32_t pre = run[d] + rank;
            for (int w = 0; w < wv; w++) pre += wc[w][d];
            kout[pre] = k;
            vout[pre] = v;
        }
        __syncthreads();
        int32_t add = 0;
        for (int w = 0; w < RS_T / MC_WAVE; w++) add += wc[w][tid];
        run[tid] += add;
    }
}

// run heads of the sorted keys
__global__ void k_rs_heads(const uint64_t* __restrict__ key, int64_t m, int32_t* __restrict__ flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        flag[i] = i == 0 || key[i] != key[i - 1];
}

// Segmented sums of the runs, one wavefront-striped pass: item i of run u
// (uidx: exclusive prefix of the heads). A run's head writes the target,
// the last item of each run's piece in a wavefront adds the piece's sum,
// and a row's first and last runs set its offset and end.
__global__ void k_rs_reduce(const uint64_t* __restrict__ key, const int64_t* __restrict__ val, int64_t m,
                            const int32_t* __restrict__ head, const int32_t* __restrict__ uidx, int32_t bits,
                            DGraph dst, int32_t* __restrict__ rend) {
    const uint64_t mask = ((uint64_t)1 << bits) - 1;
    const int lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // the trip count is the same for all lanes of a wavefront
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x - lane); i0 < m; i0 += stride) {
        const int64_t i = i0 + lane;
        const bool valid = i < m;
        const uint64_t k = valid ? key[i] : 0;
        int64_t s = valid ? val[i] : 0;
        const bool h = valid && head[i];
        const int32_t u = valid ? uidx[i] - (h ? 0 : 1) : 0;
        // inclusive segmented sum inside the wavefront
        bool f = h || lane == 0;
        for (int d = 1; d < MC_WAVE; d <<= 1) {
            const int64_t t = __shfl_up(s, d);
            const bool g = __shfl_up(f, d);
            if (lane >= d) {
                if (!f) s += t;
                f = f || g;
            }
        }
        if (!valid) continue;
        const bool last_in_run = i + 1 >= m || head[i + 1];
        const int32_t a = (int32_t)(k >> bits);
        if (h) {
            dst.col[u] = (int32_t)(k & mask);
            if (i == 0 || (int32_t)(key[i - 1] >> bits) != a) dst.off[a] = u;
        }
        if (last_in_run || lane == MC_WAVE - 1) atomic_add_i64(&dst.w[u], s);
        if (last_in_run && (i + 1 >= m || (int32_t)(key[i + 1] >> bits) != a)) rend[a] = u + 1;
    }
}

// degrees: the same wavefront-level segmented sum keyed by row (one atomic
// per row and wavefront, so a row of millions of entries costs thousands
// of atomics, not a loop over its entries)
__global__ void k_rs_degrees(const uint64_t* __restrict__ key, const int64_t* __restrict__ val, int64_t m,
                             int32_t bits, int64_t* __restrict__ deg) {
    const int lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x - lane); i0 < m; i0 += stride) {
        const int64_t i = i0 + lane;
        const bool valid = i < m;
        const int32_t a = valid ? (int32_t)(key[i] >> bits) : -1;
        int64_t s = valid ? val[i] : 0;
        const bool h = valid && (i == 0 || (int32_t)(key[i - 1] >> bits) != a);
        bool f = h || lane == 0;
        for (int d = 1; d < MC_WAVE; d <<= 1) {
            const int64_t t = __shfl_up(s, d);
            const bool g = __shfl_up(f, d);
            if (lane >= d) {
                if (!f) s += t;
                f = f || g;
            }
        }
        if (!valid) continue;
        const bool last = i + 1 >= m || (int32_t)(key[i + 1] >> bits) != a;
        if (last || lane == MC_WAVE - 1) atomic_add_i64(&deg[a], s);
    }
}

// lengths (rows without entries keep offset 0 and end 0)
__global__ void k_rs_rows(DGraph dst, const int32_t* __restrict__ rend) {
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < dst.n; a += (int64_t)gridDim.x * blockDim.x)
        dst.len[a] = rend[a] - dst.off[a];
}

}  // namespace

void sort_ws_carve(Arena& a, int32_t n, int64_t cap, SortWS& w) {
    w.cap = cap;
    for (int q = 0; q < 2; q++) {
        w.key[q] = a.take<uint64_t>((size_t)cap + 1);
        w.val[q] = a.take<int64_t>((size_t)cap + 1);
    }
    w.flag = a.take<int32_t>((size_t)cap + 2);
    w.uidx = a.take<int32_t>((size_t)cap + 2);
    const int64_t ntiles = cap / RS_TILE + 2;
    w.hist = a.take<int32_t>((size_t)(RS_RADIX * ntiles + 2));
    w.scan_tmp = a.take<int32_t>(scan_tmp_elems(std::max<int64_t>(RS_RADIX * ntiles + 1, cap + 1)) + 16);
    w.wcnt = a.take<int32_t>((size_t)8192 * EM_WAVES + 2);
    w.rend = a.take<int32_t>((size_t)n + 1);
}

bool contract_sorted(const DGraph& src, const int32_t* L, int32_t n2, DGraph& dst, ContractWS& ws, DevScalars* sc,
                     hipStream_t s) {
    SortWS& w = ws.sw;
    dst.n = n2;
    int32_t bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) <= n2) bits++;   // labels and n2 itself fit in bits
    // 1. emit: units, count per wavefront, place, write
    k_sort_units<<<grid_for(src.n, 256), 256, 0, s>>>(src, L, w.rend);
    MC_LAUNCHED("k_sort_units");
    if (!scan_i32(w.rend, w.rend, src.n, w.scan_tmp, s)) return false;
    const int eb = grid_for((int64_t)src.n, 64 * EM_WAVES, 8192);
    const int64_t nw = (int64_t)eb * EM_WAVES;
    k_sort_emit<<<eb, EM_T, 0, s>>>(src, L, bits, w.rend, w.wcnt, nullptr, nullptr, nullptr);
    MC_LAUNCHED("k_sort_emit");
    if (!scan_i32(w.wcnt, w.wcnt, nw, w.scan_tmp, s)) return false;
    k_sort_emit<<<eb, EM_T, 0, s>>>(src, L, bits, w.rend, nullptr, w.wcnt, w.key[0], w.val[0]);
    MC_LAUNCHED("k_sort_emit");
    int32_t m32 = 0;
    if (!mc_hip_ok(hipMemcpyAsync(&m32, w.wcnt + nw, sizeof(int32_t), hipMemcpyDeviceToHost, s), "sort: count") ||
        !mc_hip_ok(hipStreamSynchronize(s), "sort: count"))
        return false;
    const int64_t m = m32;
    // 2. radix sort on 2 bits of key
    int cur = 0;
    if (m > 1) {
        const int32_t ntiles = (int32_t)((m + RS_TILE - 1) / RS_TILE);
        for (int shift = 0; shift < 2 * bits; shift += 8) {
            k_rs_hist<<<ntiles, RS_T, 0, s>>>(w.key[cur], m, shift, ntiles, w.hist);
            MC_LAUNCHED("k_rs_hist");
            if (!scan_i32(w.hist, w.hist, (int64_t)RS_RADIX * ntiles, w.scan_tmp, s)) return false;
            k_rs_scatter<<<ntiles, RS_T, 0, s>>>(w.key[cur], w.val[cur], w.key[cur ^ 1], w.val[cur ^ 1], m, shift,
                                                 ntiles, w.hist);
            MC_LAUNCHED("k_rs_scatter");
            cur ^= 1;
        }
    }
    // 3. runs -> rows (rend is free again: the units were only for the emit)
    if (!fill_i32(dst.off, 0, n2, s) || !fill_i32(w.rend, 0, n2, s) || !fill_i64(dst.deg, 0, n2, s)) return false;
    if (m > 0) {
        if (!fill_i64(dst.w, 0, m, s)) return false;
        k_rs_heads<<<grid_for(m, 256), 256, 0, s>>>(w.key[cur], m, w.flag);
        MC_LAUNCHED("k_rs_heads");
        if (!scan_i32(w.flag, w.uidx, m, w.scan_tmp, s)) return false;
        k_rs_reduce<<<grid_for(m, 256), 256, 0, s>>>(w.key[cur], w.val[cur], m, w.flag, w.uidx, bits, dst, w.rend);
        MC_LAUNCHED("k_rs_reduce");
        k_rs_degrees<<<grid_for(m, 256), 256, 0, s>>>(w.key[cur], w.val[cur], m, bits, dst.deg);
        MC_LAUNCHED("k_rs_degrees");
    }
    k_rs_rows<<<grid_for(n2, 256), 256, 0, s>>>(dst, w.rend);
    MC_LAUNCHED("k_rs_rows");
    return min_degree(dst, ws, sc, s);
}
