// Batched exact minimum cuts: many graphs solved in one call, with one set
// of launches per round for all of them (Algorithm 2 run side by side).
//
// The graphs are laid side by side as one union graph: graph i owns the
// vertex range [voff[i], voff[i+1]) and no edge joins two ranges. Each step
// of the round then runs once on the union graph:
//  - the reduction tests read the bound of each vertex's own graph;
//  - CAPFOREST runs one pass per graph, each in one workgroup on its own
//    range (the instance mode of k_capforest_private), so small graphs cost
//    a workgroup, not a launch;
//  - union-find, relabelling and contraction are those of the single solve:
//    canonical labels number components by their smallest vertex, so every
//    graph's vertices stay contiguous and its new range is a prefix count
//    of the component roots;
//  - bounds, collapsed degrees (Section 2.1 "Overall algorithm"), the
//    sequential fallback of Algorithm 2 and the sides are kept per graph.
// A graph leaves the rounds when at most two of its vertices remain. The
// label-propagation heuristic is not run here: every graph starts from its
// minimum degree (the bound only changes the work, not the result).
#include <algorithm>
#include <vector>

#include "mc_internal.h"

namespace {

inline int grid_for(int64_t count, int threads, int cap = 8192) {
    int64_t b = (count + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

struct BatchGraph {
    const int32_t* rp;
    const int32_t* col;
    const int64_t* w;
    int32_t n;
    int32_t nnz;
};

// last index i in [0, k) with a[i] <= x (a non-decreasing, a[0] = 0 <= x)
__device__ __forceinline__ int32_t seg_of(const int32_t* a, int32_t k, int64_t x) {
    int32_t lo = 0, hi = k;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if ((int64_t)a[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ void bg_err(DevScalars* sc, int32_t code) { atomicCAS(&sc->err, 0, code); }

// Gather the graphs (device pointers in tab) into one CSR with shifted ids,
// checking each graph on its own: row_ptr monotone from 0 to nnz, targets
// in the graph's own range, weights >= 0.
__global__ void k_bg_gather(const BatchGraph* tab, int32_t k, const int32_t* voff, const int32_t* eoff, int32_t N,
                            int32_t C, int32_t* rp, int32_t* col, int64_t* w, DevScalars* sc) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = tid; v <= N; v += nth) {
        if (v == N) { rp[N] = C; continue; }
        const int32_t i = seg_of(voff, k, v);
        const BatchGraph gi = tab[i];
        const int32_t lv = (int32_t)v - voff[i];
        const int32_t a = gi.rp[lv], b = gi.rp[lv + 1];
        if (a > b || (lv == 0 && a != 0) || (lv == gi.n - 1 && b != gi.nnz)) bg_err(sc, MC_E_BAD_GRAPH);
        rp[v] = a + eoff[i];
    }
    for (int64_t e = tid; e < C; e += nth) {
        const int32_t i = seg_of(eoff, k, e);
        const BatchGraph gi = tab[i];
        const int32_t le = (int32_t)e - eoff[i];
        const int32_t x = gi.col[le];
        const int64_t c = gi.w[le];
        if (x < 0 || x >= gi.n || c < 0) bg_err(sc, MC_E_BAD_GRAPH);
        col[e] = x + voff[i];
        w[e] = c;
    }
}

// host inputs were copied as they are: shift row offsets and targets
__global__ void k_bg_shift(int32_t k, const int32_t* voff, const int32_t* eoff, int32_t N, int32_t C, int32_t* rp,
                           int32_t* col) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = tid; v <= N; v += nth) {
        if (v == N) { rp[N] = C; continue; }
        rp[v] += eoff[seg_of(voff, k, v)];
    }
    for (int64_t e = tid; e < C; e += nth) col[e] += voff[seg_of(eoff, k, e)];
}

__global__ void k_bg_vinst(const int32_t* voff, int32_t k, int32_t N, int32_t* vinst) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += (int64_t)gridDim.x * blockDim.x)
        vinst[v] = seg_of(voff, k, v);
}

// minimum degree of every graph's range, smallest vertex on ties (one
// workgroup per graph)
__global__ __launch_bounds__(256) void k_bg_segmin(const int64_t* deg, const int32_t* voff, int32_t k,
                                                  int64_t* dmin, int32_t* darg) {
    __shared__ int64_t sv[4];
    __shared__ int32_t si[4];
    for (int32_t i = blockIdx.x; i < k; i += gridDim.x) {
        int64_t best = 0;
        int32_t bid = -1;
        for (int32_t v = voff[i] + threadIdx.x; v < voff[i + 1]; v += 256) {
            const int64_t d = deg[v];
            if (bid < 0 || d < best) { best = d; bid = v; }
        }
        wave_argmin(best, bid);
        __syncthreads();
        if (lane_id() == 0) { sv[threadIdx.x / MC_WAVE] = best; si[threadIdx.x / MC_WAVE] = bid; }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int q = 1; q < 4; q++)
                if (si[q] >= 0 && (bid < 0 || sv[q] < best || (sv[q] == best && si[q] < bid))) { best = sv[q]; bid = si[q]; }
            dmin[i] = bid >= 0 ? best : INT64_MAX;
            darg[i] = bid;
        }
    }
}

// voff2[i] = number of component roots before voff[i] (scan of root flags)
__global__ void k_bg_offsets(const int32_t* scan, const int32_t* voff, int32_t k, int32_t* voff2) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= k; i += gridDim.x * blockDim.x)
        voff2[i] = scan[voff[i]];
}

// start of the rounds: bound = minimum degree (snapshot of its vertex);
// graphs in more than one component have lambda = 0
__global__ void k_bg_start(const int32_t* voff, const int32_t* voff2, int32_t k, const int64_t* dmin, int64_t* lam,
                           uint8_t* done, uint8_t* snap) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
        const int32_t ni = voff[i + 1] - voff[i];
        if (voff2[i + 1] - voff2[i] > 1) {
            lam[i] = 0;
            done[i] = 1;
            snap[i] = 3;
        } else {
            lam[i] = dmin[i];
            done[i] = ni <= 2;
            snap[i] = 1;
        }
    }
}

// side of the graphs with snap = 3: outside the component of their first vertex
__global__ void k_bg_side_comp(uint8_t* side, const int32_t* parent, const int32_t* inst0, const int32_t* ioff,
                               const uint8_t* snap, int32_t N0) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N0; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = inst0[v];
        if (snap[i] == 3) side[v] = parent[v] != parent[ioff[i]];
    }
}

// CAPFOREST results: a smaller alpha (a cut of its scanned prefix) lowers
// the graph's bound; the prefix becomes the side (snap = 2)
__global__ void k_bg_alpha(const int64_t* alpha, const uint8_t* done, int32_t k, int64_t* lam, uint8_t* snap) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x)
        if (!done[i] && alpha[i] < lam[i]) {
            lam[i] = alpha[i];
            snap[i] = 2;
        }
}

// inpref[v] = val for the first alpha_len[i] scanned vertices of graphs with
// snap = 2 (order positions share the graphs' vertex ranges)
__global__ void k_bg_prefix(const int32_t* order, const int32_t* voff, const int32_t* vinst, const int32_t* alpha_len,
                            const uint8_t* snap, int32_t N, uint8_t* inpref, uint8_t val) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < N; q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = vinst[q];
        if (snap[i] == 2 && q - voff[i] < alpha_len[i]) inpref[order[q]] = val;
    }
}

// snapshot the side of graphs whose bound dropped this round: snap = 1:
// the vertex darg[i]; snap = 2: the marked prefix
__global__ void k_bg_side(uint8_t* side, const int32_t* map0, const int32_t* inst0, int32_t N0, const uint8_t* snap,
                          const int32_t* darg, const uint8_t* inpref) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N0; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = inst0[v];
        const uint8_t s = snap[i];
        if (s == 1) side[v] = map0[v] == darg[i];
        else if (s == 2) side[v] = inpref[map0[v]];
    }
}

__global__ void k_bg_clear_snap(uint8_t* snap, int32_t k) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) snap[i] = 0;
}

// graphs still in the rounds whose graph kept every vertex (no union this
// round) get the complete fallback pass; *cnt counts them
__global__ void k_bg_fallback(const int32_t* voff, const int32_t* voff2, const uint8_t* done, int32_t k,
                              uint8_t* prun, int32_t* cnt) {
    int32_t c = 0;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
        const bool need = !done[i] && voff2[i + 1] - voff2[i] == voff[i + 1] - voff[i];
        prun[i] = need;
        c += need;
    }
    c = wave_sum_i32(c);
    if (lane_id() == 0 && c) atomicAdd(cnt, c);
}

__global__ void k_bg_active(const uint8_t* done, int32_t k, uint8_t* prun) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) prun[i] = !done[i];
}

// after contraction: collapsed degrees bound each graph (while two or more
// of its vertices remain); graphs down to two vertices are done; *cnt
// counts the graphs still running
__global__ void k_bg_bound(const int32_t* voff2, const int64_t* dmin, int32_t k, int64_t* lam, uint8_t* done,
                           uint8_t* snap, int32_t* cnt) {
    int32_t c = 0;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
        if (done[i]) continue;
        const int32_t ni = voff2[i + 1] - voff2[i];
        if (ni >= 2 && dmin[i] < lam[i]) {
            lam[i] = dmin[i];
            snap[i] = 1;
        }
        if (ni <= 2) done[i] = 1;
        else c++;
    }
    c = wave_sum_i32(c);
    if (lane_id() == 0 && c) atomicAdd(cnt, c);
}

struct BatchWS {
    DevScalars* sc;
    int32_t* cnt;                  // [4] counters read by the host
    int32_t *voff, *voff2, *ioff, *eoff;
    BatchGraph* tab;
    int32_t *in_rp, *in_col;
    int64_t* in_w;
    DGraph g[3];
    int32_t *L, *parent, *flag, *map0, *vinst, *inst0;
    uint8_t *side, *inpref, *done, *snap, *prun;
    int64_t *lam, *dmin;
    int32_t* darg;
    ContractWS cw;
    Pr12WS prw;
    Pr34WS tw;
    PrivateArgs pv;
    unsigned long long* pmarks;
    unsigned long long* vpart;
};

void carve_batch(Arena& a, int32_t k, int32_t N, int64_t C, BatchWS& w) {
    w.sc = a.take<DevScalars>(1);
    w.cnt = a.take<int32_t>(4);
    w.voff = a.take<int32_t>((size_t)k + 1);
    w.voff2 = a.take<int32_t>((size_t)k + 1);
    w.ioff = a.take<int32_t>((size_t)k + 1);
    w.eoff = a.take<int32_t>((size_t)k + 1);
    w.tab = a.take<BatchGraph>((size_t)k);
    w.in_rp = a.take<int32_t>((size_t)N + 1);
    w.in_col = a.take<int32_t>((size_t)C + 1);
    w.in_w = a.take<int64_t>((size_t)C + 1);
    for (int q = 0; q < 3; q++) {
        DGraph& g = w.g[q];
        g.n = N;
        g.cap = C;
        g.off = a.take<int32_t>((size_t)N + 1);
        g.len = a.take<int32_t>((size_t)N + 1);
        g.col = a.take<int32_t>((size_t)C + 1);
        g.w = a.take<int64_t>((size_t)C + 1);
        g.deg = a.take<int64_t>((size_t)N + 1);
    }
    w.L = a.take<int32_t>((size_t)N + 1);
    w.parent = a.take<int32_t>((size_t)N + 1);
    w.flag = a.take<int32_t>((size_t)N + 2);
    w.map0 = a.take<int32_t>((size_t)N + 1);
    w.vinst = a.take<int32_t>((size_t)N + 1);
    w.inst0 = a.take<int32_t>((size_t)N + 1);
    w.side = a.take<uint8_t>((size_t)N + 1);
    w.inpref = a.take<uint8_t>((size_t)N + 1);
    w.done = a.take<uint8_t>((size_t)k + 1);
    w.snap = a.take<uint8_t>((size_t)k + 1);
    w.prun = a.take<uint8_t>((size_t)k + 1);
    w.lam = a.take<int64_t>((size_t)k + 1);
    w.dmin = a.take<int64_t>((size_t)k + 1);
    w.darg = a.take<int32_t>((size_t)k + 1);
    contract_ws_carve(a, N, C, w.cw);
    pr12_ws_carve(a, N, C, w.prw);
    pr34_ws_carve(a, N, w.tw);
    // CAPFOREST passes in instance mode: one set of per-vertex arrays
    PrivateArgs& pv = w.pv;
    pv = PrivateArgs{};
    pv.passes = k;
    pv.stride = N;
    pv.st = a.take<int32_t>((size_t)N + 1);
    pv.r = a.take<int64_t>((size_t)N + 1);
    pv.fifo = a.take<int32_t>((size_t)N + 1);
    pv.touched = a.take<int32_t>((size_t)N + 1);
    pv.order = a.take<int32_t>((size_t)N + 1);
    pv.stride1 = (int64_t)N / 64 + k + 2;
    pv.l1 = a.take<int64_t>((size_t)pv.stride1);
    pv.dlist = a.take<int32_t>((size_t)pv.stride1);
    pv.dbits = a.take<uint32_t>((size_t)N / 2048 + 2 * (size_t)k + 4);
    pv.nscan = a.take<int32_t>((size_t)k);
    pv.alpha = a.take<int64_t>((size_t)k);
    pv.alpha_len = a.take<int32_t>((size_t)k);
    pv.lam_out = a.take<int64_t>((size_t)k);
    w.pmarks = a.take<unsigned long long>((size_t)k);
    w.vpart = a.take<unsigned long long>(1024);
}

bool batch_sizes(int32_t k, const mc_csr* gs, int32_t& N, int64_t& C, int32_t& nmax) {
    int64_t n = 0, c = 0;
    nmax = 0;
    for (int32_t i = 0; i < k; i++) {
        n += gs[i].n;
        c += gs[i].nnz;
        nmax = std::max(nmax, gs[i].n);
    }
    if (n >= INT32_MAX / 2 || c >= INT32_MAX / 2) return false;
    N = (int32_t)n;
    C = c;
    return true;
}

}  // namespace

extern "C" mc_status mc_batch_workspace_size(const mc_ctx* c, int32_t k, const mc_csr* gs, size_t* bytes) {
    if (!c || !gs || !bytes || k <= 0) return mc_fail(MC_E_INVALID_ARG, "mc_batch_workspace_size: bad argument");
    int32_t N, nmax;
    int64_t C;
    if (!batch_sizes(k, gs, N, C, nmax)) return mc_fail(MC_E_OVERFLOW, "batch too large (vertices or entries >= 2^30)");
    Arena a;
    BatchWS w;
    carve_batch(a, k, N, C, w);
    *bytes = a.used + 256;
    return MC_OK;
}

#define BG_HIP(x) do { if ((x) != hipSuccess) return mc_fail(MC_E_DEVICE, #x); } while (0)
#define BG_OK(x) do { if (!(x)) return MC_E_DEVICE; } while (0)

extern "C" mc_status mc_mincut_batch(mc_ctx* c, int32_t k, const mc_csr* gs, void* dev_ws, size_t ws_bytes,
                                     int64_t* lambdas, uint8_t* const* sides, mc_status* per_graph) {
    if (!c || !gs || !lambdas || k <= 0 || !dev_ws) return mc_fail(MC_E_INVALID_ARG, "mc_mincut_batch: bad argument");
    const int32_t loc = gs[0].location;
    for (int32_t i = 0; i < k; i++) {
        if (gs[i].n < 2) return mc_fail(MC_E_INVALID_ARG, "mc_mincut_batch: every graph needs n >= 2");
        if (gs[i].location != loc || (loc != MC_HOST && loc != MC_DEVICE))
            return mc_fail(MC_E_INVALID_ARG, "mc_mincut_batch: all graphs must share one location");
        if (!gs[i].row_ptr || gs[i].nnz < 0 || (gs[i].nnz > 0 && (!gs[i].col || !gs[i].w)))
            return mc_fail(MC_E_INVALID_ARG, "mc_mincut_batch: bad CSR pointers");
    }
    int32_t N, nmax;
    int64_t C64;
    if (!batch_sizes(k, gs, N, C64, nmax)) return mc_fail(MC_E_OVERFLOW, "batch too large (vertices or entries >= 2^30)");
    const int32_t C = (int32_t)C64;
    Arena a;
    a.base = (char*)dev_ws;
    a.size = ws_bytes;
    BatchWS w;
    carve_batch(a, k, N, C, w);
    if (a.used > ws_bytes) return mc_fail(MC_E_INVALID_ARG, "mc_mincut_batch: workspace too small");
    if (hipSetDevice(c->device) != hipSuccess) return mc_fail(MC_E_DEVICE, "hipSetDevice failed");
    hipStream_t s = c->stream;
    auto readback = [&]() -> bool {
        return hipMemcpyAsync(c->hsc, w.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s) == hipSuccess &&
               hipStreamSynchronize(s) == hipSuccess;
    };
    std::vector<int32_t> hcnt(4);
    auto read_cnt = [&]() -> bool {
        return hipMemcpyAsync(hcnt.data(), w.cnt, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s) == hipSuccess &&
               hipStreamSynchronize(s) == hipSuccess;
    };

    // offsets and the union CSR
    std::vector<int32_t> voff(k + 1), eoff(k + 1);
    voff[0] = eoff[0] = 0;
    for (int32_t i = 0; i < k; i++) {
        voff[i + 1] = voff[i] + gs[i].n;
        eoff[i + 1] = eoff[i] + gs[i].nnz;
    }
    BG_HIP(hipMemcpyAsync(w.voff, voff.data(), sizeof(int32_t) * (k + 1), hipMemcpyHostToDevice, s));
    BG_HIP(hipMemcpyAsync(w.ioff, voff.data(), sizeof(int32_t) * (k + 1), hipMemcpyHostToDevice, s));
    BG_HIP(hipMemcpyAsync(w.eoff, eoff.data(), sizeof(int32_t) * (k + 1), hipMemcpyHostToDevice, s));
    BG_OK(fill_i32((int32_t*)w.sc, 0, sizeof(DevScalars) / 4, s));
    BG_OK(fill_i32(w.cnt, 0, 4, s));
    if (loc == MC_DEVICE) {
        std::vector<BatchGraph> tab(k);
        for (int32_t i = 0; i < k; i++) tab[i] = {gs[i].row_ptr, gs[i].col, gs[i].w, gs[i].n, gs[i].nnz};
        BG_HIP(hipMemcpyAsync(w.tab, tab.data(), sizeof(BatchGraph) * k, hipMemcpyHostToDevice, s));
        k_bg_gather<<<grid_for((int64_t)C + N + 1, 256), 256, 0, s>>>(w.tab, k, w.voff, w.eoff, N, C, w.in_rp, w.in_col,
                                                                     w.in_w, w.sc);
        BG_OK(mc_hip_ok(hipGetLastError(), "k_bg_gather"));
    } else {
        for (int32_t i = 0; i < k; i++) {
            // host checks of each graph (row_ptr, targets in range, weights)
            const mc_csr& g = gs[i];
            if (g.row_ptr[0] != 0 || g.row_ptr[g.n] != g.nnz) return mc_fail(MC_E_BAD_GRAPH, "malformed row_ptr");
            for (int32_t v = 0; v < g.n; v++)
                if (g.row_ptr[v + 1] < g.row_ptr[v]) return mc_fail(MC_E_BAD_GRAPH, "row_ptr not monotone");
            for (int32_t j = 0; j < g.nnz; j++)
                if (g.col[j] < 0 || g.col[j] >= g.n || g.w[j] < 0) return mc_fail(MC_E_BAD_GRAPH, "bad entry");
            BG_HIP(hipMemcpyAsync(w.in_rp + voff[i], g.row_ptr, sizeof(int32_t) * g.n, hipMemcpyHostToDevice, s));
            if (g.nnz > 0) {
                BG_HIP(hipMemcpyAsync(w.in_col + eoff[i], g.col, sizeof(int32_t) * g.nnz, hipMemcpyHostToDevice, s));
                BG_HIP(hipMemcpyAsync(w.in_w + eoff[i], g.w, sizeof(int64_t) * g.nnz, hipMemcpyHostToDevice, s));
            }
        }
        k_bg_shift<<<grid_for((int64_t)C + N + 1, 256), 256, 0, s>>>(k, w.voff, w.eoff, N, C, w.in_rp, w.in_col);
        BG_OK(mc_hip_ok(hipGetLastError(), "k_bg_shift"));
    }
    // total weight (2^62 limit) over the union
    BG_OK(validate_csr(w.in_rp, w.in_col, w.in_w, N, C, w.sc, w.vpart, s));
    if (!readback()) return mc_fail(MC_E_DEVICE, "readback failed");
    if (c->hsc->err) return mc_fail((mc_status)c->hsc->err, "malformed graph in the batch");

    // normalise (in place when already normal)
    BG_OK(canon_check(w.in_rp, w.in_col, w.in_w, N, w.g[0].len, w.g[0].deg, &w.sc->noncanon, s));
    if (!readback()) return mc_fail(MC_E_DEVICE, "readback failed");
    if (c->hsc->noncanon == 0) {
        w.g[0].off = w.in_rp;
        w.g[0].col = w.in_col;
        w.g[0].w = w.in_w;
    } else {
        DGraph user = w.g[1];
        user.n = N;
        user.cap = C;
        user.col = w.in_col;
        user.w = w.in_w;
        BG_OK(csr_to_padded(w.in_rp, N, user.off, user.len, s));
        BG_OK(contract(user, nullptr, N, w.g[0], w.cw, w.sc, s));
    }
    BG_OK(iota_i32(w.map0, N, s));
    k_bg_vinst<<<grid_for(N, 256), 256, 0, s>>>(w.voff, k, N, w.inst0);
    BG_OK(mc_hip_ok(hipGetLastError(), "k_bg_vinst"));
    {
        PrivateArgs one = w.pv;   // st and r: one vertex-indexed array for all passes
        one.passes = 1;
        BG_OK(capforest_private_reset(one, s));
    }
    // per-graph connectivity and minimum degree
    BG_OK(uf_init(w.parent, N, s));
    BG_OK(uf_connectivity(w.g[0], w.parent, (int32_t*)w.vpart, s));
    BG_OK(uf_labels(w.parent, N, w.L, w.flag, w.cw.scan_tmp, w.sc, s));
    k_bg_offsets<<<grid_for(k + 1, 256), 256, 0, s>>>(w.flag, w.voff, k, w.voff2);
    k_bg_segmin<<<std::min(k, 8192), 256, 0, s>>>(w.g[0].deg, w.voff, k, w.dmin, w.darg);
    k_bg_start<<<grid_for(k, 256), 256, 0, s>>>(w.voff, w.voff2, k, w.dmin, w.lam, w.done, w.snap);
    k_bg_side_comp<<<grid_for(N, 256), 256, 0, s>>>(w.side, w.parent, w.inst0, w.ioff, w.snap, N);
    k_bg_side<<<grid_for(N, 256), 256, 0, s>>>(w.side, w.map0, w.inst0, N, w.snap, w.darg, w.inpref);
    k_bg_clear_snap<<<grid_for(k, 256), 256, 0, s>>>(w.snap, k);
    BG_OK(mc_hip_ok(hipGetLastError(), "batch start"));
    BG_OK(fill_u8(w.inpref, 0, N, s));

    const int32_t len_cap = c->opt.pass_len_cap > 0 ? c->opt.pass_len_cap : (c->opt.pass_len_cap < 0 ? 0 : 32768);
    const int32_t D = c->opt.pr_tri_deg_cap;
    bool tri_on = D > 0;
    DGraph* cur = &w.g[0];
    int nxt_idx = 1;
    int32_t* voff_d = w.voff;
    int32_t* voff2_d = w.voff2;
    for (int32_t round = 0;; round++) {
        if (round > N + 64) return mc_fail(MC_E_DEVICE, "mc_mincut_batch: no progress");
        DGraph* nxt = &w.g[nxt_idx];
        const int32_t n = cur->n;
        BG_OK(fill_i32(w.cnt, 0, 4, s));
        // marks counters of the round
        BG_OK(fill_i64((int64_t*)&w.sc->marks_pr, 0, 3, s));
        BG_OK(uf_init(w.parent, n, s));
        k_bg_vinst<<<grid_for(n, 256), 256, 0, s>>>(voff_d, k, n, w.vinst);
        BG_OK(mc_hip_ok(hipGetLastError(), "k_bg_vinst"));
        // reduction tests with each graph's own bound
        BG_OK(pr12(*cur, w.lam, w.parent, &w.sc->marks_pr, nullptr, tri_on ? w.tw.ptr2 : nullptr, w.prw, s, w.vinst));
        if (tri_on) BG_OK(pr34(*cur, w.lam, D, w.parent, &w.sc->marks_tri, w.tw.ptr2, w.tw, nullptr, nullptr, s, w.vinst));
        // one CAPFOREST pass per graph still in the rounds
        k_bg_active<<<grid_for(k, 256), 256, 0, s>>>(w.done, k, w.prun);
        PrivateArgs pa = w.pv;
        pa.g = *cur;
        pa.lam = w.lam;
        pa.parent = w.parent;
        pa.len_cap = len_cap;
        pa.seed = c->opt.seed;
        pa.round = round;
        pa.start = -1;
        pa.marks = &w.sc->marks_cf;
        pa.steps = nullptr;
        pa.diag = nullptr;
        pa.pvoff = voff_d;
        pa.plam = w.lam;
        pa.prun = w.prun;
        pa.pmarks = w.pmarks;
        BG_OK(capforest_private(pa, s, nmax));
        k_bg_alpha<<<grid_for(k, 256), 256, 0, s>>>(pa.alpha, w.done, k, w.lam, w.snap);
        BG_OK(uf_labels(w.parent, n, w.L, w.flag, w.cw.scan_tmp, w.sc, s));
        k_bg_offsets<<<grid_for(k + 1, 256), 256, 0, s>>>(w.flag, voff_d, k, voff2_d);
        k_bg_fallback<<<grid_for(k, 256), 256, 0, s>>>(voff_d, voff2_d, w.done, k, w.prun, w.cnt);
        BG_OK(mc_hip_ok(hipGetLastError(), "batch round"));
        if (!read_cnt()) return mc_fail(MC_E_DEVICE, "readback failed");
        if (tri_on && !readback()) return mc_fail(MC_E_DEVICE, "readback failed");
        if (tri_on && c->hsc->marks_tri * 100 < (unsigned long long)n) tri_on = false;
        if (hcnt[0] > 0) {
            // Algorithm 2: graphs without a contractible edge get one complete
            // pass (with a fixed bound it marks an edge, else the bound drops)
            // first record the truncated passes' prefixes (their alpha may
            // have lowered the bound)
            k_bg_prefix<<<grid_for(n, 256), 256, 0, s>>>(pa.order, voff_d, w.vinst, pa.alpha_len, w.snap, n, w.inpref, 1);
            k_bg_side<<<grid_for(N, 256), 256, 0, s>>>(w.side, w.map0, w.inst0, N, w.snap, w.darg, w.inpref);
            k_bg_prefix<<<grid_for(n, 256), 256, 0, s>>>(pa.order, voff_d, w.vinst, pa.alpha_len, w.snap, n, w.inpref, 0);
            k_bg_clear_snap<<<grid_for(k, 256), 256, 0, s>>>(w.snap, k);
            PrivateArgs pf = pa;
            pf.len_cap = 0;
            pf.round = round + 7777;
            BG_OK(capforest_private(pf, s, nmax));
            k_bg_alpha<<<grid_for(k, 256), 256, 0, s>>>(pf.alpha, w.done, k, w.lam, w.snap);
            BG_OK(uf_labels(w.parent, n, w.L, w.flag, w.cw.scan_tmp, w.sc, s));
            k_bg_offsets<<<grid_for(k + 1, 256), 256, 0, s>>>(w.flag, voff_d, k, voff2_d);
            BG_OK(mc_hip_ok(hipGetLastError(), "batch fallback"));
        }
        // sides of graphs whose bound dropped to a pass's prefix
        k_bg_prefix<<<grid_for(n, 256), 256, 0, s>>>(pa.order, voff_d, w.vinst, pa.alpha_len, w.snap, n, w.inpref, 1);
        k_bg_side<<<grid_for(N, 256), 256, 0, s>>>(w.side, w.map0, w.inst0, N, w.snap, w.darg, w.inpref);
        k_bg_prefix<<<grid_for(n, 256), 256, 0, s>>>(pa.order, voff_d, w.vinst, pa.alpha_len, w.snap, n, w.inpref, 0);
        k_bg_clear_snap<<<grid_for(k, 256), 256, 0, s>>>(w.snap, k);
        if (!readback()) return mc_fail(MC_E_DEVICE, "readback failed");
        const int32_t n2 = c->hsc->n2;
        // contraction of the union graph, collapsed degrees per graph
        BG_OK(contract(*cur, w.L, n2, *nxt, w.cw, w.sc, s));
        BG_OK(map_update(w.map0, w.L, N, s));
        k_bg_segmin<<<std::min(k, 8192), 256, 0, s>>>(nxt->deg, voff2_d, k, w.dmin, w.darg);
        BG_OK(fill_i32(w.cnt, 0, 4, s));
        k_bg_bound<<<grid_for(k, 256), 256, 0, s>>>(voff2_d, w.dmin, k, w.lam, w.done, w.snap, w.cnt);
        k_bg_side<<<grid_for(N, 256), 256, 0, s>>>(w.side, w.map0, w.inst0, N, w.snap, w.darg, w.inpref);
        k_bg_clear_snap<<<grid_for(k, 256), 256, 0, s>>>(w.snap, k);
        BG_OK(mc_hip_ok(hipGetLastError(), "batch bound"));
        if (!read_cnt()) return mc_fail(MC_E_DEVICE, "readback failed");
        std::swap(voff_d, voff2_d);
        cur = nxt;
        nxt_idx = nxt_idx == 1 ? 2 : 1;
        if (hcnt[0] == 0) break;
    }
    // results
    BG_HIP(hipMemcpyAsync(lambdas, w.lam, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s));
    std::vector<uint8_t> hside;
    if (sides) {
        hside.resize(N);
        BG_HIP(hipMemcpyAsync(hside.data(), w.side, N, hipMemcpyDeviceToHost, s));
    }
    BG_HIP(hipStreamSynchronize(s));
    for (int32_t i = 0; i < k; i++) {
        if (per_graph) per_graph[i] = MC_OK;
        if (sides && sides[i]) {
            const uint8_t flip = hside[voff[i]];
            for (int32_t v = 0; v < gs[i].n; v++) sides[i][v] = hside[voff[i] + v] ^ flip;
        }
    }
    return MC_OK;
}
