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
// label-propagation heuristic coarsens every graph at admission and bounds
// its lambda with the collapsed degrees it meets (the bound only changes the
// work, not the result).
#include <algorithm>
#include <chrono>
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

// Per-graph checks of device inputs (what check_host_csr does on the host,
// without the symmetry check), one workgroup per graph at a time:
// row_ptr[0] = 0, row_ptr[n] = nnz and non-decreasing, every target in
// [0, n) and every weight >= 0 (MC_E_BAD_GRAPH), then the graph's own total
// weight below 2^62 (MC_E_OVERFLOW). gerr[i] receives graph i's status.
constexpr unsigned long long BG_WCAP = 1ULL << 62;
__global__ __launch_bounds__(256) void k_bg_check(const BatchGraph* tab, int32_t k, int32_t* gerr) {
    __shared__ unsigned long long ssum[256];
    __shared__ int32_t sbad;
    for (int32_t i = blockIdx.x; i < k; i += gridDim.x) {
        const BatchGraph g = tab[i];
        if (threadIdx.x == 0) sbad = 0;
        __syncthreads();
        bool bad = threadIdx.x == 0 && (g.rp[0] != 0 || g.rp[g.n] != g.nnz);
        for (int32_t v = threadIdx.x; v < g.n; v += blockDim.x)
            if (g.rp[v + 1] < g.rp[v]) bad = true;
        unsigned long long sum = 0;
        for (int32_t j = threadIdx.x; j < g.nnz; j += blockDim.x) {
            const int32_t x = g.col[j];
            const int64_t c = g.w[j];
            if (x < 0 || x >= g.n || c < 0) {
                bad = true;
            } else {
                // sum < 2^62 and c < 2^63 before the add: no wrap
                sum += (unsigned long long)c;
                if (sum >= BG_WCAP) sum = BG_WCAP;
            }
        }
        if (bad) sbad = 1;
        ssum[threadIdx.x] = sum;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) {
                const unsigned long long t = ssum[threadIdx.x] + ssum[threadIdx.x + o];
                ssum[threadIdx.x] = t >= BG_WCAP ? BG_WCAP : t;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) gerr[i] = sbad ? MC_E_BAD_GRAPH : (ssum[0] >= BG_WCAP ? MC_E_OVERFLOW : MC_OK);
        __syncthreads();
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

// the largest total degree of one graph (its vertex range voff[i] ..
// voff[i+1]) into sc->gmax: every degree of any contraction of the batch is
// below it, since a cluster lies inside one graph
__global__ __launch_bounds__(256) void k_bg_wmax(const int64_t* deg, const int32_t* voff, int32_t k,
                                                DevScalars* sc) {
    __shared__ int64_t ss[4];
    for (int32_t i = blockIdx.x; i < k; i += gridDim.x) {
        int64_t t = 0;
        for (int32_t v = voff[i] + threadIdx.x; v < voff[i + 1]; v += 256) t += deg[v];
        t = wave_sum_i64(t);
        __syncthreads();
        if (lane_id() == 0) ss[threadIdx.x / MC_WAVE] = t;
        __syncthreads();
        if (threadIdx.x == 0)
            atomicMax((unsigned long long*)&sc->gmax, (unsigned long long)(ss[0] + ss[1] + ss[2] + ss[3]));
    }
}

// voff2[i] = number of component roots before voff[i] (scan of root flags)
__global__ void k_bg_offsets(const int32_t* scan, const int32_t* voff, int32_t k, int32_t* voff2) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= k; i += gridDim.x * blockDim.x)
        voff2[i] = scan[voff[i]];
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
// the vertex darg[i]; snap = 2: the marked prefix; snap = 3: the cut the
// finisher found (fside over the current vertices)
__global__ void k_bg_side(uint8_t* side, const int32_t* map0, const int32_t* inst0, int32_t N0, const uint8_t* snap,
                          const int32_t* darg, const uint8_t* inpref, const uint8_t* fside) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N0; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t m = map0[v];
        if (m < 0) continue;                      // input vertex no longer tracked
        const int32_t i = inst0[v];
        const uint8_t s = snap[i];
        if (s == 1) side[v] = m == darg[i];
        else if (s == 2) side[v] = inpref[m];
        else if (s == 3) side[v] = fside[m];      // the finisher's best cut
    }
}

// graphs the finisher completed with a lower bound take its cut as side
__global__ void k_bg_fin_snap(const int32_t* flist, int32_t cnt, const int32_t* fdrop, uint8_t* snap) {
    for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < cnt; q += gridDim.x * blockDim.x) {
        const int32_t i = flist[q];
        if (fdrop[i]) snap[i] = 3;
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
        if (ni <= 2 || lam[i] == 0) done[i] = 1;   // nothing lower than 0
        else c++;
    }
    c = wave_sum_i32(c);
    if (lane_id() == 0 && c) atomicAdd(cnt, c);
}

// ----------------------------------------------------------- the engine
// Labels of a round with dropped graphs: roots of live graphs are numbered
// in vertex order; every vertex of a graph marked dead gets -1, so the
// contraction removes it.
__global__ void k_root_flag_live(const int32_t* par, const int32_t* vinst, const uint8_t* dead, int32_t n,
                                 int32_t* flag) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        flag[v] = par[v] == v && !dead[vinst[v]];
}

__global__ void k_label_live(const int32_t* par, const int32_t* newid, const int32_t* vinst, const uint8_t* dead,
                             int32_t n, int32_t* L, DevScalars* sc) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        L[v] = dead[vinst[v]] ? -1 : newid[par[v]];
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->n2 = newid[n];
}

// Append the staged (normal-form) graphs S behind the current graph: vertex
// v of S becomes vbase + v, its row moves behind the current graph's last
// window (ebase).
__global__ void k_eg_append(DGraph S, int64_t s_entries, DGraph cur, int32_t vbase, int64_t ebase) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = tid; v < S.n; v += nth) {
        cur.off[vbase + v] = (int32_t)(S.off[v] + ebase);
        cur.len[vbase + v] = S.len[v];
        cur.deg[vbase + v] = S.deg[v];
    }
    for (int64_t e = tid; e < s_entries; e += nth) {
        cur.col[ebase + e] = S.col[e] + vbase;
        cur.w[ebase + e] = S.w[e];
    }
}

// input vertices of newly admitted graphs: map to their current vertex
__global__ void k_eg_admit_map(int32_t* map0, uint8_t* side, int32_t n0base, int32_t vbase, int32_t count) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < count; v += (int64_t)gridDim.x * blockDim.x) {
        map0[n0base + v] = vbase + (int32_t)v;
        side[n0base + v] = 0;
    }
}

// move the input-vertex ranges of the graphs still tracked to the front:
// position q of the new layout belongs to graph j (new offsets nio), whose
// old range started at oio[j]
__global__ void k_eg_n0_compact(const int32_t* nio, const int32_t* oio, int32_t k, int32_t used, const int32_t* map0,
                                const uint8_t* side, int32_t* map0b, uint8_t* sideb) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < used; q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = seg_of(nio, k, q);
        const int64_t old = oio[j] + (q - nio[j]);
        map0b[q] = map0[old];
        sideb[q] = side[old];
    }
}

__global__ void k_eg_untrack(int32_t* map0, int32_t from, int32_t count) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < count; v += (int64_t)gridDim.x * blockDim.x)
        map0[from + v] = -1;
}

// first-round bound of newly admitted graphs: minimum degree, side = its vertex
__global__ void k_eg_start(const int64_t* dmin, const int32_t* darg, int32_t k, int64_t* lam, uint8_t* snap) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
        lam[i] = dmin[i];
        snap[i] = 1;
    }
}

// The label-propagation heuristic of Section 2.1 ("Lowering the upper
// bound") on newly admitted graphs, all at once: label propagation, every
// cluster contracted to one vertex, and again on the coarse graphs, while
// they shrink. A collapsed vertex's degree is the capacity of the cut
// around the input vertices it stands for, so each level's smallest
// collapsed degree (while a graph still has two or more coarse vertices)
// bounds that graph's lambda, with those input vertices as the side.
// Clusters never join two graphs (no edge does), so the coarse vertices of
// each graph stay one contiguous range.
__global__ void k_eg_level_bound(const int32_t* coff2, const int64_t* dmin, int32_t k, int64_t* best, uint8_t* hit) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
        hit[i] = 0;
        if (coff2[i + 1] - coff2[i] >= 2 && dmin[i] < best[i]) {
            best[i] = dmin[i];
            hit[i] = 1;
        }
    }
}

// side of graphs whose bound dropped at this level: stage vertex v is on the
// side iff its coarse vertex is the graph's smallest-degree one
__global__ void k_eg_level_side(const int32_t* maps, const int32_t* inst_rel, const uint8_t* hit, const int32_t* darg,
                                int32_t ns, uint8_t* sideh) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < ns; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = inst_rel[v];
        if (hit[i]) sideh[v] = maps[v] == darg[i];
    }
}

// the heuristic's bound replaces the minimum degree where it is smaller
__global__ void k_eg_apply_heuristic(const int64_t* best, int32_t k, int64_t* lam, uint8_t* use) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
        use[i] = best[i] < lam[i];
        if (use[i]) lam[i] = best[i];
    }
}

__global__ void k_eg_side_heuristic(uint8_t* side, const int32_t* inst_rel, const uint8_t* use, const uint8_t* sideh,
                                    int32_t ns) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < ns; v += (int64_t)gridDim.x * blockDim.x)
        if (use[inst_rel[v]]) side[v] = sideh[v];
}

struct Caps {
    int32_t N = 0;        // vertices of the union graph
    int64_t C = 0;        // entry capacity of the union graph
    int32_t N0 = 0;       // input vertices tracked at once (sides)
    int32_t K = 0;        // graphs in the rounds at once
    int32_t Ns = 0;       // vertices staged by one admission
    int64_t Cs = 0;       // entries staged by one admission
    int32_t nmax = 0;     // largest graph (vertices)
};

struct EngineWS {
    DevScalars* sc;
    int32_t* cnt;
    int32_t *voff, *voff2, *ioff, *ioff2, *s_voff, *s_eoff;
    int64_t *lam, *dmin;
    int32_t* darg;
    uint8_t *done, *snap, *prun, *dead;
    int32_t* gstart_total;
    BatchGraph* tab;
    int32_t* gerr;            // [K] per-graph status of device-input checks
    int32_t *in_rp, *in_col;
    int64_t* in_w;
    DGraph g[3];
    DGraph stage;
    int32_t *L, *parent, *flag, *vinst, *inst0;
    uint8_t* inpref;
    int32_t *map0, *map0b;
    uint8_t *side, *sideb;
    ContractWS cw;
    Pr12WS prw;
    Pr34WS tw;
    LpWS lw;
    int32_t *h_lab, *h_map;   // [Ns] canonical cluster labels; stage vertex -> coarse vertex
    uint8_t* h_side;          // [Ns] side of the heuristic's best bound
    int32_t *h_off, *h_off2;  // [K+1] coarse ranges of the graphs
    int64_t *best, *h_dmin;   // [K]
    int32_t* h_darg;          // [K]
    uint8_t* h_hit;           // [K]
    PrivateArgs pv;
    unsigned long long* pmarks;
    unsigned long long* vpart;
    int32_t *flist, *fdrop, *frounds, *ferr;   // finisher: graphs, lowered bound, rounds, error and work-queue ticket
    uint8_t* fside;           // [N] the finisher's side over the current vertices
};

void carve_engine(Arena& a, const Caps& cp, EngineWS& w) {
    const int32_t N = cp.N, K = cp.K, Ns = cp.Ns;
    const int64_t C = cp.C, Cs = cp.Cs;
    w.sc = a.take<DevScalars>(1);
    w.cnt = a.take<int32_t>(4);
    w.voff = a.take<int32_t>((size_t)K + 1);
    w.voff2 = a.take<int32_t>((size_t)K + 1);
    w.ioff = a.take<int32_t>((size_t)K + 1);
    w.ioff2 = a.take<int32_t>((size_t)K + 1);
    w.s_voff = a.take<int32_t>((size_t)K + 1);
    w.s_eoff = a.take<int32_t>((size_t)K + 1);
    w.lam = a.take<int64_t>((size_t)K + 1);
    w.dmin = a.take<int64_t>((size_t)K + 1);
    w.darg = a.take<int32_t>((size_t)K + 1);
    w.done = a.take<uint8_t>((size_t)K + 1);
    w.snap = a.take<uint8_t>((size_t)K + 1);
    w.prun = a.take<uint8_t>((size_t)K + 1);
    w.dead = a.take<uint8_t>((size_t)K + 1);
    w.gstart_total = a.take<int32_t>(1);
    w.tab = a.take<BatchGraph>((size_t)K);
    w.gerr = a.take<int32_t>((size_t)K);
    w.in_rp = a.take<int32_t>((size_t)Ns + 1);
    w.in_col = a.take<int32_t>((size_t)Cs + 1);
    w.in_w = a.take<int64_t>((size_t)Cs + 1);
    auto graph = [&](DGraph& g, int32_t n, int64_t cap) {
        g.n = n;
        g.cap = cap;
        g.off = a.take<int32_t>((size_t)n + 1);
        g.len = a.take<int32_t>((size_t)n + 1);
        g.col = a.take<int32_t>((size_t)cap + 1);
        g.w = a.take<int64_t>((size_t)cap + 1);
        g.deg = a.take<int64_t>((size_t)n + 1);
    };
    for (int q = 0; q < 3; q++) graph(w.g[q], N, C);
    graph(w.stage, Ns, Cs);
    w.L = a.take<int32_t>((size_t)N + 1);
    w.parent = a.take<int32_t>((size_t)N + 1);
    w.flag = a.take<int32_t>((size_t)std::max(N, Ns) + 2);
    w.vinst = a.take<int32_t>((size_t)N + 1);
    w.inst0 = a.take<int32_t>((size_t)cp.N0 + 1);
    w.inpref = a.take<uint8_t>((size_t)N + 1);
    w.map0 = a.take<int32_t>((size_t)cp.N0 + 1);
    w.map0b = a.take<int32_t>((size_t)cp.N0 + 1);
    w.side = a.take<uint8_t>((size_t)cp.N0 + 1);
    w.sideb = a.take<uint8_t>((size_t)cp.N0 + 1);
    contract_ws_carve(a, std::max(N, Ns), std::max(C, Cs), w.cw);
    pr12_ws_carve(a, N, C, w.prw);
    pr34_ws_carve(a, N, w.tw);
    lp_ws_carve(a, Ns, Cs, w.lw);
    w.h_lab = a.take<int32_t>((size_t)Ns + 1);
    w.h_map = a.take<int32_t>((size_t)Ns + 1);
    w.h_side = a.take<uint8_t>((size_t)Ns + 1);
    w.h_off = a.take<int32_t>((size_t)K + 1);
    w.h_off2 = a.take<int32_t>((size_t)K + 1);
    w.best = a.take<int64_t>((size_t)K + 1);
    w.h_dmin = a.take<int64_t>((size_t)K + 1);
    w.h_darg = a.take<int32_t>((size_t)K + 1);
    w.h_hit = a.take<uint8_t>((size_t)K + 1);
    PrivateArgs& pv = w.pv;
    pv = PrivateArgs{};
    pv.passes = K;
    pv.stride = N;
    pv.st = a.take<int32_t>((size_t)N + 1);
    pv.r = a.take<int64_t>((size_t)N + 1);
    pv.fifo = a.take<int32_t>((size_t)N + 1);
    pv.touched = a.take<int32_t>((size_t)N + 1);
    pv.order = a.take<int32_t>((size_t)N + 1);
    pv.stride1 = (int64_t)N / 64 + K + 2;
    pv.l1 = a.take<int64_t>((size_t)pv.stride1);
    pv.dlist = a.take<int32_t>((size_t)pv.stride1);
    pv.dbits = a.take<uint32_t>((size_t)N / 2048 + 2 * (size_t)K + 4);
    pv.nscan = a.take<int32_t>((size_t)K);
    pv.alpha = a.take<int64_t>((size_t)K);
    pv.alpha_len = a.take<int32_t>((size_t)K);
    pv.lam_out = a.take<int64_t>((size_t)K);
    w.pmarks = a.take<unsigned long long>((size_t)K);
    w.vpart = a.take<unsigned long long>(1024);
    w.flist = a.take<int32_t>((size_t)K + 1);
    w.fdrop = a.take<int32_t>((size_t)K + 1);
    w.frounds = a.take<int32_t>((size_t)K + 1);
    w.ferr = a.take<int32_t>(4);
    w.fside = a.take<uint8_t>((size_t)N + 1);
}

#define EG_HIP(x) do { if ((x) != hipSuccess) return mc_fail(MC_E_DEVICE, #x); } while (0)
#define EG_OK(x) do { if (!(x)) return MC_E_DEVICE; } while (0)

}  // namespace

// One graph in the rounds.
struct EngineInst {
    uint64_t id = 0;
    int32_t n0 = 0;           // input vertices
    int32_t ioff = 0;         // start of its input vertices in the side arrays
    int32_t voff = 0, nv = 0; // its vertex range in the current union graph
    int64_t lam = 0;
    bool done = false;        // at most two vertices left (or lambda = 0): result final
    bool dead = false;        // result taken; its vertices leave in the next contraction
    int32_t rounds = 0;
};

// The round engine shared by the batched and the served forms: a union
// graph of independent graphs, admitted at round boundaries, that all move
// through the rounds of Algorithm 2 together.
struct Engine {
    mc_ctx* c = nullptr;
    hipStream_t s = nullptr;
    Caps cap;
    EngineWS w{};
    int cur = 0;                  // index of the current graph in w.g
    int32_t n = 0;                // its vertices
    int64_t used = 0;             // entries up to its last row window
    int32_t n0_used = 0;
    std::vector<EngineInst> insts;
    bool tri_on = true;
    int32_t round = 0;

    mc_status init(mc_ctx* ctx, const Caps& cp, void* ws, size_t bytes) {
        c = ctx;
        s = ctx->stream;
        cap = cp;
        Arena a;
        a.base = (char*)ws;
        a.size = bytes;
        carve_engine(a, cp, w);
        if (a.used > bytes) return mc_fail(MC_E_INVALID_ARG, "engine: workspace too small");
        if (hipSetDevice(c->device) != hipSuccess) return mc_fail(MC_E_DEVICE, "hipSetDevice failed");
        PrivateArgs one = w.pv;   // st and r: one vertex-indexed array for all passes
        one.passes = 1;
        EG_OK(capforest_private_reset(one, s));
        EG_OK(fill_i32((int32_t*)w.sc, 0, sizeof(DevScalars) / 4, s));
        // prefix marks are set and cleared per round; they start all zero
        EG_OK(fill_u8(w.inpref, 0, (int64_t)cp.N + 1, s));
        tri_on = c->opt.pr_tri_deg_cap > 0;
        cur = 0;
        n = 0;
        used = 0;
        n0_used = 0;
        insts.clear();
        return MC_OK;
    }

    bool readback() {
        return hipMemcpyAsync(c->hsc, w.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s) == hipSuccess &&
               hipStreamSynchronize(s) == hipSuccess;
    }

    // Room for k more graphs of nv vertices and ne entries in total?
    bool fits(int32_t k, int64_t nv, int64_t ne) const {
        int32_t live0 = 0;
        for (const EngineInst& x : insts) live0 += x.dead ? 0 : x.n0;
        return (int64_t)insts.size() + k <= cap.K && n + nv <= cap.N && used + ne <= cap.C && nv <= cap.Ns &&
               ne <= cap.Cs && live0 + nv <= cap.N0;
    }

    // Append graphs (normalised on the way) behind the current graph. Every
    // graph must already have passed its own checks (check_host_csr for
    // host graphs, check_device for device graphs): admission relies on
    // them and checks only sizes and capacity.
    mc_status admit(const mc_csr* gs, int32_t k, const uint64_t* ids) {
        if (k <= 0) return MC_OK;
        const int32_t loc = gs[0].location;
        int64_t nv = 0, ne = 0;
        std::vector<int32_t> sv(k + 1), se(k + 1);
        sv[0] = se[0] = 0;
        for (int32_t i = 0; i < k; i++) {
            const mc_csr& g = gs[i];
            if (g.n < 2) return mc_fail(MC_E_INVALID_ARG, "every graph needs n >= 2");
            if (g.location != loc || (loc != MC_HOST && loc != MC_DEVICE))
                return mc_fail(MC_E_INVALID_ARG, "all graphs of one call must share one location");
            if (!g.row_ptr || g.nnz < 0 || (g.nnz > 0 && (!g.col || !g.w)))
                return mc_fail(MC_E_INVALID_ARG, "bad CSR pointers");
            if (g.n > cap.nmax) return mc_fail(MC_E_OOM, "graph larger than the engine's largest graph");
            sv[i + 1] = sv[i] + g.n;
            se[i + 1] = se[i] + g.nnz;
            nv += g.n;
            ne += g.nnz;
        }
        if (!fits(k, nv, ne)) return mc_fail(MC_E_OOM, "the graphs do not fit the engine's capacity");
        if (n0_used + nv > cap.N0) {
            // input-vertex ranges of finished graphs leave holes: close them
            if (!compact_n0()) return MC_E_DEVICE;
            if (n0_used + nv > cap.N0) return mc_fail(MC_E_OOM, "the graphs do not fit the engine's capacity");
        }
        const int32_t NS = (int32_t)nv, CS = (int32_t)ne;
        EG_HIP(hipMemcpyAsync(w.s_voff, sv.data(), sizeof(int32_t) * (k + 1), hipMemcpyHostToDevice, s));
        EG_HIP(hipMemcpyAsync(w.s_eoff, se.data(), sizeof(int32_t) * (k + 1), hipMemcpyHostToDevice, s));
        EG_OK(fill_i32(&w.sc->err, 0, 1, s));
        if (loc == MC_DEVICE) {
            std::vector<BatchGraph> tab(k);
            for (int32_t i = 0; i < k; i++) tab[i] = {gs[i].row_ptr, gs[i].col, gs[i].w, gs[i].n, gs[i].nnz};
            EG_HIP(hipMemcpyAsync(w.tab, tab.data(), sizeof(BatchGraph) * k, hipMemcpyHostToDevice, s));
            k_bg_gather<<<grid_for((int64_t)CS + NS + 1, 256), 256, 0, s>>>(w.tab, k, w.s_voff, w.s_eoff, NS, CS,
                                                                           w.in_rp, w.in_col, w.in_w, w.sc);
            EG_OK(mc_hip_ok(hipGetLastError(), "k_bg_gather"));
        } else {
            for (int32_t i = 0; i < k; i++) {
                const mc_csr& g = gs[i];
                EG_HIP(hipMemcpyAsync(w.in_rp + sv[i], g.row_ptr, sizeof(int32_t) * g.n, hipMemcpyHostToDevice, s));
                if (g.nnz > 0) {
                    EG_HIP(hipMemcpyAsync(w.in_col + se[i], g.col, sizeof(int32_t) * g.nnz, hipMemcpyHostToDevice, s));
                    EG_HIP(hipMemcpyAsync(w.in_w + se[i], g.w, sizeof(int64_t) * g.nnz, hipMemcpyHostToDevice, s));
                }
            }
            k_bg_shift<<<grid_for((int64_t)CS + NS + 1, 256), 256, 0, s>>>(k, w.s_voff, w.s_eoff, NS, CS, w.in_rp,
                                                                          w.in_col);
            EG_OK(mc_hip_ok(hipGetLastError(), "k_bg_shift"));
        }
        if (loc == MC_DEVICE) {
            // the gather repeats the structural checks of k_bg_check; the
            // graphs were checked before admission, so this only catches
            // inputs changed in between
            if (!readback()) return mc_fail(MC_E_DEVICE, "readback failed");
            if (c->hsc->err) return mc_fail((mc_status)c->hsc->err, "malformed graph");
        }
        // normal form: in place when already normal, else contraction by
        // the identity into the staging graph
        DGraph S = w.stage;
        S.n = NS;
        S.cap = CS;
        EG_OK(canon_check(w.in_rp, w.in_col, w.in_w, NS, 0, w.stage.len, w.stage.deg, &w.sc->noncanon, nullptr, nullptr, nullptr, s));
        // the largest graph's total degree (of the input rows, loops and
        // parallel entries counted: an upper bound) decides whether the
        // label-propagation rounds may keep 32-bit sums
        EG_OK(fill_i64(&w.sc->gmax, 0, 1, s));
        k_bg_wmax<<<std::min(k, 8192), 256, 0, s>>>(w.stage.deg, w.s_voff, k, w.sc);
        EG_OK(mc_hip_ok(hipGetLastError(), "k_bg_wmax"));
        if (!readback()) return mc_fail(MC_E_DEVICE, "readback failed");
        const bool narrow = c->hsc->gmax < ((int64_t)1 << 32);
        if (c->hsc->noncanon == 0) {
            S.off = w.in_rp;
            S.col = w.in_col;
            S.w = w.in_w;
        } else {
            DGraph user = w.g[(cur + 1) % 3];   // its off/len arrays serve as scratch
            user.n = NS;
            user.cap = CS;
            user.col = w.in_col;
            user.w = w.in_w;
            EG_OK(csr_to_padded(w.in_rp, NS, user.off, user.len, s));
            EG_OK(contract(user, nullptr, NS, S, w.cw, w.sc, s));
        }
        // the label-propagation heuristic on the staged graphs (every graph
        // at once); its best bounds are applied after the minimum degrees
        const bool lp = c->opt.batch_lp == 1 || (c->opt.batch_lp == 0 && c->opt.heuristic_min_n > 0);
        if (lp) EG_OK(heuristic_levels(S, k, NS, sv, narrow));
        DGraph& G = w.g[cur];
        k_eg_append<<<grid_for((int64_t)CS + NS, 256), 256, 0, s>>>(S, CS, G, n, used);
        EG_OK(mc_hip_ok(hipGetLastError(), "k_eg_append"));
        k_eg_admit_map<<<grid_for(NS, 256), 256, 0, s>>>(w.map0, w.side, n0_used, n, NS);
        EG_OK(mc_hip_ok(hipGetLastError(), "k_eg_admit_map"));
        // first bounds: minimum degrees of the new ranges, and their vertices as sides
        std::vector<int32_t> vo(k + 1);
        for (int32_t i = 0; i <= k; i++) vo[i] = n + sv[i];
        EG_HIP(hipMemcpyAsync(w.voff, vo.data(), sizeof(int32_t) * (k + 1), hipMemcpyHostToDevice, s));
        k_bg_segmin<<<std::min(k, 8192), 256, 0, s>>>(G.deg, w.voff, k, w.dmin, w.darg);
        k_eg_start<<<grid_for(k, 256), 256, 0, s>>>(w.dmin, w.darg, k, w.lam, w.snap);
        // graph index (among the k new graphs) of each new input vertex; the
        // rounds recompute it for the whole table
        k_bg_vinst<<<grid_for(NS, 256), 256, 0, s>>>(w.s_voff, k, NS, w.inst0 + n0_used);
        EG_OK(mc_hip_ok(hipGetLastError(), "admit bounds"));
        k_bg_side<<<grid_for(NS, 256), 256, 0, s>>>(w.side + n0_used, w.map0 + n0_used, w.inst0 + n0_used, NS, w.snap,
                                                    w.darg, w.inpref, w.fside);
        k_bg_clear_snap<<<grid_for(k, 256), 256, 0, s>>>(w.snap, k);
        if (lp) {
            k_eg_apply_heuristic<<<grid_for(k, 256), 256, 0, s>>>(w.best, k, w.lam, w.h_hit);
            k_eg_side_heuristic<<<grid_for(NS, 256), 256, 0, s>>>(w.side + n0_used, w.inst0 + n0_used, w.h_hit,
                                                                  w.h_side, NS);
        }
        EG_OK(mc_hip_ok(hipGetLastError(), "admit sides"));
        std::vector<int64_t> lam(k);
        EG_HIP(hipMemcpyAsync(lam.data(), w.lam, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s));
        EG_HIP(hipStreamSynchronize(s));
        for (int32_t i = 0; i < k; i++) {
            EngineInst x;
            x.id = ids ? ids[i] : (uint64_t)i;
            x.n0 = gs[i].n;
            x.ioff = n0_used + sv[i];
            x.voff = n + sv[i];
            x.nv = gs[i].n;
            x.lam = lam[i];
            x.done = x.nv <= 2 || x.lam == 0;
            insts.push_back(x);
        }
        n += NS;
        used += CS;
        n0_used += NS;
        return MC_OK;
    }

    // Multi-level label propagation on the staged graphs S (k graphs, NS
    // vertices, ranges sv): w.best receives each graph's best collapsed
    // degree and w.h_side the matching side. The coarse graphs live in the
    // two union-graph buffers that are not current.
    bool heuristic_levels(const DGraph& S, int32_t k, int32_t NS, const std::vector<int32_t>& sv, bool narrow) {
        const int iters = c->opt.lp_iters > 0 ? c->opt.lp_iters : 2;
        if (!fill_i64(w.best, INT64_MAX, k, s) || !fill_u8(w.h_side, 0, NS, s) || !iota_i32(w.h_map, NS, s))
            return false;
        MC_HIP(hipMemcpyAsync(w.h_off, sv.data(), sizeof(int32_t) * (k + 1), hipMemcpyHostToDevice, s));
        // graph index of every stage vertex (relative ranges)
        k_bg_vinst<<<grid_for(NS, 256), 256, 0, s>>>(w.s_voff, k, NS, w.vinst);
        MC_LAUNCHED("k_bg_vinst");
        DGraph Gc = S;
        int bi = (cur + 1) % 3;
        std::vector<int32_t> co(k + 1);
        for (int level = 0; level < 32; level++) {
            const int32_t nc = Gc.n;
            int32_t* la = w.parent;
            int32_t* lb = w.L;
            // the first round starts from singleton labels on a normal graph
            if (!lp_first(Gc, lb, w.lw, w.cw, s)) return false;
            std::swap(la, lb);
            for (int it = 1; it < iters; it++) {
                if (!lp_round(Gc, la, lb, w.lw, w.cw, s, narrow)) return false;
                std::swap(la, lb);
            }
            if (!lp_relabel(la, nc, w.h_lab, w.flag, w.cw.scan_tmp, w.sc, s)) return false;
            k_bg_offsets<<<grid_for(k + 1, 256), 256, 0, s>>>(w.flag, w.h_off, k, w.h_off2);
            MC_LAUNCHED("k_bg_offsets");
            if (!readback()) return false;
            const int32_t n2 = c->hsc->n2;
            if ((int64_t)n2 * 20 > (int64_t)nc * 19) break;   // shrank by less than 5 percent
            DGraph& Gn = w.g[bi];
            if (!contract(Gc, w.h_lab, n2, Gn, w.cw, w.sc, s) || !map_update(w.h_map, w.h_lab, NS, s)) return false;
            k_bg_segmin<<<std::min(k, 8192), 256, 0, s>>>(Gn.deg, w.h_off2, k, w.h_dmin, w.h_darg);
            k_eg_level_bound<<<grid_for(k, 256), 256, 0, s>>>(w.h_off2, w.h_dmin, k, w.best, w.h_hit);
            k_eg_level_side<<<grid_for(NS, 256), 256, 0, s>>>(w.h_map, w.vinst, w.h_hit, w.h_darg, NS, w.h_side);
            MC_LAUNCHED("heuristic level");
            std::swap(w.h_off, w.h_off2);
            Gc = Gn;
            bi = bi == (cur + 1) % 3 ? (cur + 2) % 3 : (cur + 1) % 3;
            // stop once no graph has more than two coarse vertices
            MC_HIP(hipMemcpyAsync(co.data(), w.h_off, sizeof(int32_t) * (k + 1), hipMemcpyDeviceToHost, s));
            MC_HIP(hipStreamSynchronize(s));
            bool more = false;
            for (int32_t i = 0; i < k && !more; i++) more = co[i + 1] - co[i] > 2;
            if (!more) break;
        }
        return true;
    }

    // Per-graph checks of k device graphs (check_host_csr's checks without
    // symmetry, on the device): st[i] receives graph i's status. Pointers and
    // n were checked on the host.
    mc_status check_device(const mc_csr* gs, int32_t k, mc_status* st) {
        if (k <= 0) return MC_OK;
        if (k > cap.K) return mc_fail(MC_E_INVALID_ARG, "engine: too many graphs to check");
        std::vector<BatchGraph> tab(k);
        for (int32_t i = 0; i < k; i++) tab[i] = {gs[i].row_ptr, gs[i].col, gs[i].w, gs[i].n, gs[i].nnz};
        std::vector<int32_t> e(k);
        EG_HIP(hipMemcpyAsync(w.tab, tab.data(), sizeof(BatchGraph) * k, hipMemcpyHostToDevice, s));
        k_bg_check<<<std::min(k, 4096), 256, 0, s>>>(w.tab, k, w.gerr);
        EG_OK(mc_hip_ok(hipGetLastError(), "k_bg_check"));
        EG_HIP(hipMemcpyAsync(e.data(), w.gerr, sizeof(int32_t) * k, hipMemcpyDeviceToHost, s));
        EG_HIP(hipStreamSynchronize(s));
        for (int32_t i = 0; i < k; i++) st[i] = (mc_status)e[i];
        return MC_OK;
    }

    // Move the input-vertex ranges of live graphs to the front.
    bool compact_n0() {
        const int32_t k = (int32_t)insts.size();
        if (k == 0) { n0_used = 0; return true; }
        std::vector<int32_t> nio(k + 1), oio(k + 1);
        int32_t run = 0;
        for (int32_t i = 0; i < k; i++) {
            oio[i] = insts[i].ioff;
            nio[i] = run;
            run += insts[i].n0;
        }
        nio[k] = oio[k] = run;
        if (hipMemcpyAsync(w.ioff, nio.data(), sizeof(int32_t) * (k + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(w.ioff2, oio.data(), sizeof(int32_t) * (k + 1), hipMemcpyHostToDevice, s) != hipSuccess)
            return false;
        k_eg_n0_compact<<<grid_for(run, 256), 256, 0, s>>>(w.ioff, w.ioff2, k, run, w.map0, w.side, w.map0b, w.sideb);
        if (!mc_hip_ok(hipGetLastError(), "k_eg_n0_compact")) return false;
        std::swap(w.map0, w.map0b);
        std::swap(w.side, w.sideb);
        for (int32_t i = 0; i < k; i++) insts[i].ioff = nio[i];
        n0_used = run;
        return true;
    }

    int32_t live() const {
        int32_t a = 0;
        for (const EngineInst& x : insts) a += !x.done;
        return a;
    }

    // One round for every graph in the engine. Graphs whose result became
    // final are appended to `finished` (their sides are then read with
    // side_of); graphs finished in the previous round leave the union graph.
    mc_status step(std::vector<EngineInst>& finished) {
        const int32_t k = (int32_t)insts.size();
        if (k == 0) return MC_OK;
        DGraph& G = w.g[cur];
        G.n = n;
        DGraph& Nx = w.g[(cur + 1) % 3];
        // instance arrays of the round
        std::vector<int32_t> vo(k + 1), io(k + 1);
        std::vector<int64_t> lam(k);
        std::vector<uint8_t> done(k), dead(k);
        // graphs of at most finish_max_n vertices finish every remaining
        // round in the finisher (one workgroup each, before this round's
        // launches); they take no part in the round and leave the union
        // graph in its contraction
        const int32_t fmax = c->opt.finish_max_n < 0 ? 0
                             : (c->opt.finish_max_n > 0 ? std::min(c->opt.finish_max_n, FIN_N) : FIN_N);
        std::vector<int32_t> flist;
        for (int32_t i = 0; i < k; i++) {
            vo[i] = insts[i].voff;
            io[i] = insts[i].ioff;
            lam[i] = insts[i].lam;
            const bool fin = !insts[i].done && !insts[i].dead && insts[i].nv > 2 && insts[i].nv <= fmax &&
                             insts[i].lam > 0;
            if (fin) flist.push_back(i);
            done[i] = insts[i].done || insts[i].dead || fin;
            dead[i] = insts[i].dead || fin;
        }
        vo[k] = n;
        io[k] = n0_used;
        EG_HIP(hipMemcpyAsync(w.voff, vo.data(), sizeof(int32_t) * (k + 1), hipMemcpyHostToDevice, s));
        EG_HIP(hipMemcpyAsync(w.ioff, io.data(), sizeof(int32_t) * (k + 1), hipMemcpyHostToDevice, s));
        EG_HIP(hipMemcpyAsync(w.lam, lam.data(), sizeof(int64_t) * k, hipMemcpyHostToDevice, s));
        EG_HIP(hipMemcpyAsync(w.done, done.data(), k, hipMemcpyHostToDevice, s));
        EG_HIP(hipMemcpyAsync(w.dead, dead.data(), k, hipMemcpyHostToDevice, s));
        EG_OK(fill_u8(w.snap, 0, k, s));
        EG_OK(fill_i32(w.cnt, 0, 4, s));
        EG_OK(fill_i64((int64_t*)&w.sc->marks_pr, 0, 3, s));
        k_bg_vinst<<<grid_for(n, 256), 256, 0, s>>>(w.voff, k, n, w.vinst);
        k_bg_vinst<<<grid_for(n0_used, 256), 256, 0, s>>>(w.ioff, k, n0_used, w.inst0);
        EG_OK(mc_hip_ok(hipGetLastError(), "k_bg_vinst"));
        const int32_t nf = (int32_t)flist.size();
        if (nf > 0) {
            EG_HIP(hipMemcpyAsync(w.flist, flist.data(), sizeof(int32_t) * nf, hipMemcpyHostToDevice, s));
            EG_OK(fill_i32(w.ferr, 0, 2, s));
            FinishArgs fa{};
            fa.g = G;
            fa.gvoff = w.voff;
            fa.glist = w.flist;
            fa.lam_in = w.lam;
            fa.lam_out = w.lam;
            fa.dropped = w.fdrop;
            fa.fside = w.fside;
            fa.xcol[0] = w.g[(cur + 1) % 3].col;
            fa.xw[0] = w.g[(cur + 1) % 3].w;
            fa.xcol[1] = w.g[(cur + 2) % 3].col;
            fa.xw[1] = w.g[(cur + 2) % 3].w;
            fa.xwindow = 1;
            fa.seed = c->opt.seed ^ ((uint64_t)(uint32_t)round << 20);
            fa.rounds = w.frounds;
            fa.err = w.ferr;
            fa.qnext = w.ferr + 1;
            fa.qmode = c->opt.queue;
            EG_OK(finish_graphs(fa, nf, c->cus, s));
            k_bg_fin_snap<<<grid_for(nf, 256), 256, 0, s>>>(w.flist, nf, w.fdrop, w.snap);
            EG_OK(mc_hip_ok(hipGetLastError(), "k_bg_fin_snap"));
        }
        EG_OK(uf_init(w.parent, n, s));
        // reduction tests with each graph's own bound
        EG_OK(pr12(G, w.lam, w.parent, &w.sc->marks_pr, nullptr, tri_on ? w.tw.ptr2 : nullptr, w.prw, s, w.vinst));
        if (tri_on)
            EG_OK(pr34(G, w.lam, c->opt.pr_tri_deg_cap, w.parent, &w.sc->marks_tri, w.tw.ptr2, w.tw, nullptr, nullptr,
                       s, w.vinst));
        // one CAPFOREST pass per graph still in the rounds
        k_bg_active<<<grid_for(k, 256), 256, 0, s>>>(w.done, k, w.prun);
        PrivateArgs pa = w.pv;
        pa.g = G;
        pa.lam = w.lam;
        pa.parent = w.parent;
        pa.passes = k;
        pa.len_cap = c->opt.pass_len_cap > 0 ? c->opt.pass_len_cap : (c->opt.pass_len_cap < 0 ? 0 : 32768);
        pa.seed = c->opt.seed;
        pa.round = round;
        pa.start = -1;
        pa.marks = &w.sc->marks_cf;
        pa.steps = nullptr;
        pa.diag = nullptr;
        pa.pvoff = w.voff;
        pa.plam = w.lam;
        pa.prun = w.prun;
        pa.pmarks = w.pmarks;
        pa.threads = c->opt.batch_pass_threads;
        EG_OK(capforest_private(pa, s, cap.nmax));
        k_bg_alpha<<<grid_for(k, 256), 256, 0, s>>>(pa.alpha, w.done, k, w.lam, w.snap);
        EG_OK(labels(k));
        k_bg_offsets<<<grid_for(k + 1, 256), 256, 0, s>>>(w.flag, w.voff, k, w.voff2);
        k_bg_fallback<<<grid_for(k, 256), 256, 0, s>>>(w.voff, w.voff2, w.done, k, w.prun, w.cnt);
        EG_OK(mc_hip_ok(hipGetLastError(), "round"));
        int32_t hcnt[4];
        EG_HIP(hipMemcpyAsync(hcnt, w.cnt, sizeof(hcnt), hipMemcpyDeviceToHost, s));
        if (!readback()) return mc_fail(MC_E_DEVICE, "readback failed");
        if (tri_on && c->hsc->marks_tri * 100 < (unsigned long long)std::max(n, 1)) tri_on = false;
        if (hcnt[0] > 0) {
            // Algorithm 2: graphs without a contractible edge get one complete
            // pass; first take the sides of the truncated passes' prefixes
            EG_OK(prefix_sides(pa, k));
            PrivateArgs pf = pa;
            pf.len_cap = 0;
            pf.round = round + 7777;
            EG_OK(capforest_private(pf, s, cap.nmax));
            k_bg_alpha<<<grid_for(k, 256), 256, 0, s>>>(pf.alpha, w.done, k, w.lam, w.snap);
            EG_OK(labels(k));
            k_bg_offsets<<<grid_for(k + 1, 256), 256, 0, s>>>(w.flag, w.voff, k, w.voff2);
            EG_OK(mc_hip_ok(hipGetLastError(), "fallback"));
        }
        EG_OK(prefix_sides(pa, k));
        if (!readback()) return mc_fail(MC_E_DEVICE, "readback failed");
        const int32_t n2 = c->hsc->n2;
        // contraction (dead graphs leave), collapsed degrees per graph
        EG_OK(contract(G, w.L, n2, Nx, w.cw, w.sc, s));
        EG_OK(map_update(w.map0, w.L, n0_used, s));
        k_bg_segmin<<<std::min(k, 8192), 256, 0, s>>>(Nx.deg, w.voff2, k, w.dmin, w.darg);
        k_bg_bound<<<grid_for(k, 256), 256, 0, s>>>(w.voff2, w.dmin, k, w.lam, w.done, w.snap, w.cnt);
        k_bg_side<<<grid_for(n0_used, 256), 256, 0, s>>>(w.side, w.map0, w.inst0, n0_used, w.snap, w.darg, w.inpref,
                                                          w.fside);
        EG_OK(mc_hip_ok(hipGetLastError(), "bound"));
        // new ranges, bounds and states; the entries in use of the new graph
        std::vector<int32_t> v2(k + 1);
        EG_HIP(hipMemcpyAsync(v2.data(), w.voff2, sizeof(int32_t) * (k + 1), hipMemcpyDeviceToHost, s));
        EG_HIP(hipMemcpyAsync(lam.data(), w.lam, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s));
        EG_HIP(hipMemcpyAsync(done.data(), w.done, k, hipMemcpyDeviceToHost, s));
        int32_t total = 0;
        EG_HIP(hipMemcpyAsync(&total, w.cw.gstart + n2, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        std::vector<int32_t> frounds(k, 0);
        int32_t ferr = 0;
        if (nf > 0) {
            EG_HIP(hipMemcpyAsync(frounds.data(), w.frounds, sizeof(int32_t) * k, hipMemcpyDeviceToHost, s));
            EG_HIP(hipMemcpyAsync(&ferr, w.ferr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        }
        EG_HIP(hipStreamSynchronize(s));
        if (ferr != 0) return mc_fail(MC_E_DEVICE, "engine: a graph could not finish (code " + std::to_string(ferr) + ")");
        std::vector<uint8_t> finished_now(k, 0);
        for (int32_t i : flist) finished_now[i] = 1;
        std::vector<EngineInst> keep;
        keep.reserve(k);
        for (int32_t i = 0; i < k; i++) {
            EngineInst x = insts[i];
            if (finished_now[i]) {
                // the finisher completed it: its bound is lambda, its side is
                // in place; its vertices left in this contraction
                x.lam = lam[i];
                x.rounds += 1 + frounds[i];
                x.done = true;
                x.dead = true;
                x.nv = 0;
                finished.push_back(x);
                continue;
            }
            if (x.dead) continue;                 // left the union graph in this contraction
            x.voff = v2[i];
            x.nv = v2[i + 1] - v2[i];
            x.lam = lam[i];
            x.rounds++;
            if (!x.done && (done[i] || x.lam == 0 || x.nv <= 2)) {
                x.done = true;
                finished.push_back(x);
                x.dead = true;                    // leaves in the next round
            } else if (x.done) {
                x.dead = true;
            }
            keep.push_back(x);
        }
        insts.swap(keep);
        n = n2;
        used = total;
        cur = &Nx - w.g;
        round++;
        return MC_OK;
    }

    // labels of the round: canonical components, -1 for dead graphs
    bool labels(int32_t k) {
        const int32_t nn = n;
        (void)k;
        if (!uf_labels(w.parent, nn, w.L, w.flag, w.cw.scan_tmp, w.sc, s)) return false;   // compresses
        k_root_flag_live<<<grid_for(nn, 256), 256, 0, s>>>(w.parent, w.vinst, w.dead, nn, w.flag);
        if (!mc_hip_ok(hipGetLastError(), "k_root_flag_live")) return false;
        if (!scan_i32(w.flag, w.flag, nn, w.cw.scan_tmp, s)) return false;
        k_label_live<<<grid_for(nn, 256), 256, 0, s>>>(w.parent, w.flag, w.vinst, w.dead, nn, w.L, w.sc);
        return mc_hip_ok(hipGetLastError(), "k_label_live");
    }

    // sides of graphs whose bound dropped to a pass's prefix this round
    bool prefix_sides(const PrivateArgs& pa, int32_t k) {
        k_bg_prefix<<<grid_for(n, 256), 256, 0, s>>>(pa.order, w.voff, w.vinst, pa.alpha_len, w.snap, n, w.inpref, 1);
        k_bg_side<<<grid_for(n0_used, 256), 256, 0, s>>>(w.side, w.map0, w.inst0, n0_used, w.snap, w.darg, w.inpref,
                                                          w.fside);
        k_bg_prefix<<<grid_for(n, 256), 256, 0, s>>>(pa.order, w.voff, w.vinst, pa.alpha_len, w.snap, n, w.inpref, 0);
        k_bg_clear_snap<<<grid_for(k, 256), 256, 0, s>>>(w.snap, k);
        return mc_hip_ok(hipGetLastError(), "prefix sides");
    }

    // side of a finished graph (host, n0 bytes, side[0] = 0); then its input
    // vertices are no longer tracked
    mc_status side_of(const EngineInst& x, uint8_t* out) {
        if (out) {
            EG_HIP(hipMemcpyAsync(out, w.side + x.ioff, x.n0, hipMemcpyDeviceToHost, s));
            EG_HIP(hipStreamSynchronize(s));
            const uint8_t flip = out[0];
            if (flip)
                for (int32_t v = 0; v < x.n0; v++) out[v] ^= 1;
        }
        k_eg_untrack<<<grid_for(x.n0, 256), 256, 0, s>>>(w.map0, x.ioff, x.n0);
        EG_OK(mc_hip_ok(hipGetLastError(), "k_eg_untrack"));
        return MC_OK;
    }
};

namespace {

Caps batch_caps(int32_t k, const mc_csr* gs, bool& ok) {
    // graphs that can never be admitted (n < 2, nnz < 0) take no room
    Caps cp;
    int64_t n = 0, e = 0;
    int32_t nmax = 0;
    for (int32_t i = 0; i < k; i++) {
        if (gs[i].n < 2 || gs[i].nnz < 0) continue;
        n += gs[i].n;
        e += gs[i].nnz;
        nmax = std::max(nmax, gs[i].n);
    }
    ok = n < INT32_MAX / 2 && e < INT32_MAX / 2;
    cp.N = cp.N0 = cp.Ns = (int32_t)std::max<int64_t>(n, 2);
    cp.C = cp.Cs = e;
    cp.K = k;
    cp.nmax = std::max(nmax, 2);
    return cp;
}

}  // namespace

extern "C" mc_status mc_batch_workspace_size(const mc_ctx* c, int32_t k, const mc_csr* gs, size_t* bytes) {
    if (!c || !gs || !bytes || k <= 0) return mc_fail(MC_E_INVALID_ARG, "mc_batch_workspace_size: bad argument");
    bool ok;
    Caps cp = batch_caps(k, gs, ok);
    if (!ok) return mc_fail(MC_E_OVERFLOW, "batch too large (vertices or entries >= 2^30)");
    Arena a;
    EngineWS w;
    carve_engine(a, cp, w);
    *bytes = a.used + 256;
    return MC_OK;
}

extern "C" mc_status mc_mincut_batch(mc_ctx* c, int32_t k, const mc_csr* gs, void* dev_ws, size_t ws_bytes,
                                     int64_t* lambdas, uint8_t* const* sides, mc_status* per_graph) {
    if (!c || !gs || !lambdas || k <= 0 || !dev_ws) return mc_fail(MC_E_INVALID_ARG, "mc_mincut_batch: bad argument");
    const int32_t loc = gs[0].location;
    for (int32_t i = 0; i < k; i++)
        if (gs[i].location != loc || (loc != MC_HOST && loc != MC_DEVICE))
            return mc_fail(MC_E_INVALID_ARG, "mc_mincut_batch: all graphs of one call must share one location");
    bool ok;
    Caps cp = batch_caps(k, gs, ok);
    if (!ok) return mc_fail(MC_E_OVERFLOW, "batch too large (vertices or entries >= 2^30)");
    // every graph is checked on its own: one bad graph does not stop the
    // others when per_graph is given
    std::vector<mc_status> st((size_t)k, MC_OK);
    std::vector<std::string> why((size_t)k);
    std::vector<int32_t> dev_idx;
    for (int32_t i = 0; i < k; i++) {
        const mc_csr& g = gs[i];
        if (loc == MC_HOST) {
            st[i] = check_host_csr(&g, c->opt.validate != 0);
        } else if (g.n < 2) {
            st[i] = mc_fail(MC_E_INVALID_ARG, "need n >= 2");
        } else if (g.nnz < 0 || !g.row_ptr || (g.nnz > 0 && (!g.col || !g.w))) {
            st[i] = mc_fail(MC_E_INVALID_ARG, "bad CSR pointers");
        } else {
            dev_idx.push_back(i);
        }
        if (st[i] != MC_OK) why[i] = mc_error_slot();
    }
    Engine E;
    mc_status r = E.init(c, cp, dev_ws, ws_bytes);
    if (r != MC_OK) return r;
    if (!dev_idx.empty()) {
        std::vector<mc_csr> dg;
        for (int32_t i : dev_idx) dg.push_back(gs[i]);
        std::vector<mc_status> ds(dg.size());
        if ((r = E.check_device(dg.data(), (int32_t)dg.size(), ds.data())) != MC_OK) return r;
        for (size_t q = 0; q < dg.size(); q++) {
            st[dev_idx[q]] = ds[q];
            if (ds[q] == MC_E_BAD_GRAPH) why[dev_idx[q]] = "malformed CSR (row_ptr, col or w)";
            if (ds[q] == MC_E_OVERFLOW) why[dev_idx[q]] = "total weight must be below 2^62";
        }
    }
    std::vector<mc_csr> good;
    std::vector<uint64_t> ids;
    for (int32_t i = 0; i < k; i++) {
        if (st[i] == MC_OK) {
            good.push_back(gs[i]);
            ids.push_back((uint64_t)i);
        } else if (!per_graph) {
            return mc_fail(st[i], "mc_mincut_batch: graph " + std::to_string(i) + ": " + why[i]);
        }
    }
    if (!good.empty() && (r = E.admit(good.data(), (int32_t)good.size(), ids.data())) != MC_OK) return r;
    std::vector<EngineInst> fin;
    // graphs final at admission (two vertices, or lambda 0)
    for (EngineInst& x : E.insts)
        if (x.done) fin.push_back(x);
    for (EngineInst& x : E.insts)
        if (x.done) x.dead = true;
    // results are staged and written only once every graph is done, so a
    // failing call leaves the outputs untouched
    std::vector<int64_t> lam_out((size_t)k, 0);
    std::vector<std::vector<uint8_t>> side_out(sides ? (size_t)k : 0);
    size_t got = 0;
    for (int32_t rounds = 0;; rounds++) {
        for (; got < fin.size(); got++) {
            const EngineInst& x = fin[got];
            lam_out[x.id] = x.lam;
            uint8_t* so = nullptr;
            if (sides && sides[x.id]) {
                side_out[x.id].resize((size_t)x.n0);
                so = side_out[x.id].data();
            }
            if ((r = E.side_of(x, so)) != MC_OK) return r;
        }
        if (E.live() == 0) break;
        if (rounds > cp.N + 64) return mc_fail(MC_E_DEVICE, "mc_mincut_batch: no progress");
        if ((r = E.step(fin)) != MC_OK) return r;
    }
    for (int32_t i = 0; i < k; i++) {
        if (per_graph) per_graph[i] = st[i];
        if (st[i] != MC_OK) continue;
        lambdas[i] = lam_out[i];
        if (sides && sides[i]) std::copy(side_out[i].begin(), side_out[i].end(), sides[i]);
    }
    return MC_OK;
}

// The autotuner: time the batch engine on a sample of the batch under every
// candidate setting (best of two runs each) and keep the fastest. A batch
// takes as long as the passes of its largest graphs, so the sample holds the
// batch's largest graphs (an eighth of it, by entries) and a spread of the
// rest.
extern "C" mc_status mc_batch_autotune(mc_ctx* c, int32_t k, const mc_csr* gs, void* dev_ws, size_t ws_bytes,
                                       int32_t sample, mc_tuning* out) {
    if (!c || !gs || k <= 0 || !dev_ws || !out) return mc_fail(MC_E_INVALID_ARG, "mc_batch_autotune: bad argument");
    const int32_t m = sample <= 0 || sample >= k ? k : sample;
    std::vector<mc_csr> sub;
    sub.reserve((size_t)m);
    {
        std::vector<int32_t> idx((size_t)k);
        for (int32_t i = 0; i < k; i++) idx[i] = i;
        const int32_t big = m < k ? m / 8 : 0;
        std::partial_sort(idx.begin(), idx.begin() + big, idx.end(),
                          [&](int32_t a, int32_t b) { return gs[a].nnz > gs[b].nnz || (gs[a].nnz == gs[b].nnz && a < b); });
        std::vector<char> taken((size_t)k, 0);
        for (int32_t i = 0; i < big; i++) { taken[idx[i]] = 1; sub.push_back(gs[idx[i]]); }
        const int32_t rest = m - big;
        for (int32_t i = 0; i < rest; i++) {
            int64_t j = (int64_t)i * k / rest;
            while (taken[j]) j = (j + 1) % k;   // k > m, so a free one exists
            taken[j] = 1;
            sub.push_back(gs[j]);
        }
    }
    std::vector<int64_t> lam((size_t)m);
    const mc_options saved = c->opt;
    static const int32_t threads[] = {64, 128, 256, 512, 1024};
    mc_tuning t{};
    t.sample = m;
    // one untimed run first: first-touch costs are not any setting's
    mc_status r = mc_mincut_batch(c, m, sub.data(), dev_ws, ws_bytes, lam.data(), nullptr, nullptr);
    if (r != MC_OK) { c->opt = saved; return r; }
    double best = 0;
    // the faster of two synchronised runs of the sample with the current options
    auto timed = [&](double* ms) -> mc_status {
        *ms = 0;
        for (int rep = 0; rep < 2; rep++) {
            if (hipStreamSynchronize(c->stream) != hipSuccess) return mc_fail(MC_E_DEVICE, "mc_batch_autotune: sync");
            const auto t0 = std::chrono::steady_clock::now();
            const mc_status rr = mc_mincut_batch(c, m, sub.data(), dev_ws, ws_bytes, lam.data(), nullptr, nullptr);
            if (rr != MC_OK) return rr;
            const double t1 = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            *ms = rep == 0 || t1 < *ms ? t1 : *ms;
        }
        return MC_OK;
    };
    auto record = [&](double ms) {
        const int32_t j = t.candidates++;
        t.cand_threads[j] = c->opt.batch_pass_threads;
        t.cand_lp[j] = c->opt.batch_lp;
        t.cand_finish[j] = c->opt.finish_max_n;
        t.cand_queue[j] = c->opt.queue;
        t.cand_ms[j] = ms;
        if (j == 0 || ms < best) {
            best = ms;
            t.pass_threads = c->opt.batch_pass_threads;
            t.lp = c->opt.batch_lp;
            t.finish_max_n = c->opt.finish_max_n;
            t.queue = c->opt.queue;
        }
    };
    // stage 1: pass workgroup size and admission bound
    for (int32_t lp = 1; lp <= 2; lp++) {
        for (int32_t th : threads) {
            c->opt.batch_pass_threads = th;
            c->opt.batch_lp = lp;
            double ms;
            if ((r = timed(&ms)) != MC_OK) { c->opt = saved; return r; }
            record(ms);
        }
    }
    // stage 2: the finisher's size limit, then its queue
    c->opt.batch_pass_threads = t.pass_threads;
    c->opt.batch_lp = t.lp;
    static const int32_t limits[] = {512, 256, -1};
    for (int32_t f : limits) {
        c->opt.finish_max_n = f;
        c->opt.queue = t.queue;
        double ms;
        if ((r = timed(&ms)) != MC_OK) { c->opt = saved; return r; }
        record(ms);
    }
    if (t.finish_max_n >= 0) {
        const int32_t q0 = t.queue;
        for (int32_t q = 0; q <= 2; q++) {
            if (q == q0) continue;
            c->opt.finish_max_n = t.finish_max_n;
            c->opt.queue = q;
            double ms;
            if ((r = timed(&ms)) != MC_OK) { c->opt = saved; return r; }
            record(ms);
        }
    }
    c->opt = saved;
    c->opt.batch_pass_threads = t.pass_threads;
    c->opt.batch_lp = t.lp;
    c->opt.finish_max_n = t.finish_max_n;
    c->opt.queue = t.queue;
    *out = t;
    return MC_OK;
}

// ------------------------------------------------------------ the server
// Continuous batching over the engine: requests are checked and copied at
// submission and queued; every mc_server_step admits queued requests in
// arrival order while they fit the engine's capacity (graphs in flight,
// vertices, entries; all carved from one device allocation of the
// configured HBM budget), runs one round for every graph in flight, and
// collects the graphs whose result became final. Graphs admitted while
// others are half way through their rounds join them in the same launches;
// a graph's rounds do not depend on the others (its bound, passes and
// contractions touch only its own range), so its result is the one it gets
// alone. Large requests (n >= solo_min_n) are solved by mc_mincut on a
// worker thread with a context and non-blocking stream of their own, from a
// workspace set aside in the budget, so their kernels overlap the engine's
// rounds on the device and nothing waits for them.
#include <atomic>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>

struct mc_server {
    mc_ctx* c = nullptr;
    void* mem = nullptr;
    size_t bytes = 0;             // engine part of mem
    size_t solo_bytes = 0;        // workspace of each solo slot
    Engine E;
    int32_t solo_min_n = 0;
    double deadline_ms = 0;
    std::chrono::steady_clock::time_point t0;
    struct Req {
        std::vector<int32_t> rp, col;
        std::vector<int64_t> w;
        int32_t n = 0, nnz = 0;
        int state = 0;             // 0 queued, 1 in flight, 2 done, 3 cancelled, 4 failed, 5 timed out
        bool cancel = false;
        bool solo = false;
        mc_status status = MC_OK;  // of a failed request
        std::string err;
        int64_t lam = 0;
        std::vector<uint8_t> side;
        mc_req_stats st{};
    };
    // one large request at a time per slot, on its own context and stream
    struct Slot {
        mc_ctx* ctx = nullptr;
        hipStream_t stream = nullptr;
        void* ws = nullptr;
        std::thread th;
        std::atomic<int> busy{0};  // 0 free, 1 running, 2 result ready
        uint64_t id = 0;
        mc_status st = MC_OK;
        std::string err;
        int64_t lam = 0;
        std::vector<uint8_t> side;
    };
    std::vector<std::unique_ptr<Slot>> slots;
    std::unordered_map<uint64_t, Req> reqs;
    std::deque<uint64_t> queue;
    uint64_t next = 1;
    double now() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    bool late(const Req& r, double t) const { return deadline_ms > 0 && t - r.st.t_submit_ms > deadline_ms; }
};

namespace {

Caps server_caps(const mc_server_opts& o, int64_t C) {
    Caps cp;
    cp.K = o.max_inflight > 0 ? o.max_inflight : 1024;
    cp.nmax = o.max_request_n > 0 ? o.max_request_n : (1 << 20);
    const int64_t rn = o.max_request_nnz > 0 ? o.max_request_nnz : ((int64_t)1 << 25);
    cp.C = C;
    cp.N = (int32_t)std::min<int64_t>(C / 2 + 4 * (int64_t)cp.K, INT32_MAX / 4);
    cp.N0 = cp.N;
    cp.Ns = (int32_t)std::min<int64_t>(std::max<int64_t>(cp.nmax, cp.N / 4), cp.N);
    cp.Cs = std::min<int64_t>(std::max<int64_t>(rn, C / 4), C);
    return cp;
}

size_t engine_bytes(const Caps& cp) {
    Arena a;
    EngineWS w;
    carve_engine(a, cp, w);
    return a.used + 256;
}

mc_status finish(mc_server* S, const EngineInst& x) {
    auto it = S->reqs.find(x.id);
    if (it == S->reqs.end()) return mc_fail(MC_E_DEVICE, "server: unknown graph in flight");
    mc_server::Req& r = it->second;
    r.side.assign((size_t)r.n, 0);
    mc_status st = S->E.side_of(x, r.side.data());
    if (st != MC_OK) return st;
    r.lam = x.lam;
    r.st.t_done_ms = S->now();
    r.st.rounds = x.rounds;
    r.state = r.cancel ? 3 : (S->late(r, r.st.t_done_ms) ? 5 : 2);
    return MC_OK;
}

void fail_req(mc_server::Req& r, mc_status st, const std::string& why, double t) {
    r.state = 4;
    r.status = st;
    r.err = why;
    r.st.t_done_ms = t;
}

mc_csr host_csr(const mc_server::Req& r) {
    mc_csr g;
    g.n = r.n;
    g.nnz = r.nnz;
    g.row_ptr = r.rp.data();
    g.col = r.col.data();
    g.w = r.w.data();
    g.location = MC_HOST;
    return g;
}

// collect the results of solo slots whose solve ended
void collect_solo(mc_server* S) {
    for (auto& sp : S->slots) {
        mc_server::Slot& sl = *sp;
        if (sl.busy.load(std::memory_order_acquire) != 2) continue;
        sl.th.join();
        mc_server::Req& r = S->reqs[sl.id];
        const double t = S->now();
        if (sl.st != MC_OK) {
            fail_req(r, sl.st, sl.err, t);
        } else {
            r.lam = sl.lam;
            r.side.swap(sl.side);
            r.st.t_done_ms = t;
            r.st.rounds = 0;
            r.state = r.cancel ? 3 : (S->late(r, t) ? 5 : 2);
        }
        sl.busy.store(0, std::memory_order_relaxed);
    }
}

bool start_solo(mc_server* S, uint64_t id) {
    for (auto& sp : S->slots) {
        mc_server::Slot& sl = *sp;
        if (sl.busy.load(std::memory_order_acquire) != 0) continue;
        mc_server::Req& r = S->reqs[id];
        r.state = 1;
        r.solo = true;
        r.st.t_admit_ms = S->now();
        sl.id = id;
        sl.side.assign((size_t)r.n, 0);
        sl.busy.store(1, std::memory_order_relaxed);
        const mc_csr g = host_csr(r);
        mc_server::Slot* p = &sl;
        const size_t wsb = S->solo_bytes;
        sl.th = std::thread([p, g, wsb]() {
            p->st = mc_mincut(p->ctx, &g, p->ws, wsb, &p->lam, p->side.data(), nullptr);
            if (p->st != MC_OK) p->err = mc_last_error();
            p->busy.store(2, std::memory_order_release);
        });
        return true;
    }
    return false;
}

// drop an engine request in flight (cancelled or past its deadline): its
// vertices leave the union graph in the next contraction
mc_status drop_inflight(mc_server* S, uint64_t id) {
    for (EngineInst& x : S->E.insts) {
        if (x.id != id || x.dead) continue;
        x.done = true;
        x.dead = true;
        return S->E.side_of(x, nullptr);   // stops tracking its input vertices
    }
    return MC_OK;
}

}  // namespace

extern "C" mc_status mc_server_create(mc_ctx* c, const mc_server_opts* opts, mc_server** out) {
    if (!c || !opts || !out) return mc_fail(MC_E_INVALID_ARG, "mc_server_create: NULL argument");
    if (opts->hbm_bytes < ((size_t)64 << 20)) return mc_fail(MC_E_INVALID_ARG, "mc_server_create: budget below 64 MiB");
    if (opts->solo_slots < 0 || opts->solo_slots > 8 || opts->deadline_ms < 0)
        return mc_fail(MC_E_INVALID_ARG, "mc_server_create: solo_slots must be in [0, 8] and deadline_ms >= 0");
    // requests of at least solo_min_n vertices are solved on solo slots by
    // the single-graph solver (whole-GPU CAPFOREST steps, the full
    // heuristic); the rest of the budget holds the engine
    const int32_t rn = opts->max_request_n > 0 ? opts->max_request_n : (1 << 20);
    const int64_t re = opts->max_request_nnz > 0 ? opts->max_request_nnz : ((int64_t)1 << 25);
    const int32_t solo_min_n = opts->solo_min_n > 0 ? opts->solo_min_n : (1 << 16);
    const int32_t nslots = rn >= solo_min_n ? (opts->solo_slots > 0 ? opts->solo_slots : 1) : 0;
    size_t solo = 0;
    if (nslots > 0) {
        solo = workspace_min_bytes(c, rn, (int32_t)std::min<int64_t>(re, INT32_MAX / 2));
        solo = (solo + 4095) & ~(size_t)4095;
    }
    if (solo * nslots + ((size_t)64 << 20) > opts->hbm_bytes)
        return mc_fail(MC_E_INVALID_ARG, "mc_server_create: budget too small for the largest request");
    const size_t engine_budget = opts->hbm_bytes - solo * nslots;
    // the largest entry capacity whose engine fits the budget
    mc_server_opts eo = *opts;
    if (rn >= solo_min_n) eo.max_request_n = solo_min_n - 1;
    int64_t lo = 1024, hi = (int64_t)1 << 30;
    if (engine_bytes(server_caps(eo, lo)) > engine_budget)
        return mc_fail(MC_E_INVALID_ARG, "mc_server_create: budget too small for the options");
    while (hi - lo > 1024) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (engine_bytes(server_caps(eo, mid)) <= engine_budget) lo = mid; else hi = mid;
    }
    const Caps cp = server_caps(eo, lo);
    std::unique_ptr<mc_server> S(new (std::nothrow) mc_server());
    if (!S) return mc_fail(MC_E_OOM, "mc_server_create: out of host memory");
    S->c = c;
    S->bytes = (engine_bytes(cp) + 4095) & ~(size_t)4095;
    S->solo_bytes = solo;
    S->solo_min_n = solo_min_n;
    S->deadline_ms = opts->deadline_ms;
    if (hipSetDevice(c->device) != hipSuccess || hipMalloc(&S->mem, S->bytes + solo * nslots) != hipSuccess)
        return mc_fail(MC_E_OOM, "mc_server_create: device allocation of the budget failed");
    auto cleanup = [&]() {
        for (auto& sl : S->slots) {
            if (sl->ctx) mc_ctx_destroy(sl->ctx);
            if (sl->stream) (void)hipStreamDestroy(sl->stream);
        }
        (void)hipFree(S->mem);
    };
    for (int32_t q = 0; q < nslots; q++) {
        std::unique_ptr<mc_server::Slot> sl(new mc_server::Slot());
        sl->ws = (char*)S->mem + S->bytes + solo * q;
        // default priority, non-blocking: it must not wait for work on the
        // legacy default stream the engine may use
        if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess) {
            S->slots.push_back(std::move(sl));
            cleanup();
            return mc_fail(MC_E_DEVICE, "mc_server_create: stream creation failed");
        }
        mc_status r = mc_ctx_create(c->device, sl->stream, &c->opt, &sl->ctx);
        S->slots.push_back(std::move(sl));
        if (r != MC_OK) { cleanup(); return r; }
    }
    mc_status r = S->E.init(c, cp, S->mem, S->bytes);
    if (r != MC_OK) { cleanup(); return r; }
    S->t0 = std::chrono::steady_clock::now();
    *out = S.release();
    return MC_OK;
}

extern "C" mc_status mc_server_destroy(mc_server* S) {
    if (!S) return MC_OK;
    for (auto& sl : S->slots) {
        if (sl->th.joinable()) sl->th.join();   // a running solve ends first
        if (sl->ctx) mc_ctx_destroy(sl->ctx);
        if (sl->stream) (void)hipStreamDestroy(sl->stream);
    }
    if (S->mem) (void)hipFree(S->mem);
    delete S;
    return MC_OK;
}

extern "C" mc_status mc_server_submit(mc_server* S, const mc_csr* g, uint64_t* ticket) {
    if (!S || !g || !ticket) return mc_fail(MC_E_INVALID_ARG, "mc_server_submit: NULL argument");
    if (g->location != MC_HOST) return mc_fail(MC_E_INVALID_ARG, "mc_server_submit: host graphs only");
    // the request's contents are checked here, so admission never fails on
    // data
    mc_status v = check_host_csr(g, S->c->opt.validate != 0);
    if (v != MC_OK) return v;
    const Caps& cp = S->E.cap;
    if (g->n >= S->solo_min_n) {
        size_t need = 0;
        need = workspace_min_bytes(S->c, g->n, g->nnz);
        if (S->slots.empty() || need > S->solo_bytes)
            return mc_fail(MC_E_OOM, "mc_server_submit: graph larger than the server admits");
    } else if (g->n > cp.nmax || g->n > cp.Ns || g->nnz > cp.Cs || g->n > cp.N || g->nnz > cp.C) {
        return mc_fail(MC_E_OOM, "mc_server_submit: graph larger than the server admits");
    }
    mc_server::Req r;
    r.n = g->n;
    r.nnz = g->nnz;
    r.rp.assign(g->row_ptr, g->row_ptr + g->n + 1);
    r.col.assign(g->col, g->col + g->nnz);
    r.w.assign(g->w, g->w + g->nnz);
    r.st.t_submit_ms = S->now();
    const uint64_t id = S->next++;
    S->reqs.emplace(id, std::move(r));
    S->queue.push_back(id);
    *ticket = id;
    return MC_OK;
}

extern "C" mc_status mc_server_step(mc_server* S, int32_t* in_flight, int32_t* queued) {
    if (!S) return mc_fail(MC_E_INVALID_ARG, "mc_server_step: NULL server");
    Engine& E = S->E;
    mc_status st;
    collect_solo(S);
    double t = S->now();
    // requests in the engine that were cancelled or passed their deadline
    // leave it now
    for (size_t i = 0; i < E.insts.size(); i++) {
        const EngineInst x = E.insts[i];
        if (x.dead || x.done) continue;
        mc_server::Req& r = S->reqs[x.id];
        if (!r.cancel && !S->late(r, t)) continue;
        if ((st = drop_inflight(S, x.id)) != MC_OK) return st;
        r.state = r.cancel ? 3 : 5;
        r.st.t_done_ms = t;
    }
    // admission in arrival order: large requests to free solo slots, the
    // others into the engine while they fit (the first that does not fit
    // stops the engine's admission, so small requests keep their order)
    std::vector<mc_csr> adm;
    std::vector<uint64_t> ids;
    std::deque<uint64_t> rest;
    int64_t nv = 0, ne = 0;
    bool engine_full = false;
    for (uint64_t id : S->queue) {
        mc_server::Req& r = S->reqs[id];
        if (r.cancel) { r.state = 3; continue; }
        if (S->late(r, t)) { r.state = 5; r.st.t_done_ms = t; continue; }
        if (r.n >= S->solo_min_n) {
            if (!start_solo(S, id)) rest.push_back(id);
            continue;
        }
        if (engine_full) { rest.push_back(id); continue; }
        if (!E.fits((int32_t)adm.size() + 1, nv + r.n, ne + r.nnz)) {
            if (adm.empty() && E.live() == 0 && E.insts.empty()) {
                if (!E.compact_n0()) return MC_E_DEVICE;
                if (!E.fits(1, r.n, r.nnz)) {
                    fail_req(r, MC_E_OOM, "request does not fit the server's engine", t);
                    continue;
                }
            } else {
                engine_full = true;
                rest.push_back(id);
                continue;
            }
        }
        adm.push_back(host_csr(r));
        ids.push_back(id);
        nv += r.n;
        ne += r.nnz;
    }
    S->queue.swap(rest);
    if (!adm.empty()) {
        const size_t before = E.insts.size();
        if ((st = E.admit(adm.data(), (int32_t)adm.size(), ids.data())) != MC_OK) {
            // each request of the failed admission gets the error as its own
            // result; the engine keeps the graphs already in flight
            const std::string why = mc_error_slot();
            E.insts.resize(before);
            for (uint64_t id : ids) fail_req(S->reqs[id], st, why, S->now());
            return mc_fail(st, why);
        }
        t = S->now();
        for (uint64_t id : ids) { S->reqs[id].state = 1; S->reqs[id].st.t_admit_ms = t; }
        for (size_t i = before; i < E.insts.size(); i++)
            if (E.insts[i].done) {
                if ((st = finish(S, E.insts[i])) != MC_OK) return st;
                E.insts[i].dead = true;
            }
    }
    if (!E.insts.empty()) {
        // one round; with only finished graphs left it drops them from the
        // union graph
        std::vector<EngineInst> fin;
        if ((st = E.step(fin)) != MC_OK) {
            const std::string why = mc_error_slot();
            for (const EngineInst& x : E.insts)
                if (!x.dead) fail_req(S->reqs[x.id], st, why, S->now());
            (void)E.init(S->c, E.cap, S->mem, S->bytes);   // an empty engine for what follows
            return mc_fail(st, why);
        }
        for (const EngineInst& x : fin)
            if ((st = finish(S, x)) != MC_OK) return st;
    } else {
        // nothing on the engine: give a running solo solve a moment instead
        // of returning at once to a caller that polls in a loop
        for (auto& sl : S->slots)
            if (sl->busy.load(std::memory_order_acquire) == 1) {
                std::this_thread::sleep_for(std::chrono::microseconds(200));
                break;
            }
        collect_solo(S);
    }
    int32_t solo_running = 0;
    for (auto& sl : S->slots) solo_running += sl->busy.load(std::memory_order_acquire) != 0;
    if (in_flight) *in_flight = E.live() + solo_running;
    if (queued) *queued = (int32_t)S->queue.size();
    return MC_OK;
}

extern "C" mc_status mc_server_poll(mc_server* S, uint64_t ticket, int64_t* lambda, uint8_t* side, mc_req_stats* st) {
    if (!S) return mc_fail(MC_E_INVALID_ARG, "mc_server_poll: NULL server");
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return mc_fail(MC_E_INVALID_ARG, "mc_server_poll: unknown ticket");
    mc_server::Req& r = it->second;
    if (r.state == 3) {
        S->reqs.erase(it);
        return mc_fail(MC_E_CANCELLED, "mc_server_poll: request cancelled");
    }
    if (r.state == 4) {
        const mc_status code = r.status;
        const std::string why = r.err;
        S->reqs.erase(it);
        return mc_fail(code, "mc_server_poll: request failed: " + why);
    }
    if (r.state == 5) {
        S->reqs.erase(it);
        return mc_fail(MC_E_TIMEOUT, "mc_server_poll: request passed its deadline");
    }
    if (r.state != 2) return MC_E_NOT_READY;
    if (lambda) *lambda = r.lam;
    if (side) std::copy(r.side.begin(), r.side.end(), side);
    if (st) *st = r.st;
    S->reqs.erase(it);
    return MC_OK;
}

extern "C" mc_status mc_server_state(const mc_server* S, uint64_t ticket, int32_t* state) {
    if (!S || !state) return mc_fail(MC_E_INVALID_ARG, "mc_server_state: NULL argument");
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return mc_fail(MC_E_INVALID_ARG, "mc_server_state: unknown ticket");
    *state = it->second.state;
    return MC_OK;
}

extern "C" mc_status mc_server_cancel(mc_server* S, uint64_t ticket) {
    if (!S) return mc_fail(MC_E_INVALID_ARG, "mc_server_cancel: NULL server");
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return mc_fail(MC_E_INVALID_ARG, "mc_server_cancel: unknown ticket");
    it->second.cancel = true;
    if (it->second.state == 2) it->second.state = 3;
    return MC_OK;
}

extern "C" mc_status mc_server_capacity(const mc_server* S, int64_t* entries, int32_t* vertices, int32_t* graphs,
                                        size_t* bytes) {
    if (!S) return mc_fail(MC_E_INVALID_ARG, "mc_server_capacity: NULL server");
    if (entries) *entries = S->E.cap.C;
    if (vertices) *vertices = S->E.cap.N;
    if (graphs) *graphs = S->E.cap.K;
    if (bytes) *bytes = S->bytes + S->solo_bytes * S->slots.size();
    return MC_OK;
}
