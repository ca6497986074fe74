// Host-side declarations shared by the translation units of the library:
// workspace carving, kernel launchers and the per-call state.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "mc_device.h"
#include "mc_host.h"
#include "mincut.h"

// Records the first HIP failure of a call; launchers return false on error.
bool mc_hip_ok(hipError_t e, const char* what);
#define MC_HIP(call) do { if (!mc_hip_ok((call), #call)) return false; } while (0)
#define MC_LAUNCHED(what) do { if (!mc_hip_ok(hipGetLastError(), what)) return false; } while (0)

// ------------------------------------------------------------ profiling
// Optional timing of the hot kernels (mc_profile): while a solve runs on a
// context with profiling on, each timed launch is bracketed by two HIP
// events on its stream, and its algorithmic bytes go either to a device
// counter the kernel adds to (prof_dev_bytes) or are added by the host when
// the host knows them (prof_host_bytes). With profiling off, prof_dev_bytes
// returns nullptr and the kernels skip the count.
enum ProfKernel {
    PK_CFS_EDGES = 0, PK_MERGE_SMALL, PK_BIG_INSERT, PK_GROUP_COUNT, PK_GROUP_SCATTER, PK_PR12, PK_UF_LINK_REST,
    PK_LP_SMALL, PK_LP_FIRST, PK_MID_MERGE, PK_PR1_FIRST, PK_PR1_REST,
    PK_COUNT
};
void prof_begin(int k, hipStream_t s);
void prof_end(int k, hipStream_t s);
unsigned long long* prof_dev_bytes(int k);
void prof_host_bytes(int k, double bytes);

// Counters that many workgroups add to are split into SPREAD partial
// counters SPREAD_STRIDE words (128 B) apart and folded afterwards: atomics
// on one address serialise.
constexpr int SPREAD = 64;
constexpr int SPREAD_STRIDE = 16;

// Bump allocator over the caller's device workspace. With base == nullptr
// it only measures, so mc_workspace_size and the solver carve identically.
struct Arena {
    char* base = nullptr;
    size_t size = 0;
    size_t used = 0;
    template <class T>
    T* take(size_t count) {
        size_t off = (used + 255) & ~(size_t)255;
        used = off + count * sizeof(T);
        return base ? reinterpret_cast<T*>(base + off) : nullptr;
    }
};

// --------------------------------------------------------------- scan
// Exclusive prefix sum of in[0..count) into out[0..count]; out[count] is
// the total. in and out may alias. tmp must hold scan_tmp_elems(count).
size_t scan_tmp_elems(int64_t count);
bool scan_i32(const int32_t* in, int32_t* out, int64_t count, int32_t* tmp, hipStream_t s);

// ------------------------------------------------------- fill / misc
bool fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t s);
bool fill_i64(int64_t* p, int64_t v, int64_t count, hipStream_t s);
bool fill_u8(uint8_t* p, uint8_t v, int64_t count, hipStream_t s);
bool iota_i32(int32_t* p, int64_t count, hipStream_t s);

// ------------------------------------------------------- contraction
// Scratch of the contraction (sized for at most n input vertices and cap
// entries).
// Workspace of the sort-based edge merge (mc_sort.hip)
struct SortWS {
    int64_t cap = 0;
    uint64_t* key[2] = {};   // [cap+1] keys, ping-pong
    int64_t* val[2] = {};    // [cap+1] weights, ping-pong
    int32_t* flag = nullptr; // [cap+2] run heads
    int32_t* uidx = nullptr; // [cap+2] their exclusive prefix
    int32_t* hist = nullptr; // [256 * tiles + 2] per-tile digit counts -> offsets
    int32_t* scan_tmp = nullptr;
    int32_t* wcnt = nullptr; // per-wavefront entry counts -> offsets
    int32_t* rend = nullptr; // [n+1] end of each row's entries
};
void sort_ws_carve(Arena& a, int32_t n, int64_t cap, SortWS& w);

struct ContractWS {
    int32_t* gcnt;    // [n+1]  members per group -> vstart
    int32_t* vstart;  // [n+1]
    int32_t* gcur;    // [n]
    int32_t* perm;    // [n]    vertices grouped by label
    int32_t* mstart;  // [n+1]  entry offset of each member (perm order)
    int32_t* gstart;  // [n+1]  entry offset of each group
    int32_t* tsize;   // [n+1]  hash-table slots of each large group -> tbase
    int32_t* bigm;    // [n+1]  entries of each large group -> bebase
    int32_t* bcur;    // [n]
    int32_t* tkey;    // [4*cap+1024]
    int64_t* tval;    // [4*cap+1024]
    int32_t* dslot;   // [n+1]  dense accumulator of a giant group, or -1
    int32_t* dinfo;   // [1+DENSE_MAX] count, then the group of each slot
    int64_t* dense;   // [dense_elems] accumulators, n2 each; zeroed by each contraction for its giant groups
    int64_t dense_elems;
    int32_t* scan_tmp;
    int64_t* red_val; // [1024] per-block minima
    int32_t* red_id;  // [1024]
    int64_t* red_m;   // [1024] per-block entry counts
    int64_t* red_d;   // [1024] per-block maximum degrees
    int32_t* cg;      // [(cap+4n)/512+4] first group of every merge chunk
    int32_t* tinfo;   // [2*(cap/4096+2)] group and first member of every large-group tile
    int32_t* xg;      // [(5 cap/2)/256+8] group of every 256-slot table tile
    int32_t* mlist;   // [n+1] groups merged by one workgroup each in LDS
    int32_t* mcnt;    // [4] their count
    int32_t* sstart;  // [n+2] entry counts of the small groups (others 0) -> their prefix
    bool sorted = false;   // merge by sorting (mc_sort.hip) instead of hashing
    SortWS sw;
};
// sort: also carve the sort merge's workspace and use it in contract()
void contract_ws_carve(Arena& a, int32_t n, int64_t cap, ContractWS& ws, bool sort = false);

// Contract `src` by labels L (L == nullptr: identity, which only folds
// loops, parallel and zero-weight entries) into `dst` with n2 vertices.
// A vertex with label -1 is dropped (with its row; no kept row may point at
// it).
// dst.cap must be >= the sum of src.len. Of src.cap only one use is made:
// it bounds the sum of src.len and sizes the launch grids, so a caller that
// knows that sum may pass it there (entries_view). Writes
// dst.off/len/col/w/deg and the minimum degree (and its vertex) into
// sc->dmin / sc->dmin_arg.
// g with cap lowered to m, the sum of its row lengths when the caller knows
// it (m < 0: unknown), for contract and lp_round: their grids then follow
// the graph's entries rather than its arrays' capacity. Entry positions
// (off + j) may exceed m, so the view serves those two calls alone.
inline DGraph entries_view(const DGraph& g, int64_t m) {
    DGraph v = g;
    if (m >= 0 && m < v.cap) v.cap = m;
    return v;
}
bool contract(const DGraph& src, const int32_t* L, int32_t n2, DGraph& dst, ContractWS& ws,
              DevScalars* sc, hipStream_t s);

// contract() by a radix sort of the contracted entries and a segmented
// reduction (rows sorted by target); needs ws.sw.
bool contract_sorted(const DGraph& src, const int32_t* L, int32_t n2, DGraph& dst, ContractWS& ws, DevScalars* sc,
                     hipStream_t s);

// Minimum degree of g (ties: smallest vertex) into sc->dmin / dmin_arg, its
// entry count into sc->m2 and its maximum degree into sc->dmax.
bool min_degree(const DGraph& g, ContractWS& ws, DevScalars* sc, hipStream_t s);

// --------------------------------------------------------- union-find
bool uf_init(int32_t* parent, int32_t n, hipStream_t s);
// Union the endpoints of every entry with positive weight.
bool uf_all_edges(const DGraph& g, int32_t* parent, hipStream_t s);
// The same components for a graph whose entries all have positive weight
// (a normalised graph), with far fewer unions when there is a giant
// component (hooking sweeps, then sampling-based linking); tmp holds one
// int.
// lambda = 0 test: parent[] ends as a union-find of all edges of g. tmp: 4
// ints; inbig: n bytes; snap: n ints (scratch).
bool uf_connectivity(const DGraph& g, int32_t* parent, int32_t* tmp, uint8_t* inbig, int32_t* snap, hipStream_t s);
// Compress parent[] and write canonical labels (components numbered by
// their smallest vertex) to L; the count goes to sc->n2.
bool uf_labels(int32_t* parent, int32_t n, int32_t* L, int32_t* flag_tmp, int32_t* scan_tmp,
               DevScalars* sc, hipStream_t s);

// ----------------------------------------------------- reduction tests
// Padberg-Rinaldi test 1 (entry weight >= lam) and test 2 (one pointer per
// vertex to its heaviest neighbour when 2 c(v,p) >= c(v)), unioned into
// parent. Optional outputs for parity checks: flag1[entry], ptr2[vertex].
struct Pr12WS {
    int32_t* long_list;   // rows too long for the per-row pass
    int32_t* counters;
    int32_t* task_off;
    int64_t* part_w;
    int32_t* part_x;
    unsigned long long* spread;   // [SPREAD * SPREAD_STRIDE] partial mark counts
    int32_t* first;       // [n] a test-1 neighbour of each row, or -1
    int32_t* second;      // [n] a second test-1 neighbour of each row, or -1
    int32_t* heavy;       // [n] test-1 entries of each row
    int32_t* mode;        // [1] root of the largest sampled component
    uint8_t* inbig;       // [n] 1 for the vertices of that component
    int32_t* snap;        // [n] root of every vertex after the first two unions of each row
    int32_t* tscan;       // [n + 1] exclusive prefix count of the roots (tree numbers; [n] = trees)
    int32_t* scan_tmp;    // scratch of the prefix count
    uint32_t* tbits;      // [256 * 256 / 32] pairs of trees joined by a test-1 entry
    int32_t* troot;       // [256] root vertex of each tree
    int32_t* tmap;        // [256] root vertex of each tree's component
};
void pr12_ws_carve(Arena& a, int32_t n, int64_t cap, Pr12WS& w);
// With vinst (per-vertex instance) the bound of vertex v is lam[vinst[v]]
// (batched solves of many graphs in one union graph); else lam[0].
bool pr12(const DGraph& g, const int64_t* lam, int32_t* parent, unsigned long long* marks,
          uint8_t* flag1, int32_t* ptr2, Pr12WS& w, hipStream_t s, const int32_t* vinst = nullptr);

// Padberg-Rinaldi tests 3 and 4 on the edges whose rows both have at most
// D (<= 64) entries; test-4 edges and the accepted test-3 matching (mutual
// smallest partners touching no test-2 pointer of ptr2) are unioned into
// parent. Optional parity outputs: flag4[entry], acc3[vertex] (-1: none).
struct Pr34WS {
    int32_t* part3;   // [n] smallest test-3 partner
    uint8_t* touch;   // [n] test-2 pointer endpoints
    int32_t* ptr2;    // [n] test-2 pointers of the round (filled by pr12)
    unsigned long long* spread;
};
void pr34_ws_carve(Arena& a, int32_t n, Pr34WS& w);
bool pr34(const DGraph& g, const int64_t* lam, int32_t D, int32_t* parent, unsigned long long* marks,
          const int32_t* ptr2, Pr34WS& w, uint8_t* flag4, int32_t* acc3, hipStream_t s,
          const int32_t* vinst = nullptr);

// ---------------------------------------------------- label propagation
// Scratch of lp_round besides the contraction scratch it borrows (row
// prefix, scan temp, global tables).
struct LpWS {
    int32_t* long_list;   // rows longer than the chunked path takes
    int32_t* long_base;   // their global-table offsets
    int32_t* long_lab;    // smallest other label of the heaviest weight
    unsigned long long* long_best;   // heaviest other-label weight
    unsigned long long* long_own;    // weight of the row's own label
    int32_t* task_row;    // long row of every task
    int32_t* task_idx;    // task index within its row
    int32_t* counters;    // long rows, table slots, tasks
    int32_t* cg;          // first row of every chunk
};
void lp_ws_carve(Arena& a, int32_t n, int64_t cap, LpWS& w);
// One synchronous label-propagation round over g (Section 2.1 heuristic):
// lab_out[v] = heaviest neighbour label, keeping lab_in[v] unless another
// label is strictly heavier, smallest label on ties. Uses cw.mstart,
// cw.scan_tmp, cw.tkey and cw.tval as scratch. g.cap bounds the sum of
// g.len (it sizes the launch grids, as in contract). narrow: every row's degree is
// below 2^32, so (below 2^27 vertices) the per-label sums of short rows are
// kept in 32 bits, beside a 32-bit key, in one word of the chunk's table.
bool lp_round(const DGraph& g, const int32_t* lab_in, int32_t* lab_out, LpWS& w, ContractWS& cw, hipStream_t s,
              bool narrow = false);
// *narrow = every row of g has a weight sum below 2^32 (reads every weight;
// synchronises s). flag_tmp: one int of device scratch.
bool lp_narrow(const DGraph& g, int32_t* flag_tmp, bool* narrow, hipStream_t s);
// The same round from singleton labels (lab_in[v] = v) on a normal graph:
// lab_out[v] = v's heaviest neighbour, the smallest on ties, v if isolated.
bool lp_first(const DGraph& g, int32_t* lab_out, LpWS& w, ContractWS& cw, hipStream_t s);
// Canonical relabel of arbitrary labels in [0, n): L[v] = rank of lab[v]
// among the labels in use; the count goes to sc->n2.
bool lp_relabel(const int32_t* lab, int32_t n, int32_t* L, int32_t* flag_tmp, int32_t* scan_tmp, DevScalars* sc,
                hipStream_t s);

// ----------------------------------------------------------- CAPFOREST
struct CapforestArgs {
    DGraph g;
    const int64_t* lam;     // bound at launch
    int32_t* parent;        // union-find of contractible edges
    int32_t* claim;         // [n] shared visited array (round-tagged)
    int32_t tag;            // round tag for claim[]
    int32_t shared;         // 1: passes share the visited array
    int32_t passes;
    int32_t len_cap;        // scans per pass, 0 = unlimited
    int32_t pop_cap = 0;    // pops per pass, scanned or blacklisted (0 = unlimited)
    uint64_t seed;
    int32_t start;          // >= 0: every pass starts here (parity runs)
    int32_t* order;         // [passes * CF_HC] scanned vertices per pass
    int32_t* nscan;         // [passes]
    int64_t* alpha;         // [passes] smallest alpha of the pass (INT64_MAX: none)
    int32_t* alpha_len;     // [passes] prefix length of that alpha
    int64_t* lam_out;       // [passes] bound at the end of the pass
    unsigned long long* marks;
};
constexpr int CF_HC = 2048;     // per-pass LDS hash capacity (vertices touched)
bool capforest_passes(const CapforestArgs& a, hipStream_t s);
// Reduce per-pass results: smallest alpha (ties: smallest pass) and its
// prefix length into sc->best_alpha / best_pass / best_len.
bool capforest_reduce(const CapforestArgs& a, DevScalars* sc, hipStream_t s);

// One complete sequential pass (Algorithm 2's fallback): no capacity limit.
struct CompleteArgs {
    DGraph g;
    const int64_t* lam;
    int32_t* parent;
    int32_t start;
    int32_t tag;
    int32_t* st;            // [n] per-vertex state, tagged
    int64_t* r;             // [n]
    int64_t* l1;            // [n/64 + 1] block maxima of queued r
    int32_t* order;         // [n]
    int32_t* nscan;         // [1]
    int64_t* alpha;         // [1]
    int32_t* alpha_len;     // [1]
    int64_t* lam_out;       // [1]
    unsigned long long* marks;
};
bool capforest_complete(const CompleteArgs& a, hipStream_t s);

// Private passes with capped batches: `passes` workgroups, each one pass
// with its own dense state over the vertices (no shared visited array), so
// passes never fragment each other's traversal. All queued vertices whose
// key is capped at lam are scanned together as one batch.
struct PrivateArgs {
    DGraph g;
    const int64_t* lam;
    int32_t* parent;
    int32_t passes;
    int32_t len_cap;        // scans per pass, 0 = unlimited (complete pass)
    uint64_t seed;
    int32_t round;
    int32_t start;          // >= 0: every pass starts here
    int64_t stride;         // elements per pass in the per-pass arrays (>= n)
    int64_t region;         // elements of each per-pass array (0: passes * stride); passes * stride <= region
    int64_t region1;        // elements of l1 / dlist (0: passes * stride1)
    int32_t* st;            // [passes*stride] 0 new, 1 queued, 2 scanned, 3 in batch; all 0 between calls
    int64_t* r;             // [passes*stride] all 0 between calls
    int32_t* fifo;          // [passes*stride] capped vertices in crossing order
    int32_t* touched;       // [passes*stride]
    int32_t* order;         // [passes*stride] scanned vertices
    int64_t stride1;        // elements per pass in l1 / dlist (>= n/64 + 1)
    int64_t* l1;            // [passes*stride1] per 64-vertex block: max r of queued uncapped vertices
    int32_t* dlist;         // [passes*stride1] blocks whose l1 may be stale
    uint32_t* dbits;        // [passes*(stride1/32+1)] dirty flags of the blocks
    int32_t* nscan;         // [passes]
    int64_t* alpha;         // [passes]
    int32_t* alpha_len;     // [passes]
    int64_t* lam_out;       // [passes]
    unsigned long long* marks;
    int32_t* steps;         // [passes] batches + single pops (diagnostics)
    int64_t* diag;          // [passes*8] optional counters (nullptr: off)
    // Instance mode (batched solves, k_capforest_private only): pass p runs
    // on the vertex range [pvoff[p], pvoff[p+1]) of a union graph whose
    // ranges share no edge. st and r are then indexed by vertex id (one
    // array for all passes); fifo, touched and order start at pvoff[p]; l1
    // and dlist at pvoff[p]/64 + p; dbits at pvoff[p]/2048 + 2p. The bound
    // of pass p is plam[p]; passes with prun[p] = 0 or fewer than 3 vertices
    // do nothing (nscan 0, alpha INT64_MAX). pmarks[p] counts its marks.
    const int32_t* pvoff = nullptr;
    const int64_t* plam = nullptr;
    const uint8_t* prun = nullptr;
    unsigned long long* pmarks = nullptr;
    int32_t threads = 0;    // workgroup size of a pass (64..1024; 0 = 256 in instance mode, else 1024)
    // set by capforest_private: the level-1 index lives in LDS after the
    // l1_at level-2 entries (0: in HBM at l1)
    int32_t l1_at = 0;
};
constexpr size_t PRIV_BYTES_PER_VERTEX = 4 + 8 + 4 + 4 + 4 + 1;
bool capforest_private(const PrivateArgs& a, hipStream_t s, int32_t max_pass_n = 0);
// clear st/r of a fresh workspace region (once per solve)
bool capforest_private_reset(const PrivateArgs& a, hipStream_t s);

// The same private passes run level-synchronously over the whole GPU: per
// step, one launch picks every pass's batch, one processes the entries of
// all batches in tiles over all compute units, one finishes the step.
struct StepCtl {
    int32_t head, tail, tn, dn;
    int32_t nscan, done, bcount, bsingle;
    int32_t E, single_pending, best_len, steps;
    int32_t singles, maxbatch;
    int32_t streak, pad_;     // single pops since the last batch
    int64_t entries;
    int64_t alpha, best_alpha, lam, part, intra;
    unsigned long long marks;
};
struct StepArgs {
    PrivateArgs pv;
    StepCtl* ctl;       // [passes]
    int32_t* bpre;      // [passes*(bcap+1)] prefix of the batch's row lengths
    int32_t bcap;       // largest batch
    int32_t* single;    // [passes]
    int32_t* ptile;     // [passes+1]
    int32_t* running;   // [1]
    int64_t* popk;      // [passes*512] parts of the single-pop maximum
    int32_t* popv;
    int32_t max_singles;  // single pops in a row after which a pass stops (0: no bound)
    int32_t steps_run;    // out (host): whole-GPU steps the last call took
    int64_t scans_run;    // out (host): vertices its passes scanned
    unsigned long long* prof;  // algorithmic-byte counter (profiling) or nullptr
    // per pass, SPREAD partial sums 128 B apart of the step's intra-batch
    // weight ([0]) and marks ([1]), so the edge tiles do not all add to one
    // address; k_cfs_finish folds and clears them
    unsigned long long* spread;   // [passes * SPREAD * SPREAD_STRIDE]
    // vertices with at least HUB_LEN entries receive their entries through
    // HUB_SLOTS partial sums per pass (see k_cfs_hubfix)
    int32_t* hid;                 // [n] hub index or -1
    int32_t* hv;                  // [max_hubs] vertex of each hub
    int32_t* nhub;                // [1]
    int32_t max_hubs;             // >= entries / HUB_LEN
    unsigned long long* hacc;     // [passes * max_hubs * HUB_SLOTS * 2]
    int32_t* tinfo;               // [2 * max_tiles] pass and first batch vertex of each edge tile
    int64_t max_tiles;            // >= edge tiles of one step
};
constexpr int HUB_LEN = 512;
constexpr int HUB_SLOTS = 16;

// With cap (a non-default stream of the caller's device) and kernel timing
// off, each group of steps between two polls is captured once as a HIP
// graph on cap and replayed on s.
bool capforest_steps(StepArgs& a, int32_t* running_host, hipStream_t s, hipStream_t cap = nullptr);

// ------------------------------------------------------------ finisher
// Device-resident exact rounds for graphs of at most FIN_N vertices: one
// workgroup per graph runs every remaining round of Algorithm 2 (complete
// CAPFOREST pass with an LDS bucket queue or heap, union-find, contraction,
// collapsed-degree bounds) in one launch.
constexpr int FIN_N = 1024;
struct FinishArgs {
    DGraph g;                 // current graph (rows of every graph to finish)
    const int32_t* gvoff;     // [K+1] vertex ranges of the graphs (nullptr: one graph, all of g)
    const int32_t* glist;     // [count] ranges to finish (nullptr: 0..count-1)
    const int64_t* lam_in;    // [K] bound of each range at entry
    int64_t* lam_out;         // [K] bound at the end: lambda of the graph (may alias lam_in)
    int32_t* dropped;         // [K] 1 when the finisher lowered the bound
    uint8_t* fside;           // [g.n] side over the current vertices of dropped graphs
    int32_t* xcol[2];         // two scratch buffers for the contracted graphs
    int64_t* xw[2];
    int32_t xwindow;          // 1: a graph writes the scratch at its own window in g
                              // (buffers with g's capacity); 0: from position 0
                              // (buffers of at least FIN_N * (FIN_N - 1) entries,
                              // or g's entry count if smaller)
    uint64_t seed;
    int32_t* rounds;          // [K] rounds taken (may be nullptr)
    int32_t* err;             // [1] 0, or why a graph could not finish
    int32_t qmode;            // 0 buckets while lam < 2048 else heap, 1 buckets, 2 heap
    int32_t* qnext;           // [1] work-queue ticket, 0 at the launch
};
// count graphs of a.glist, by at most `cus` persistent workgroups that draw
// the graphs from a work queue (a.qnext must be 0)
bool finish_graphs(const FinishArgs& a, int32_t count, int32_t cus, hipStream_t s);
// one pass of the finisher's CAPFOREST (step ABI): see k_fin_pass
bool finish_pass(const DGraph& g, int32_t start, int32_t qmode, int64_t* lam_io, int64_t* best_alpha,
                 int32_t* parent, int32_t* order, int32_t* nscan, int32_t* best_len, hipStream_t s);

// -------------------------------------------------------- side tracking
bool map_update(int32_t* map0, const int32_t* L, int32_t n0, hipStream_t s);
// side[v0] = (map0[v0] == target)
bool side_from_vertex(uint8_t* side, const int32_t* map0, int32_t n0, const int32_t* target_dev,
                      hipStream_t s);
// flag[v] = 1 for v in order[0..len) (len read from device), else 0 (flag
// has n entries); then side[v0] = flag[map0[v0]]
bool side_from_prefix(uint8_t* side, const int32_t* map0, int32_t n0, uint8_t* flag, int32_t n,
                      const int32_t* order, const int32_t* len_dev, hipStream_t s);
// side[v0] = flag[map0[v0]] (every input vertex tracked)
bool side_from_flag(uint8_t* side, const int32_t* map0, int32_t n0, const uint8_t* flag, hipStream_t s);
// side[v0] = (root(map0[v0]) != root(0)) over a compressed parent array
bool side_from_components(uint8_t* side, const int32_t* parent, const int32_t* map, int32_t n0, hipStream_t s);

// ------------------------------------------------------- input handling
// Turn a user CSR (row_ptr) into padded form (off = row_ptr, len = diff).
bool csr_to_padded(const int32_t* row_ptr, int32_t n, int32_t* off, int32_t* len, hipStream_t s);
// Normalisation fast path: len[v] and deg[v] of every row of a user CSR,
// and *noncanon = 1 if some row is not already normal (targets strictly
// increasing, no loop, positive weights). With sc (device inputs) the same
// pass checks the input into sc->err as an mc_status code: row bounds in
// [0, nnz] and non-decreasing (a row that fails is not read), targets in
// range, non-negative weights, total weight below 2^62 (part: 1024 partial
// sums). With lp1 (n entries) it also writes every row's heaviest
// neighbour (smallest on ties; the row itself when it has none): the first
// label-propagation round from singleton labels when the input is normal.
bool canon_check(const int32_t* row_ptr, const int32_t* col, const int64_t* w, int32_t n, int32_t nnz, int32_t* len,
                 int64_t* deg, int32_t* noncanon, DevScalars* sc, unsigned long long* part, int32_t* lp1,
                 hipStream_t s);

// Smallest workspace mc_mincut accepts for a graph (small rounds keep their
// first pass count); mc_workspace_size adds room for one pass per compute
// unit.
size_t workspace_min_bytes(const mc_ctx* c, int32_t n, int32_t nnz);


// The library context (opaque to callers).
struct mc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    mc_options opt{};
    int cus = 256;
    DevScalars* hsc = nullptr;   // pinned readback slot
    int32_t tag = 0;             // round tag for visited arrays (never reset)
    void* prof = nullptr;        // kernel timing (mc_profile), owned by the solver file
    void* scratch = nullptr;     // device address of this GPU's static scratch (mc_mincut_static)
    hipStream_t cap_stream = nullptr;   // private stream the step graphs are captured on (made at first use)
    bool graphs_off = false;     // no graph capture (set while mc_mincut_static runs)
};
