/*
 * mincut.h -- exact global minimum cut on one AMD MI355X (gfx950).
 *
 * Problem (paper, Section 2 "Basic Concepts"): G = (V, E, c) undirected with
 * non-negative integer edge weights. A cut (A, V\A) has two non-empty sides;
 * its capacity is the total weight of the edges between them. The solver
 * returns lambda, the smallest capacity, and one side A of a cut attaining
 * it. The method is the exact algorithm summarised in Section 2.1 and
 * Algorithm 2 (bound from a label-propagation heuristic, reduction tests
 * that depend on the bound, parallel CAPFOREST of Algorithm 1, parallel
 * contraction, collapsed degrees as bounds), run as hand-written HIP
 * kernels. All arithmetic is 64-bit integer; results are exact.
 *
 * Conventions shared by every call:
 *  - A graph is a symmetric CSR: row_ptr[n+1] (int32, row_ptr[0] = 0,
 *    non-decreasing, row_ptr[n] = nnz), col[nnz] (int32, 0 <= col < n) and
 *    w[nnz] (int64, w >= 0). Every undirected edge {u,v} with u != v is
 *    listed in row u and in row v with the same weight. Loops (col[j] = row)
 *    are allowed and ignored; parallel entries are allowed and summed.
 *    Rows need not be sorted.
 *  - `location` says where the three arrays live: MC_HOST (pageable or
 *    pinned host memory) or MC_DEVICE (device memory of the context's GPU).
 *  - The caller owns every buffer it passes. The library keeps no caller
 *    pointer after a call returns (the server copies what it is given).
 *  - Every call returns an mc_status; on error the outputs are left
 *    untouched and mc_last_error() describes the failure (thread-local).
 *  - The sum of all weights over all nnz entries must be below 2^62 so that
 *    every degree, cut and doubled sum fits in int64 (MC_E_OVERFLOW).
 */
#ifndef MINCUT_H
#define MINCUT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MC_OK = 0,
    MC_E_INVALID_ARG = -1, /* null pointer, n < 2, bad option value, small workspace */
    MC_E_BAD_GRAPH = -2,   /* row_ptr not monotone, col out of range, negative w,
                              or (with validate) an asymmetric edge list */
    MC_E_OVERFLOW = -3,    /* total weight >= 2^62, or nnz >= 2^31 */
    MC_E_OOM = -4,         /* host allocation failed, or a server request does
                              not fit its HBM budget */
    MC_E_DEVICE = -5,      /* a HIP call failed */
    MC_E_NOT_READY = -6,   /* server ticket still running */
    MC_E_CANCELLED = -7,   /* server ticket was cancelled */
    MC_E_TIMEOUT = -8
} mc_status;

enum { MC_HOST = 0, MC_DEVICE = 1 };
enum { MC_CF_PRIVATE = 0, MC_CF_SHARED = 1, MC_CF_AUTO = 2 };

typedef struct {
    int32_t n;             /* vertices, >= 2 */
    int32_t nnz;           /* entries = row_ptr[n] */
    const int32_t* row_ptr;
    const int32_t* col;
    const int64_t* w;
    int32_t location;      /* MC_HOST or MC_DEVICE */
} mc_csr;

typedef struct {
    uint64_t seed;            /* start vertices of CAPFOREST passes */
    int32_t heuristic_min_n;  /* run the label-propagation bound only when
                                 n >= this (Section 4, session 2 item 2;
                                 default 10000; <= 0 disables it) */
    int32_t lp_iters;         /* label-propagation rounds per coarsening level
                                 (default 2) */
    int32_t pr_tri_deg_cap;   /* reduction tests 3 and 4 on edges whose two
                                 rows have at most this many entries (<= 64;
                                 default 16; 0 = off) in solves that do not
                                 run the heuristic; they stop for the rest
                                 of a solve once a round gains fewer than one
                                 contraction per 100 vertices */
    int32_t capforest_passes; /* concurrent CAPFOREST passes per round
                                 (0 = automatic) */
    int32_t pass_len_cap;     /* scans per pass (0 = automatic; < 0 = until
                                 the pass's queue empties) */
    int32_t capforest_mode;   /* visited-array policy (Section 4, parallel
                                 session (1)). MC_CF_PRIVATE: passes with
                                 private visited state that scan capped
                                 vertices in batches; MC_CF_SHARED: passes
                                 that share one visited array (Algorithm 1 as
                                 printed); MC_CF_AUTO (default): on the first
                                 round of each size regime (at least / below
                                 levels_min_n vertices) that runs CAPFOREST,
                                 a short probe of shared passes (four per
                                 compute unit, 32 pops each) runs first; if
                                 it contracts fewer than one vertex in 1024
                                 private passes are kept, otherwise private
                                 passes of at most 4096 scans run in the same
                                 round and the form with more marks per
                                 millisecond is kept */
    int32_t levels_min_n;     /* current graphs with at least this many
                                 vertices advance all private passes in
                                 whole-GPU steps; smaller ones run one
                                 workgroup per pass (0 = default 65536) */
    int32_t deterministic;    /* 1: one sequential pass per round, one vertex
                                 at a time, smallest id first on ties; the
                                 whole solve then does not depend on timing */
    int32_t validate;         /* 1: check symmetry of host inputs */
    int32_t batch_pass_threads; /* threads of each graph's CAPFOREST pass in
                                 the batched and served forms: 64, 128, 256,
                                 512 or 1024 (0 = 256) */
    int32_t batch_lp;         /* label-propagation bound at admission in the
                                 batched and served forms: 0 = when
                                 heuristic_min_n > 0, 1 = always, 2 = never */
    int32_t finish_max_n;     /* current graphs with at most this many
                                 vertices (<= 1024) finish all their remaining
                                 rounds in one launch, one workgroup per graph
                                 (0 = 1024; < 0 = never) */
    int32_t queue;            /* priority queue of the finisher's CAPFOREST
                                 passes (Section 2.1 "Bounded priority
                                 queues"): 0 = buckets while the bound is
                                 below 2048, else a binary heap; 1 = buckets;
                                 2 = heap (the largest key, then the
                                 smallest id, as the sequential pass) */
    int32_t contract_mode;    /* edge merge of the contractions (Section 2:
                                 parallel edges summed, loops dropped) in
                                 mc_mincut and the step calls: 0 = hashing by
                                 contracted vertex (default); 1 = a radix
                                 sort of the contracted entries and a
                                 segmented reduction (rows sorted by target;
                                 the workspace grows by about 40 bytes per
                                 entry). The batched and served forms always
                                 hash. */
} mc_options;

typedef struct {
    int32_t rounds;              /* exact-phase rounds */
    int32_t heuristic_levels;    /* coarsening levels of the bound heuristic */
    int64_t lambda_min_degree;   /* bound from the minimum degree */
    int64_t lambda_heuristic;    /* bound after the heuristic (-1: not run) */
    int64_t marks_pr;            /* edges unioned by the reduction tests */
    int64_t marks_capforest;     /* edges unioned by CAPFOREST */
    int32_t fallback_passes;     /* sequential CAPFOREST runs (Algorithm 2) */
    int32_t n_input;             /* vertices after normalisation */
    int64_t m_input;             /* undirected edges after normalisation */
    double ms_total;             /* wall time of the call */
    int32_t rounds_pr_only;      /* rounds whose reduction tests alone at least
                                    halved the graph (CAPFOREST left to the
                                    next round) */
    int32_t input_normal;        /* 1: the input was already a simple graph
                                    with sorted rows and was used in place */
    int64_t marks_tri;           /* of marks_pr: edges unioned by tests 3, 4 */
    int32_t finish_rounds;       /* of rounds: rounds run inside the finisher
                                    (one launch for all of them) */
} mc_stats;

typedef struct mc_ctx mc_ctx;

/* Default options (seed 1, heuristic at n >= 10000, 2 LP rounds, automatic
 * pass count and length, private passes, no validation). */
void mc_default_options(mc_options* opt);

/* Create a context on HIP device `device` issuing all work on `hip_stream`
 * (a hipStream_t; NULL = the default stream). `opt` may be NULL. The
 * context holds pinned host scratch of a few KB; device memory always comes
 * from the caller's workspace. */
mc_status mc_ctx_create(int device, void* hip_stream, const mc_options* opt, mc_ctx** out);
mc_status mc_ctx_destroy(mc_ctx* ctx);
mc_status mc_ctx_set_options(mc_ctx* ctx, const mc_options* opt);

/* Device workspace bytes that mc_mincut needs for a graph with n vertices
 * and nnz entries. This includes room for one CAPFOREST pass per compute
 * unit on small graphs (rounds that contract less than a tenth of their
 * vertices raise the pass count to that); a smaller workspace that holds
 * the first count (32 passes) is accepted too, and the solve then keeps 32. */
mc_status mc_workspace_size(const mc_ctx* ctx, int32_t n, int32_t nnz, size_t* bytes);

/* Solve one graph (Algorithm 2). `dev_workspace` is device memory of at
 * least mc_workspace_size bytes, 256-byte aligned. On success *lambda is the
 * minimum cut and, if side != NULL, side[v] in {0,1} (host memory, n bytes)
 * marks one side of a minimum cut, with side[0] = 0; when lambda = 0 (the
 * graph is disconnected) side[v] = 1 exactly for the vertices outside the
 * component of vertex 0. `st` may be NULL. Synchronises the stream. */
mc_status mc_mincut(mc_ctx* ctx, const mc_csr* g, void* dev_workspace, size_t ws_bytes,
                    int64_t* lambda, uint8_t* side, mc_stats* st);

/* mc_mincut without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc. The call runs
 * exactly mc_mincut (same options, results and error behaviour) on a
 * static scratch array of 64 MiB that the library keeps on each GPU until
 * the process ends (its address is fetched when the first context on the
 * device is created); it calls no hipMalloc, hipFree or other allocating
 * routine, and kernel timing (mc_profile) is suspended for the call. Graphs
 * whose smallest workspace (32 passes on small rounds) exceeds 64 MiB get
 * MC_E_INVALID_ARG before any device work. Every call on one GPU uses that GPU's one array, which keeps
 * the last call's contents (the solve initialises all it reads): calls that
 * overlap on one GPU, from any thread or context, race and must not be
 * made. */
mc_status mc_mincut_static(mc_ctx* ctx, const mc_csr* g, int64_t* lambda, uint8_t* side, mc_stats* st);

/* Batched solves: k graphs (all in host memory or all in device memory,
 * together fewer than 2^30 vertices and 2^30 entries) solved in one call,
 * with one set of launches per round of Algorithm 2 for all of them (the
 * graphs are laid side by side as one union graph; each keeps its own
 * bound, CAPFOREST pass and side). Results are those of mc_mincut:
 * lambdas[i] (host, k values) is graph i's minimum cut; if sides != NULL and
 * sides[i] != NULL, sides[i] (host, n_i bytes) receives one side of it with
 * sides[i][0] = 0.
 * Every graph is checked on its own before anything is solved: host graphs
 * as mc_check_graph does (with symmetry when the context's validate option
 * is 1), device graphs on the device (the same checks without symmetry);
 * the 2^62 weight bound applies to each graph's own total.
 *  - per_graph != NULL (host, k values): per_graph[i] receives graph i's
 *    status; graphs that fail their checks are skipped (their lambdas[i]
 *    and sides[i] stay untouched) and the others are solved; the call
 *    returns MC_OK unless the call itself fails.
 *  - per_graph == NULL: the first graph that fails its checks fails the
 *    whole call with its status, before anything is solved.
 * On a failing call every output is left untouched. When batch_lp selects
 * it, every graph first goes through the label-propagation heuristic's
 * coarsening (LP rounds and cluster contraction while the graphs shrink;
 * the smallest collapsed degree of each level bounds lambda), all graphs in
 * the same launches, but without its reduction tests and exact finish.
 * Synchronises the stream. */
mc_status mc_batch_workspace_size(const mc_ctx* ctx, int32_t k, const mc_csr* graphs, size_t* bytes);
mc_status mc_mincut_batch(mc_ctx* ctx, int32_t k, const mc_csr* graphs, void* dev_workspace, size_t ws_bytes,
                          int64_t* lambdas, uint8_t* const* sides, mc_status* per_graph);

/* Autotuner of the batched form. Solves a sample of the batch (`sample`
 * graphs: the sample/8 largest by entries, since a batch takes as long as
 * its largest graphs' passes, and the rest spread evenly over the k given;
 * all of them when sample <= 0 or >= k) twice per candidate setting, after
 * one untimed run, times each (wall clock around the synchronised call,
 * the faster of the two), and stores the fastest setting in the context's
 * options (the other options are left as they are). Two stages: every pass
 * workgroup size of batch_pass_threads, with and without the admission
 * bound of batch_lp; then, with the best of those, the finisher's size
 * limit (finish_max_n 1024, 512, 256, or no finisher) and its queue (queue
 * 0, 1, 2 at the best limit). The results of the sample solves are
 * discarded; a setting changes only the speed, never a result.
 * dev_workspace must hold mc_batch_workspace_size of the whole batch (the
 * sample needs less). On error the options are left unchanged. */
#define MC_TUNE_MAX 16
typedef struct {
    int32_t pass_threads;      /* chosen batch_pass_threads */
    int32_t lp;                /* chosen batch_lp (1 or 2) */
    int32_t sample;            /* graphs in the timed sample */
    int32_t candidates;        /* settings timed */
    int32_t cand_threads[MC_TUNE_MAX];
    int32_t cand_lp[MC_TUNE_MAX];
    double cand_ms[MC_TUNE_MAX];  /* wall time of each setting on the sample */
    int32_t finish_max_n;      /* chosen finish_max_n (-1: no finisher) */
    int32_t queue;             /* chosen queue */
    int32_t cand_finish[MC_TUNE_MAX];
    int32_t cand_queue[MC_TUNE_MAX];
} mc_tuning;
mc_status mc_batch_autotune(mc_ctx* ctx, int32_t k, const mc_csr* graphs, void* dev_workspace, size_t ws_bytes,
                            int32_t sample, mc_tuning* out);

/* Served form: a request loop with continuous batching. The server holds
 * one device allocation of hbm_bytes (made at create) for the graphs in
 * flight. mc_server_submit checks a host graph (as mc_check_graph, with
 * symmetry when the context's validate option is 1) and copies it into a
 * queue. Each mc_server_step
 *  - collects large requests whose solve ended and drops requests that
 *    were cancelled or passed their deadline;
 *  - admits queued requests in arrival order: requests with n >=
 *    solo_min_n start on a free solo slot (mc_mincut on a worker thread
 *    with its own context and non-blocking stream, so its kernels overlap
 *    the engine's on the device and no other request waits for it); the
 *    others join the engine while they fit (graphs in flight <=
 *    max_inflight, vertices and entries within what the budget holds);
 *  - runs one round of Algorithm 2 for every graph in the engine (admitted
 *    graphs join graphs already half way through their rounds, in the same
 *    launches) and collects finished graphs.
 * A graph's result does not depend on the others in flight. Calls on one
 * server must not overlap (one thread at a time). */
typedef struct {
    size_t hbm_bytes;          /* device memory of the server (>= 64 MiB) */
    int32_t max_inflight;      /* graphs in the rounds at once (0: 1024) */
    int32_t max_request_n;     /* largest request, vertices (0: 2^20) */
    int64_t max_request_nnz;   /* largest request, entries (0: 2^25) */
    int32_t solo_min_n;        /* requests with at least this many vertices
                                  are solved by mc_mincut (whole GPU, full
                                  heuristic) on a solo slot, from a
                                  workspace set aside in the budget
                                  (0: 65536) */
    int32_t solo_slots;        /* large requests solved at once, each with a
                                  workspace of its own (0: 1; at most 8) */
    double deadline_ms;        /* a request not done this long after its
                                  submission is answered with MC_E_TIMEOUT;
                                  checked at every step (a queued request is
                                  never admitted, one in the engine leaves
                                  it at the next round, a solo solve is
                                  reported as timed out when it ends late);
                                  0: no deadline */
} mc_server_opts;
typedef struct {
    double t_submit_ms, t_admit_ms, t_done_ms;   /* since the server was created */
    int32_t rounds;                              /* engine rounds the graph took
                                                    part in (0 for a solo solve) */
} mc_req_stats;
typedef struct mc_server mc_server;
mc_status mc_server_create(mc_ctx* ctx, const mc_server_opts* opts, mc_server** out);
mc_status mc_server_destroy(mc_server* srv);
/* Check and queue a copy of host graph g; *ticket identifies it. The
 * checks' error (MC_E_INVALID_ARG, MC_E_BAD_GRAPH, MC_E_OVERFLOW) is
 * returned at once and nothing is queued; MC_E_OOM when the graph alone
 * exceeds what the server can ever admit. */
mc_status mc_server_submit(mc_server* srv, const mc_csr* g, uint64_t* ticket);
/* Collect, admit, run one round, collect. *in_flight / *queued (may be
 * NULL): requests running (engine and solo slots) and waiting after the
 * step. Synchronises the engine's stream. A device failure of an admission
 * or a round fails the requests it touched (their poll returns the error)
 * and is returned; the other requests go on. */
mc_status mc_server_step(mc_server* srv, int32_t* in_flight, int32_t* queued);
/* MC_OK with lambda, side (host, n bytes, side[0] = 0; may be NULL) and
 * timing once done (the ticket is then released); MC_E_NOT_READY before;
 * MC_E_CANCELLED for a cancelled request, MC_E_TIMEOUT for one past its
 * deadline and the failure's status for a failed one (each released). */
mc_status mc_server_poll(mc_server* srv, uint64_t ticket, int64_t* lambda, uint8_t* side, mc_req_stats* st);
/* *state: 0 queued, 1 in flight, 2 done (poll returns it), 3 cancelled,
 * 4 failed, 5 timed out. */
mc_status mc_server_state(const mc_server* srv, uint64_t ticket, int32_t* state);
/* Cancel a request: a queued one is never admitted, one in the engine
 * leaves it at the next step, a solo solve is reported as cancelled when it
 * ends. */
mc_status mc_server_cancel(mc_server* srv, uint64_t ticket);
/* Capacity the budget gives (entries, vertices, graphs in flight, bytes). */
mc_status mc_server_capacity(const mc_server* srv, int64_t* entries, int32_t* vertices, int32_t* graphs,
                             size_t* bytes);

/* Kernel timing, for measurement. While profiling is on, every launch of
 * the kernels below made by mc_mincut on this context is bracketed by two
 * HIP events on the context's stream, and the algorithmic bytes of the
 * launches (what the method must read and write: entries scanned, labels
 * gathered, rows written; no hash-table or scratch traffic) are counted.
 * Timing adds two event records per timed launch. */
enum {
    MC_K_CAPFOREST_EDGES = 0,  /* k_cfs_edges: edges of the CAPFOREST batches (Algorithm 1) */
    MC_K_CONTRACT_MERGE = 1,   /* k_merge_small: contraction of small groups */
    MC_K_CONTRACT_BIG = 2,     /* k_big_insert: contraction of large groups */
    MC_K_GROUP_COUNT = 3,      /* k_group_count: members per contracted vertex */
    MC_K_GROUP_SCATTER = 4,    /* k_group_scatter: members grouped by label */
    MC_K_PR12 = 5,             /* k_pr12: reduction tests 1 and 2 */
    MC_K_CONNECT_LINK = 6,     /* k_uf_link_rest: connectivity unions */
    MC_K_LP_SMALL = 7,         /* k_lp_flat: label-propagation round, rows of <= 256 entries
                                  (k_lp_small instead when the graph has 2^27 - 1 vertices or
                                  more, or a degree of 2^32 or more) */
    MC_K_LP_FIRST = 8,         /* k_lp_first: first label-propagation round (from singletons) of
                                  the coarse levels; a normal input's own first round is taken in
                                  the input check's pass (k_canon), untimed */
    MC_K_MID_MERGE = 9,        /* k_mid_merge<2048>, k_mid_merge<4096>: contraction of groups of
                                  513..2048 entries */
    MC_K_PR1_FIRST = 10,       /* k_pr1_first: link rounds of every row's first and second test-1
                                  entries */
    MC_K_PR1_REST = 11,        /* k_pr1_trees (at most 255 trees) or k_pr1_rest: linking of the
                                  trees those rounds leave */
    MC_K_COUNT = 12
};
typedef struct {
    char name[32];      /* kernel symbol name */
    int64_t launches;   /* timed launches since profiling was switched on */
    double ms;          /* summed time between each launch's two events */
    double bytes;       /* summed algorithmic bytes of those launches */
} mc_kernel_time;

/* on != 0: switch timing on and zero the totals (the first call allocates
 * 96 KiB of device counters, kept until mc_ctx_destroy); on = 0:
 * switch it off and keep the totals. */
mc_status mc_profile(mc_ctx* ctx, int32_t on);
/* Totals of one kernel (kernel in [0, MC_K_COUNT)); synchronous. */
mc_status mc_profile_read(mc_ctx* ctx, int32_t kernel, mc_kernel_time* out);

/* Rounds of the last mc_mincut made while timing was on, in order: kind 1
 * for a coarsening level of the bound heuristic (LP rounds, cluster
 * contraction, reduction tests and their contraction), kind 2 for a round
 * of Algorithm 2 on the heuristic's coarse graph, kind 0 for a round of
 * Algorithm 2 on the input graph. n/m are the vertices and CSR entries
 * before and after the round; ms is the device time from the round's first
 * launch to its last (HIP events on the context's stream, so the gaps
 * between launches count). *count is always written; out only when
 * 0 <= i < *count. Synchronous. */
typedef struct {
    int32_t kind;
    int32_t n_in;
    int64_t m_in;
    int32_t n_out;
    int64_t m_out;
    double ms;
} mc_round_time;
mc_status mc_profile_round(mc_ctx* ctx, int32_t i, mc_round_time* out, int32_t* count);

/* Check a host graph (location MC_HOST) exactly as mc_mincut does before it
 * touches the device: MC_E_INVALID_ARG for a NULL graph or pointer, n < 2 or
 * nnz < 0; MC_E_BAD_GRAPH for row_ptr[0] != 0, row_ptr[n] != nnz, a
 * decreasing row_ptr, a target outside [0, n) or a negative weight;
 * MC_E_OVERFLOW for a total weight of 2^62 or more; with symmetric != 0,
 * MC_E_BAD_GRAPH when some folded pair (u, v, s) (loops dropped, parallel
 * entries summed) has no matching (v, u, s). The input definition is that of
 * Section 2 "Basic Concepts" (undirected, non-negative integer weights).
 * Reads the arrays only; needs no GPU and no context. */
mc_status mc_check_graph(const mc_csr* g, int32_t symmetric);

/* Thread-local description of the last error (never NULL). */
const char* mc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MINCUT_H */
