/*
 * mincut_steps.h -- the individual steps of the exact minimum-cut round,
 * exported so each kernel can be checked on its own against the CPU oracle.
 *
 * Every call here takes device pointers only (memory of the context's GPU),
 * runs on the context's stream, and synchronises that stream before it
 * returns. Graphs are in the library's padded-CSR form (mc_dgraph): row v
 * occupies col/w[off[v] .. off[v]+len[v]); rows are disjoint and may leave
 * gaps; rows are not sorted. Workspaces come from the caller and must be at
 * least mc_step_ws_size bytes (256-byte aligned). Errors leave outputs
 * unspecified and set mc_last_error().
 */
#ifndef MINCUT_STEPS_H
#define MINCUT_STEPS_H

#include "mincut.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n;      /* vertices */
    int64_t cap;    /* capacity of col/w in entries */
    int32_t* off;   /* [n] */
    int32_t* len;   /* [n] */
    int32_t* col;   /* [cap] */
    int64_t* w;     /* [cap] */
    int64_t* deg;   /* [n] sum of the row's weights (written by contraction) */
} mc_dgraph;

/* Workspace bytes for any step on a graph of at most n vertices and cap
 * entries with up to `passes` concurrent CAPFOREST passes. */
mc_status mc_step_ws_size(int32_t n, int64_t cap, int32_t passes, size_t* bytes);

/* Contraction (paper, Section 2 "Basic Concepts"; Algorithm 2's contract
 * step): vertex g of dst stands for {v : labels[v] = g}, g in [0, n2);
 * labels == NULL means the identity (n2 = n), which folds loops, parallel
 * entries and zero weights away. dst->cap must be at least the sum of
 * src->len. Writes dst off/len/col/w/deg; *dmin / *dmin_arg (host) receive
 * the minimum degree of dst and its smallest vertex. */
mc_status mc_step_contract(mc_ctx* ctx, const mc_dgraph* src, const int32_t* labels, int32_t n2,
                           mc_dgraph* dst, void* ws, size_t ws_bytes, int64_t* dmin, int32_t* dmin_arg);

/* Canonical components of the pairs (a[i], b[i]) on [0,n): labels[v] is
 * the rank of the smallest vertex of v's component among all component
 * minima; *n2 (host) receives the component count. */
mc_status mc_step_components(mc_ctx* ctx, int32_t n, int64_t npairs, const int32_t* a, const int32_t* b,
                             int32_t* labels, int32_t* n2, void* ws, size_t ws_bytes);

/* Padberg-Rinaldi tests 1 and 2 with bound lam (reduction tests of Section
 * 2.1): flag1[j] = 1 iff entry j has weight >= lam; ptr2[v] = heaviest
 * neighbour (smallest id on ties) if twice its weight is >= deg[v], else
 * -1. Also unions both kinds of edges and returns the canonical labels of
 * the result (labels[n], *n2). flag1 / ptr2 may be NULL. g->deg must be
 * set. */
mc_status mc_step_pr12(mc_ctx* ctx, const mc_dgraph* g, int64_t lam, uint8_t* flag1, int32_t* ptr2,
                       int32_t* labels, int32_t* n2, void* ws, size_t ws_bytes);

/* Padberg-Rinaldi tests 3 and 4 (the other two local reduction tests of
 * Section 2.1; App. A) on the candidate edges {v,x} whose two rows both have
 * at most D entries (0 <= D <= 64). g must be a simple graph (a normalised
 * or contracted one) with deg set. With s = c(v,x) + sum over common
 * neighbours u of min(c(v,u), c(x,u)): test 4 holds when s >= lam; test 3
 * when some common u has 2 (c(v,x) + c(v,u)) >= c(v) and
 * 2 (c(v,x) + c(x,u)) >= c(x). Test-4 edges are unioned; of the test-3
 * edges only mutual smallest partners that touch no test-2 pointer of ptr2
 * ([n] device array, -1 = none, as mc_step_pr12 writes it) are unioned.
 * Outputs: flag4[entry] (may be NULL), acc3[v] = accepted test-3 partner or
 * -1 (may be NULL), canonical labels of the unions (labels[n], *n2). */
mc_status mc_step_pr34(mc_ctx* ctx, const mc_dgraph* g, int64_t lam, int32_t D, const int32_t* ptr2,
                       uint8_t* flag4, int32_t* acc3, int32_t* labels, int32_t* n2, void* ws, size_t ws_bytes);

/* One synchronous label-propagation round, the clustering step of the
 * bound heuristic (Section 2.1, "Lowering the upper bound"): lab_out[v] is
 * the label (among lab_in of v's neighbours, loops ignored) with the
 * largest total edge weight to v, except that v keeps lab_in[v] unless
 * another label is strictly heavier; ties among other labels go to the
 * smallest label. lab_in / lab_out: [g->n] labels in [0, n), distinct
 * arrays. lab_in NULL means singleton labels (lab_in[v] = v), the
 * heuristic's first round, taken by a streaming pass that needs g normal
 * (as contraction writes it: no loop, no parallel entries, positive
 * weights). */
mc_status mc_step_lp(mc_ctx* ctx, const mc_dgraph* g, const int32_t* lab_in, int32_t* lab_out, void* ws,
                     size_t ws_bytes);

/* CAPFOREST (Algorithm 1), in one of three forms (mode):
 *  MC_STEP_CF_SHARED (0): `passes` concurrent passes, one wavefront each,
 *     state in LDS (at most 1536 vertices touched per pass), sharing the
 *     visited array iff shared = 1; start >= 0 forces every pass to begin
 *     there;
 *  MC_STEP_CF_SEQUENTIAL (1): one pass from `start`, one vertex at a time,
 *     largest key and smallest id first, no capacity limit (Algorithm 2's
 *     sequential fallback; the deterministic reference form);
 *  MC_STEP_CF_PRIVATE (2): `passes` passes, one workgroup each, private
 *     visited state in HBM, capped vertices scanned in batches;
 *  MC_STEP_CF_LEVELS (3): the same passes advanced in steps, each step's
 *     edges processed by all compute units;
 *  MC_STEP_CF_BUCKET (4) / MC_STEP_CF_HEAP (5): one complete pass from
 *     `start` of the small-graph finisher (n <= 1024), its priority queue
 *     in LDS (Section 2.1 "Bounded priority queues"): one LIFO bucket per
 *     attainable key, or a binary heap ordered by the largest key and then
 *     the smallest id (the order of MC_STEP_CF_SEQUENTIAL).
 * Each pass stops after len_cap scans (0: none). Outputs: canonical labels
 * of the marked edges (labels[n], *n2), the scan order of pass 0 (order[n],
 * *nscan), the smallest alpha over the passes with its prefix length
 * (*best_alpha = INT64_MAX if none), and the bound after pass 0 (*lam_out). */
enum { MC_STEP_CF_SHARED = 0, MC_STEP_CF_SEQUENTIAL = 1, MC_STEP_CF_PRIVATE = 2, MC_STEP_CF_LEVELS = 3,
       MC_STEP_CF_BUCKET = 4, MC_STEP_CF_HEAP = 5 };
mc_status mc_step_capforest(mc_ctx* ctx, const mc_dgraph* g, int64_t lam, int32_t start, int32_t mode,
                            int32_t passes, int32_t shared, int32_t len_cap, int32_t* labels, int32_t* n2,
                            int32_t* order, int32_t* nscan, int64_t* best_alpha, int32_t* best_len,
                            int64_t* lam_out, void* ws, size_t ws_bytes);

#ifdef __cplusplus
}
#endif
#endif /* MINCUT_STEPS_H */
