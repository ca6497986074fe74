/*
 * CPU oracle for the exact minimum-cut solver -- TEST INFRASTRUCTURE ONLY.
 *
 * Nothing on the product path may link or call this file. It is used by the
 * tests, by the smoke check and by the CPU-baseline leg of the benchmark.
 * It shares no code with the GPU library: plain, single-threaded C written
 * for obviousness, not speed.
 *
 * Problem (paper, Section 2 "Basic Concepts"): an undirected graph with
 * non-negative integer edge weights; a cut (A, V\A) has both sides
 * non-empty; its capacity is the weight of the crossing edges; lambda is the
 * smallest capacity. Loops never cross a cut and parallel edges add up, so
 * every routine first folds the input into a simple graph.
 *
 * Whole-problem solvers (all return lambda and one minimum side):
 *   orc_brute        -- the definition, every cut enumerated (n <= 24)
 *   orc_stoer_wagner -- Stoer and Wagner (J. ACM 1997), which the paper
 *                       names as a simpler variant of the same bound and
 *                       used as its independent checker (Appendix A, B)
 *   orc_noi          -- the contraction algorithm of Section 2.1: repeated
 *                       full CAPFOREST scans with keys bounded by the
 *                       current bound, contraction of every marked edge,
 *                       collapsed degrees as bounds, until <= 2 vertices
 * Step oracles (pure functions used for bit-exact kernel parity):
 *   orc_degrees, orc_contract, orc_components, orc_pr12, orc_pr34, orc_lp,
 *   orc_capforest_pass
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------- simple graphs */
typedef struct {
    int32_t n;
    int64_t* off;   /* n+1 */
    int32_t* adj;   /* off[n] */
    int64_t* wt;    /* off[n] */
} sgraph;

static void sg_free(sgraph* g) { free(g->off); free(g->adj); free(g->wt); memset(g, 0, sizeof(*g)); }

static int cmp_i64(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

/* Fold an arbitrary symmetric CSR into a simple graph: loops dropped,
 * parallel entries summed, zero-weight pairs dropped, rows sorted. Each
 * row is folded on its own (so the input must list every edge in both rows,
 * which the symmetric CSR convention guarantees). */
static int sg_from_csr(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w, sgraph* g) {
    g->n = n;
    g->off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t nnz = rp[n];
    g->adj = (int32_t*)malloc((size_t)(nnz + 1) * sizeof(int32_t));
    g->wt = (int64_t*)malloc((size_t)(nnz + 1) * sizeof(int64_t));
    int64_t* acc = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* seen = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
    int32_t* list = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
    if (!g->off || !g->adj || !g->wt || !acc || !seen || !list) {
        free(acc); free(seen); free(list); sg_free(g); return -1;
    }
    for (int32_t i = 0; i < n; i++) seen[i] = -1;
    int64_t pos = 0;
    for (int32_t v = 0; v < n; v++) {
        int32_t cnt = 0;
        for (int64_t j = rp[v]; j < rp[v + 1]; j++) {
            int32_t x = col[j];
            if (x == v) continue;
            if (seen[x] != v) { seen[x] = v; acc[x] = 0; list[cnt++] = x; }
            acc[x] += w[j];
        }
        /* sort the distinct targets (insertion into a sorted copy via qsort) */
        int64_t* tmp = (int64_t*)malloc((size_t)(cnt + 1) * sizeof(int64_t));
        if (!tmp) { free(acc); free(seen); free(list); sg_free(g); return -1; }
        for (int32_t k = 0; k < cnt; k++) tmp[k] = list[k];
        qsort(tmp, (size_t)cnt, sizeof(int64_t), cmp_i64);
        for (int32_t k = 0; k < cnt; k++) {
            int32_t x = (int32_t)tmp[k];
            if (acc[x] == 0) continue;
            g->adj[pos] = x;
            g->wt[pos] = acc[x];
            pos++;
        }
        free(tmp);
        g->off[v + 1] = pos;
    }
    free(acc); free(seen); free(list);
    return 0;
}

static int64_t sg_degree(const sgraph* g, int32_t v) {
    int64_t s = 0;
    for (int64_t j = g->off[v]; j < g->off[v + 1]; j++) s += g->wt[j];
    return s;
}

/* capacity of the cut given by side[] (1 = side A) over the raw input */
int64_t orc_cut_value(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w,
                      const uint8_t* side) {
    int64_t s = 0;
    for (int32_t v = 0; v < n; v++)
        for (int64_t j = rp[v]; j < rp[v + 1]; j++)
            if (side[v] && !side[col[j]]) s += w[j];
    return s;
}

/* flip side[] so that vertex 0 is on side 0 */
static void canon_side(int32_t n, uint8_t* side) {
    if (n > 0 && side[0])
        for (int32_t v = 0; v < n; v++) side[v] ^= 1;
}

/* --------------------------------------------------------- brute force */
/* Every set S with vertex 0 outside it and 1 <= |S| <= n-1 is visited once
 * in Gray-code order; the capacity is updated incrementally from conn[x] =
 * c(x, S). The first strict minimum in that order is reported. */
int64_t orc_brute(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w, uint8_t* side) {
    if (n < 2 || n > 24) return -1;
    int64_t* A = (int64_t*)calloc((size_t)n * n, sizeof(int64_t));
    int64_t* conn = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    int64_t* deg = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    if (!A || !conn || !deg) { free(A); free(conn); free(deg); return -2; }
    for (int32_t v = 0; v < n; v++)
        for (int64_t j = rp[v]; j < rp[v + 1]; j++)
            if (col[j] != v) A[(int64_t)v * n + col[j]] += w[j];
    for (int32_t v = 0; v < n; v++)
        for (int32_t x = 0; x < n; x++) deg[v] += A[(int64_t)v * n + x];
    uint32_t mask = 0, best_mask = 0;
    int64_t cut = 0, best = -1;
    uint64_t total = (uint64_t)1 << (n - 1);
    for (uint64_t i = 1; i < total; i++) {
        int b = __builtin_ctzll(i);
        int32_t x = b + 1;
        const int64_t* row = A + (int64_t)x * n;
        if (!(mask & (1u << b))) {
            cut += deg[x] - 2 * conn[x];
            mask |= 1u << b;
            for (int32_t y = 0; y < n; y++) conn[y] += row[y];
        } else {
            mask &= ~(1u << b);
            for (int32_t y = 0; y < n; y++) conn[y] -= row[y];
            cut -= deg[x] - 2 * conn[x];
        }
        if (best < 0 || cut < best) { best = cut; best_mask = mask; }
    }
    if (side) {
        side[0] = 0;
        for (int32_t x = 1; x < n; x++) side[x] = (best_mask >> (x - 1)) & 1;
    }
    free(A); free(conn); free(deg);
    return best;
}

/* minimum s-t cut by enumeration (n <= 24): used to pin CAPFOREST marks */
int64_t orc_brute_st(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w,
                     int32_t s, int32_t t) {
    if (n < 2 || n > 24 || s == t) return -1;
    int64_t best = -1;
    uint64_t total = (uint64_t)1 << n;
    for (uint64_t m = 0; m < total; m++) {
        if (!((m >> s) & 1) || ((m >> t) & 1)) continue;
        int64_t c = 0;
        for (int32_t v = 0; v < n; v++) {
            if (!((m >> v) & 1)) continue;
            for (int64_t j = rp[v]; j < rp[v + 1]; j++)
                if (!((m >> col[j]) & 1)) c += w[j];
        }
        if (best < 0 || c < best) best = c;
    }
    return best;
}

/* ---------------------------------------------------------- max-heap */
typedef struct {
    int32_t size;
    int32_t* item;   /* heap position -> vertex */
    int32_t* pos;    /* vertex -> heap position, -1 if absent */
    int64_t* key;    /* vertex -> key */
} mheap;

static int mh_init(mheap* h, int32_t n) {
    h->size = 0;
    h->item = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
    h->pos = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
    h->key = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    if (!h->item || !h->pos || !h->key) return -1;
    for (int32_t i = 0; i < n; i++) h->pos[i] = -1;
    return 0;
}
static void mh_free(mheap* h) { free(h->item); free(h->pos); free(h->key); }
/* priority order: larger key first, then smaller vertex id */
static int mh_before(const mheap* h, int32_t a, int32_t b) {
    return h->key[a] > h->key[b] || (h->key[a] == h->key[b] && a < b);
}
static void mh_swap(mheap* h, int32_t i, int32_t j) {
    int32_t a = h->item[i], b = h->item[j];
    h->item[i] = b; h->item[j] = a;
    h->pos[b] = i; h->pos[a] = j;
}
static void mh_up(mheap* h, int32_t i) {
    while (i > 0) {
        int32_t p = (i - 1) / 2;
        if (!mh_before(h, h->item[i], h->item[p])) break;
        mh_swap(h, i, p);
        i = p;
    }
}
static void mh_down(mheap* h, int32_t i) {
    for (;;) {
        int32_t l = 2 * i + 1, r = l + 1, b = i;
        if (l < h->size && mh_before(h, h->item[l], h->item[b])) b = l;
        if (r < h->size && mh_before(h, h->item[r], h->item[b])) b = r;
        if (b == i) break;
        mh_swap(h, i, b);
        i = b;
    }
}
/* insert v or raise its key to k */
static void mh_set(mheap* h, int32_t v, int64_t k) {
    if (h->pos[v] < 0) {
        h->key[v] = k;
        h->item[h->size] = v;
        h->pos[v] = h->size;
        h->size++;
        mh_up(h, h->pos[v]);
    } else if (k > h->key[v]) {
        h->key[v] = k;
        mh_up(h, h->pos[v]);
    }
}
static int32_t mh_pop(mheap* h) {
    int32_t v = h->item[0];
    h->size--;
    if (h->size > 0) {
        h->item[0] = h->item[h->size];
        h->pos[h->item[0]] = 0;
        mh_down(h, 0);
    }
    h->pos[v] = -1;
    return v;
}

/* ------------------------------------------------------- Stoer-Wagner */
/* Each phase grows A by maximum adjacency (binary heap); the last vertex t
 * of the phase defines the cut-of-the-phase (members of t vs the rest) with
 * capacity w(A, t); then t is merged into the second-to-last vertex s.
 * Merged vertices keep their adjacency lists; entries are resolved through
 * rep[] so a list never needs rewriting. */
int64_t orc_stoer_wagner(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w,
                         uint8_t* side) {
    if (n < 2) return -1;
    sgraph g;
    if (sg_from_csr(n, rp, col, w, &g)) return -2;
    /* per-vertex dynamic lists (owned copies, so merges can append) */
    int32_t** la = (int32_t**)calloc((size_t)n, sizeof(int32_t*));
    int64_t** lw = (int64_t**)calloc((size_t)n, sizeof(int64_t*));
    int64_t* len = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    int64_t* cap = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    int32_t* rep = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* next = (int32_t*)malloc((size_t)n * sizeof(int32_t));   /* member list */
    int32_t* tail = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* msize = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    uint8_t* active = (uint8_t*)malloc((size_t)n);
    uint8_t* inA = (uint8_t*)malloc((size_t)n);
    int32_t* alive = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    mheap h;
    if (!la || !lw || !len || !cap || !rep || !next || !tail || !msize || !active || !inA || !alive ||
        mh_init(&h, n)) {
        sg_free(&g); return -2;
    }
    for (int32_t v = 0; v < n; v++) {
        len[v] = g.off[v + 1] - g.off[v];
        cap[v] = len[v] > 0 ? len[v] : 1;
        la[v] = (int32_t*)malloc((size_t)cap[v] * sizeof(int32_t));
        lw[v] = (int64_t*)malloc((size_t)cap[v] * sizeof(int64_t));
        memcpy(la[v], g.adj + g.off[v], (size_t)len[v] * sizeof(int32_t));
        memcpy(lw[v], g.wt + g.off[v], (size_t)len[v] * sizeof(int64_t));
        rep[v] = v; next[v] = -1; tail[v] = v; msize[v] = 1; active[v] = 1;
    }
    sg_free(&g);
    int64_t best = -1;
    int32_t best_rep = -1;
    uint8_t* best_side = (uint8_t*)calloc((size_t)n, 1);
    int32_t nact = n;
    while (nact > 1) {
        int32_t na = 0;
        for (int32_t v = 0; v < n; v++) if (active[v]) { alive[na++] = v; inA[v] = 0; }
        /* start from the smallest active vertex */
        int32_t s = -1, t = alive[0];
        mh_set(&h, t, 0);
        for (int32_t k = 1; k < na; k++) if (h.pos[alive[k]] < 0) mh_set(&h, alive[k], 0);
        int64_t wt_t = 0;
        while (h.size > 0) {
            int32_t u = mh_pop(&h);
            wt_t = h.key[u];
            s = t; t = u;
            inA[u] = 1;
            for (int64_t j = 0; j < len[u]; j++) {
                int32_t x = la[u][j];
                while (rep[x] != x) x = rep[x];
                if (x == u || inA[x]) continue;
                mh_set(&h, x, h.key[x] + lw[u][j]);
            }
        }
        for (int32_t k = 0; k < na; k++) h.key[alive[k]] = 0;
        /* cut of the phase: members of t */
        if (best < 0 || wt_t < best) {
            best = wt_t;
            best_rep = t;
            memset(best_side, 0, (size_t)n);
            for (int32_t x = t; x >= 0; x = next[x]) best_side[x] = 1;
        }
        /* merge t into s (smaller list appended to the larger one) */
        int32_t keep = s, gone = t;
        if (len[gone] > len[keep]) {
            int32_t* ta = la[keep]; la[keep] = la[gone]; la[gone] = ta;
            int64_t* tw = lw[keep]; lw[keep] = lw[gone]; lw[gone] = tw;
            int64_t tl = len[keep]; len[keep] = len[gone]; len[gone] = tl;
            int64_t tc = cap[keep]; cap[keep] = cap[gone]; cap[gone] = tc;
        }
        if (len[keep] + len[gone] > cap[keep]) {
            int64_t nc = 2 * (len[keep] + len[gone]) + 1;
            la[keep] = (int32_t*)realloc(la[keep], (size_t)nc * sizeof(int32_t));
            lw[keep] = (int64_t*)realloc(lw[keep], (size_t)nc * sizeof(int64_t));
            cap[keep] = nc;
        }
        memcpy(la[keep] + len[keep], la[gone], (size_t)len[gone] * sizeof(int32_t));
        memcpy(lw[keep] + len[keep], lw[gone], (size_t)len[gone] * sizeof(int64_t));
        len[keep] += len[gone];
        len[gone] = 0;
        rep[gone] = keep;
        active[gone] = 0;
        next[tail[keep]] = gone;
        tail[keep] = tail[gone];
        msize[keep] += msize[gone];
        nact--;
    }
    (void)best_rep;
    if (side) { memcpy(side, best_side, (size_t)n); canon_side(n, side); }
    for (int32_t v = 0; v < n; v++) { free(la[v]); free(lw[v]); }
    free(la); free(lw); free(len); free(cap); free(rep); free(next); free(tail); free(msize);
    free(active); free(inA); free(alive); free(best_side); mh_free(&h);
    return best;
}

/* ------------------------------------------------------------ degrees */
void orc_degrees(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w, int64_t* deg) {
    for (int32_t v = 0; v < n; v++) {
        int64_t s = 0;
        for (int64_t j = rp[v]; j < rp[v + 1]; j++) if (col[j] != v) s += w[j];
        deg[v] = s;
    }
}

/* --------------------------------------------------------- components */
/* Components of the graph on [0,n) whose edges are the given pairs, labelled
 * 0,1,.. in increasing order of their smallest vertex. Returns the count. */
int32_t orc_components(int32_t n, int64_t npairs, const int32_t* a, const int32_t* b, int32_t* label) {
    int64_t* off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* adj = (int32_t*)malloc((size_t)(2 * npairs + 1) * sizeof(int32_t));
    int32_t* queue = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
    if (!off || !adj || !queue) { free(off); free(adj); free(queue); return -1; }
    for (int64_t i = 0; i < npairs; i++) { off[a[i] + 1]++; off[b[i] + 1]++; }
    for (int32_t v = 0; v < n; v++) off[v + 1] += off[v];
    int64_t* cur = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    memcpy(cur, off, (size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < npairs; i++) { adj[cur[a[i]]++] = b[i]; adj[cur[b[i]]++] = a[i]; }
    free(cur);
    for (int32_t v = 0; v < n; v++) label[v] = -1;
    int32_t nc = 0;
    for (int32_t v = 0; v < n; v++) {
        if (label[v] >= 0) continue;
        int32_t qh = 0, qt = 0;
        queue[qt++] = v;
        label[v] = nc;
        while (qh < qt) {
            int32_t x = queue[qh++];
            for (int64_t j = off[x]; j < off[x + 1]; j++)
                if (label[adj[j]] < 0) { label[adj[j]] = nc; queue[qt++] = adj[j]; }
        }
        nc++;
    }
    free(off); free(adj); free(queue);
    return nc;
}

/* -------------------------------------------------------- contraction */
/* Contraction by the labels L (Section 2 "Basic Concepts"): vertex g of the
 * result stands for {v : L[v] = g}; an input entry v->x becomes g->L[x],
 * loops (L[v] = L[x]) vanish and entries between the same pair add up.
 * Output rows are sorted by target; zero-weight results are dropped.
 * Returns the number of output entries; out_* must hold nnz entries. */
int64_t orc_contract(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w,
                     const int32_t* L, int32_t n2, int32_t* out_rp, int32_t* out_col, int64_t* out_w) {
    int64_t nnz = rp[n];
    /* members of each group */
    int64_t* goff = (int64_t*)calloc((size_t)n2 + 1, sizeof(int64_t));
    int32_t* mem = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
    int64_t* buf = (int64_t*)malloc((size_t)(nnz + 1) * 2 * sizeof(int64_t));
    if (!goff || !mem || !buf) { free(goff); free(mem); free(buf); return -1; }
    for (int32_t v = 0; v < n; v++) goff[L[v] + 1]++;
    for (int32_t g = 0; g < n2; g++) goff[g + 1] += goff[g];
    int64_t* cur = (int64_t*)malloc((size_t)(n2 + 1) * sizeof(int64_t));
    memcpy(cur, goff, (size_t)n2 * sizeof(int64_t));
    for (int32_t v = 0; v < n; v++) mem[cur[L[v]]++] = v;
    free(cur);
    int64_t pos = 0;
    out_rp[0] = 0;
    for (int32_t g = 0; g < n2; g++) {
        /* collect (target, weight) pairs of the group and sort by target */
        int64_t k = 0;
        for (int64_t i = goff[g]; i < goff[g + 1]; i++) {
            int32_t v = mem[i];
            for (int64_t j = rp[v]; j < rp[v + 1]; j++) {
                int32_t t = L[col[j]];
                if (t == g) continue;
                buf[2 * k] = t;
                buf[2 * k + 1] = w[j];
                k++;
            }
        }
        qsort(buf, (size_t)k, 2 * sizeof(int64_t), cmp_i64);
        for (int64_t i = 0; i < k;) {
            int64_t t = buf[2 * i], s = 0;
            while (i < k && buf[2 * i] == t) { s += buf[2 * i + 1]; i++; }
            if (s != 0) { out_col[pos] = (int32_t)t; out_w[pos] = s; pos++; }
        }
        out_rp[g + 1] = (int32_t)pos;
    }
    free(goff); free(mem); free(buf);
    return pos;
}

/* --------------------------------------------- Padberg-Rinaldi 1 and 2 */
/* On a simple graph with current bound lam:
 *  flag1[j] = 1 iff entry j has weight >= lam (connectivity test 1)
 *  ptr2[v]  = the heaviest neighbour p of v (ties: smallest id) when
 *             2 c(v,p) >= c(v), else -1 (exchange test 2, one pointer per
 *             vertex). */
void orc_pr12(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w, int64_t lam,
              uint8_t* flag1, int32_t* ptr2) {
    for (int32_t v = 0; v < n; v++) {
        int64_t deg = 0, bw = -1;
        int32_t bp = -1;
        for (int64_t j = rp[v]; j < rp[v + 1]; j++) {
            deg += w[j];
            flag1[j] = w[j] >= lam;
            if (w[j] > bw || (w[j] == bw && col[j] < bp)) { bw = w[j]; bp = col[j]; }
        }
        ptr2[v] = (bp >= 0 && 2 * bw >= deg) ? bp : -1;
    }
}

/* ------------------------------------------ Padberg-Rinaldi tests 3, 4 */
/* Tests 3 and 4 (Section 2.1 names the four local tests of Padberg and
 * Rinaldi; App. A: sweeps may skip edges) on the candidate edges {v,x} of a
 * simple graph whose rows both have at most D entries; skipping the other
 * edges is always safe. With c(v) the degree of v:
 *   s(v,x) = c(v,x) + sum over common neighbours u of min(c(v,u), c(x,u))
 *   test 4: s(v,x) >= lam. The edge and the two-edge paths through common
 *           neighbours are edge-disjoint, so s bounds the connectivity of v
 *           and x from below.
 *   test 3: some common neighbour u has 2 (c(v,x) + c(v,u)) >= c(v) and
 *           2 (c(v,x) + c(x,u)) >= c(x).
 * Outputs: flag4[j] = 1 for every entry j of a candidate edge passing test
 * 4; part3[v] = the smallest x such that {v,x} is a candidate passing test 3
 * (-1: none); acc3[v] = x when part3[v] = x, part3[x] = v and neither v nor x
 * is the source or the target of a test-2 pointer (ptr2, as orc_pr12 gives
 * it), else -1. Rows must be those of a simple graph (no loops, no parallel
 * entries). */
void orc_pr34(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w, int64_t lam, int32_t D,
              const int32_t* ptr2, uint8_t* flag4, int32_t* part3, int32_t* acc3) {
    int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    uint8_t* touch = (uint8_t*)calloc((size_t)n + 1, 1);
    for (int32_t v = 0; v < n; v++) {
        for (int64_t j = rp[v]; j < rp[v + 1]; j++) deg[v] += w[j];
        part3[v] = -1;
        acc3[v] = -1;
        if (ptr2[v] >= 0) { touch[v] = 1; touch[ptr2[v]] = 1; }
    }
    for (int32_t v = 0; v < n; v++) {
        for (int64_t j = rp[v]; j < rp[v + 1]; j++) {
            flag4[j] = 0;
            const int32_t x = col[j];
            if (rp[v + 1] - rp[v] > D || rp[x + 1] - rp[x] > D) continue;
            const int64_t cvx = w[j];
            int64_t sum = cvx;
            int t3 = 0;
            for (int64_t a = rp[v]; a < rp[v + 1]; a++) {
                const int32_t u = col[a];
                if (u == x) continue;
                for (int64_t b = rp[x]; b < rp[x + 1]; b++) {
                    if (col[b] != u) continue;
                    const int64_t cvu = w[a], cxu = w[b];
                    sum += cvu < cxu ? cvu : cxu;
                    if (2 * (cvx + cvu) >= deg[v] && 2 * (cvx + cxu) >= deg[x]) t3 = 1;
                }
            }
            flag4[j] = sum >= lam;
            if (t3 && (part3[v] < 0 || x < part3[v])) part3[v] = x;
        }
    }
    for (int32_t v = 0; v < n; v++) {
        const int32_t x = part3[v];
        if (x >= 0 && part3[x] == v && !touch[v] && !touch[x]) acc3[v] = x;
    }
    free(deg);
    free(touch);
}

/* ------------------------------------------------- label propagation */
/* One synchronous round: v keeps lab_in[v] unless some other label carries
 * strictly more edge weight among v's neighbours; then it takes the
 * heaviest such label, the smallest one on ties. */
void orc_lp(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w,
            const int32_t* lab_in, int32_t* lab_out) {
    int64_t maxdeg = 0;
    for (int32_t v = 0; v < n; v++) if (rp[v + 1] - rp[v] > maxdeg) maxdeg = rp[v + 1] - rp[v];
    int64_t* buf = (int64_t*)malloc((size_t)(maxdeg + 1) * 2 * sizeof(int64_t));
    for (int32_t v = 0; v < n; v++) {
        int64_t k = 0, own = 0;
        for (int64_t j = rp[v]; j < rp[v + 1]; j++) {
            if (col[j] == v) continue;
            buf[2 * k] = lab_in[col[j]];
            buf[2 * k + 1] = w[j];
            k++;
        }
        qsort(buf, (size_t)k, 2 * sizeof(int64_t), cmp_i64);
        int64_t bestw = -1, bestl = -1;
        for (int64_t i = 0; i < k;) {
            int64_t l = buf[2 * i], s = 0;
            while (i < k && buf[2 * i] == l) { s += buf[2 * i + 1]; i++; }
            if (l == lab_in[v]) { own = s; continue; }
            if (s > bestw) { bestw = s; bestl = l; }   /* ascending l: first max wins */
        }
        lab_out[v] = (bestl >= 0 && bestw > own) ? (int32_t)bestl : lab_in[v];
    }
    free(buf);
}

/* ---------------------------------------------------- CAPFOREST pass */
/* One sequential pass of Algorithm 1 on a simple graph with no other pass
 * running (so no vertex is ever blacklisted), started at `start`.
 * Priority: the queued vertex with the largest min(r(y), lam), where lam is
 * the bound at the moment of the pop; ties go to the smallest id.
 * Scanning x adds c(x) - 2 r(x) to alpha; alpha bounds lam only while the
 * scanned set is a proper subset. For every edge to an unscanned y, the
 * edge is marked when r(y) < lam <= r(y) + c(e), then r(y) grows by c(e).
 * The pass stops when the queue empties or after max_scan scans
 * (max_scan <= 0: no limit). Marked pairs are returned as canonical
 * component labels; order[] receives the scanned vertices.
 * Returns the number of marked edges; *lam_io is updated in place. */
int64_t orc_capforest_pass(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w,
                           int64_t* lam_io, int32_t start, int32_t max_scan, int32_t* label,
                           int32_t* order, int32_t* nscan_out, int64_t* best_alpha_out,
                           int32_t* best_len_out) {
    int64_t lam = *lam_io;
    int64_t* r = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    uint8_t* state = (uint8_t*)calloc((size_t)n + 1, 1);     /* 0 new, 1 queued, 2 scanned */
    int32_t* queue = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
    int32_t* pa = (int32_t*)malloc((size_t)(rp[n] + 1) * sizeof(int32_t));
    int32_t* pb = (int32_t*)malloc((size_t)(rp[n] + 1) * sizeof(int32_t));
    int64_t npairs = 0, alpha = 0, best_alpha = -1;
    int32_t qn = 0, nscan = 0, best_len = 0;
    queue[qn++] = start;
    state[start] = 1;
    while (qn > 0 && (max_scan <= 0 || nscan < max_scan)) {
        /* pop: largest min(r, lam), then smallest id */
        int32_t bi = 0;
        for (int32_t i = 1; i < qn; i++) {
            int32_t a = queue[i], b = queue[bi];
            int64_t ka = r[a] < lam ? r[a] : lam, kb = r[b] < lam ? r[b] : lam;
            if (ka > kb || (ka == kb && a < b)) bi = i;
        }
        int32_t x = queue[bi];
        queue[bi] = queue[--qn];
        state[x] = 2;
        order[nscan++] = x;
        int64_t cx = 0;
        for (int64_t j = rp[x]; j < rp[x + 1]; j++) cx += w[j];
        alpha += cx - 2 * r[x];
        if (nscan < n) {
            if (best_alpha < 0 || alpha < best_alpha) { best_alpha = alpha; best_len = nscan; }
            if (alpha < lam) lam = alpha;
        }
        for (int64_t j = rp[x]; j < rp[x + 1]; j++) {
            int32_t y = col[j];
            if (state[y] == 2) continue;
            if (r[y] < lam && lam <= r[y] + w[j]) { pa[npairs] = x; pb[npairs] = y; npairs++; }
            r[y] += w[j];
            if (state[y] == 0) { state[y] = 1; queue[qn++] = y; }
        }
    }
    orc_components(n, npairs, pa, pb, label);
    *lam_io = lam;
    *nscan_out = nscan;
    *best_alpha_out = best_alpha;
    *best_len_out = best_len;
    free(r); free(state); free(queue); free(pa); free(pb);
    return npairs;
}

/* ------------------------------------------------------------------ NOI */
/* The exact loop of Section 2.1 without the heuristic and without the
 * reduction tests: lam starts at the minimum degree; each round runs one
 * full pass from the smallest vertex (binary heap on min(r, lam), keys not
 * lowered when lam falls), contracts every marked edge, and lowers lam by
 * the collapsed degrees, until at most two vertices remain. A pass that
 * lowers lam may mark nothing; the next round then starts from the lower
 * bound, so every round either marks an edge or lowers lam. The side is
 * tracked through map[] from input vertices to current ones. */
int64_t orc_noi(int32_t n, const int32_t* rp, const int32_t* col, const int64_t* w, uint8_t* side,
                int32_t* rounds_out) {
    if (n < 2) return -1;
    sgraph g;
    if (sg_from_csr(n, rp, col, w, &g)) return -2;
    int32_t* map = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    uint8_t* best = (uint8_t*)calloc((size_t)n, 1);
    for (int32_t v = 0; v < n; v++) map[v] = v;
    int64_t lam = -1;
    int32_t rounds = 0;
    /* initial bound: minimum degree */
    for (int32_t v = 0; v < n; v++) {
        int64_t d = sg_degree(&g, v);
        if (lam < 0 || d < lam) { lam = d; memset(best, 0, (size_t)n); best[v] = 1; }
    }
    while (g.n > 2 && lam > 0) {
        int32_t cn = g.n;
        int64_t lam_round_start = lam;
        int64_t* r = (int64_t*)calloc((size_t)cn, sizeof(int64_t));
        uint8_t* done = (uint8_t*)calloc((size_t)cn, 1);
        int32_t* pos_in_order = (int32_t*)malloc((size_t)cn * sizeof(int32_t));
        int32_t* par = (int32_t*)malloc((size_t)cn * sizeof(int32_t));
        for (int32_t v = 0; v < cn; v++) { par[v] = v; pos_in_order[v] = -1; }
        mheap h;
        mh_init(&h, cn);
        int64_t alpha = 0, marks = 0, round_best = -1;
        int32_t nscan = 0, best_len = 0;
        /* the scan must reach every vertex even if the graph has several
         * components: restart from the smallest unscanned vertex */
        for (int32_t s0 = 0; s0 < cn; s0++) {
            if (done[s0]) continue;
            mh_set(&h, s0, 0);
            while (h.size > 0) {
                int32_t x = mh_pop(&h);
                done[x] = 1;
                pos_in_order[x] = nscan++;
                int64_t cx = sg_degree(&g, x);
                alpha += cx - 2 * r[x];
                if (nscan < cn && alpha < lam) {
                    lam = alpha;
                    round_best = alpha;
                    best_len = nscan;
                }
                for (int64_t j = g.off[x]; j < g.off[x + 1]; j++) {
                    int32_t y = g.adj[j];
                    if (done[y]) continue;
                    if (r[y] < lam && lam <= r[y] + g.wt[j]) {
                        int32_t a = x, b = y;
                        while (par[a] != a) a = par[a];
                        while (par[b] != b) b = par[b];
                        if (a != b) { if (a < b) par[b] = a; else par[a] = b; }
                        marks++;
                    }
                    r[y] += g.wt[j];
                    mh_set(&h, y, r[y] < lam ? r[y] : lam);
                }
            }
        }
        if (round_best >= 0) {
            for (int32_t v = 0; v < n; v++) best[v] = pos_in_order[map[v]] < best_len;
        }
        /* contract the marked edges */
        int32_t* lab = (int32_t*)malloc((size_t)cn * sizeof(int32_t));
        int32_t n2 = 0;
        for (int32_t v = 0; v < cn; v++) {
            int32_t a = v;
            while (par[a] != a) a = par[a];
            par[v] = a;
        }
        for (int32_t v = 0; v < cn; v++) lab[v] = (par[v] == v) ? n2++ : -1;
        for (int32_t v = 0; v < cn; v++) lab[v] = lab[par[v]];
        if (n2 < cn) {
            int32_t* crp = (int32_t*)malloc((size_t)(cn + 1) * sizeof(int32_t));
            for (int32_t v = 0; v <= cn; v++) crp[v] = (int32_t)g.off[v];
            int32_t* nrp = (int32_t*)malloc((size_t)(n2 + 1) * sizeof(int32_t));
            int32_t* ncol = (int32_t*)malloc((size_t)(g.off[cn] + 1) * sizeof(int32_t));
            int64_t* nw = (int64_t*)malloc((size_t)(g.off[cn] + 1) * sizeof(int64_t));
            int64_t m2 = orc_contract(cn, crp, g.adj, g.wt, lab, n2, nrp, ncol, nw);
            sg_free(&g);
            g.n = n2;
            g.off = (int64_t*)malloc((size_t)(n2 + 1) * sizeof(int64_t));
            for (int32_t v = 0; v <= n2; v++) g.off[v] = nrp[v];
            g.adj = ncol;
            g.wt = nw;
            (void)m2;
            free(crp); free(nrp);
            for (int32_t v = 0; v < n; v++) map[v] = lab[map[v]];
            /* collapsed degrees are cuts of the input graph, provided the
             * other side is not empty */
            for (int32_t c = 0; n2 >= 2 && c < n2; c++) {
                int64_t d = sg_degree(&g, c);
                if (d < lam) {
                    lam = d;
                    for (int32_t v = 0; v < n; v++) best[v] = map[v] == c;
                }
            }
        }
        free(lab); free(r); free(done); free(pos_in_order); free(par); mh_free(&h);
        rounds++;
        /* a full pass with a fixed bound always marks an edge; a round that
         * neither marks nor lowers the bound would be a defect */
        if (marks == 0 && lam == lam_round_start) { lam = -3; break; }
    }
    if (side) { memcpy(side, best, (size_t)n); canon_side(n, side); }
    if (rounds_out) *rounds_out = rounds;
    sg_free(&g);
    free(map); free(best);
    return lam;
}
