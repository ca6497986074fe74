/*
 * Seeded synthetic graph generators for the minimum-cut workloads.
 *
 * This module only produces inputs. It contains none of the minimum-cut
 * method's arithmetic and is shared by the CPU oracle and the GPU path.
 *
 * Every generator writes an undirected simple edge list (u < v, no loops, no
 * duplicates) into a gen_edges record whose arrays are malloc'd here and
 * released by gen_free. Randomness comes from splitmix64 (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014).
 *
 * Published methods used:
 *  - random d-regular graphs: Steger and Wormald 1999 pairing with rejection
 *  - Erdos-Renyi G(n,p): Batagelj and Brandes 2005 geometric skipping
 *  - Chung-Lu: Miller and Hagberg 2011 O(n+m) skipping
 *  - threshold random hyperbolic graphs: Krioukov et al. 2010 model,
 *    band-partitioned generation after von Looz et al. 2015
 *  - k-core: Batagelj and Zaversnik 2003 bucket peeling
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n;
    int64_t m;
    int64_t cap;
    int32_t* u;
    int32_t* v;
    int64_t* w;
} gen_edges;

/* ------------------------------------------------------------------ RNG */
static inline uint64_t sm64_next(uint64_t* s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
/* uniform integer in [0, range) by the multiply-shift map (Lemire 2019) */
static inline uint64_t rng_below(uint64_t* s, uint64_t range) {
    return (uint64_t)(((__uint128_t)sm64_next(s) * range) >> 64);
}
/* uniform double in [0,1) with 53 random bits */
static inline double rng_unit(uint64_t* s) {
    return (double)(sm64_next(s) >> 11) * (1.0 / 9007199254740992.0);
}

/* --------------------------------------------------------------- edges */
static int edges_reserve(gen_edges* e, int64_t need) {
    if (need <= e->cap) return 0;
    int64_t nc = e->cap ? e->cap : 1024;
    while (nc < need) nc *= 2;
    int32_t* nu = (int32_t*)realloc(e->u, (size_t)nc * sizeof(int32_t));
    if (!nu) return -1;
    e->u = nu;
    int32_t* nv = (int32_t*)realloc(e->v, (size_t)nc * sizeof(int32_t));
    if (!nv) return -1;
    e->v = nv;
    e->cap = nc;
    return 0;
}
static inline int edges_push(gen_edges* e, int32_t a, int32_t b) {
    if (e->m >= e->cap && edges_reserve(e, e->m + 1)) return -1;
    if (a > b) { int32_t t = a; a = b; b = t; }
    e->u[e->m] = a;
    e->v[e->m] = b;
    e->m++;
    return 0;
}

void gen_free(gen_edges* e) {
    free(e->u); free(e->v); free(e->w);
    memset(e, 0, sizeof(*e));
}

/* assign every edge an independent uniform integer weight in [lo, hi] */
int gen_weights(gen_edges* e, int64_t lo, int64_t hi, uint64_t seed) {
    free(e->w);
    e->w = (int64_t*)malloc((size_t)(e->m > 0 ? e->m : 1) * sizeof(int64_t));
    if (!e->w) return -1;
    uint64_t s = seed ^ 0x5851F42D4C957F2DULL;
    uint64_t range = (uint64_t)(hi - lo) + 1;
    for (int64_t i = 0; i < e->m; i++) e->w[i] = lo + (int64_t)rng_below(&s, range);
    return 0;
}

/* ------------------------------------------------- random d-regular (SW) */
/* Pairing model: repeatedly join two random free points whose vertices are
 * distinct and not yet adjacent; restart when no legal pair can be found. */
static int regular_into(gen_edges* e, int32_t base, int32_t n, int32_t d, uint64_t* s) {
    if ((int64_t)n * d % 2 != 0 || d >= n) return -2;
    int64_t np = (int64_t)n * d;
    int32_t* pts = (int32_t*)malloc((size_t)np * sizeof(int32_t));
    int32_t* adj = (int32_t*)malloc((size_t)np * sizeof(int32_t));
    int32_t* deg = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!pts || !adj || !deg) { free(pts); free(adj); free(deg); return -1; }
    int64_t m0 = e->m;
    for (int attempt = 0; attempt < 1000; attempt++) {
        e->m = m0;
        for (int64_t i = 0; i < np; i++) pts[i] = (int32_t)(i / d);
        memset(deg, 0, (size_t)n * sizeof(int32_t));
        int64_t left = np;
        int ok = 1;
        while (left > 0) {
            int64_t tries = 0, limit = 64 + 8 * left;
            int joined = 0;
            while (tries++ < limit) {
                int64_t i = (int64_t)rng_below(s, (uint64_t)left);
                int64_t j = (int64_t)rng_below(s, (uint64_t)left);
                if (i == j) continue;
                int32_t a = pts[i], b = pts[j];
                if (a == b) continue;
                int dup = 0;
                for (int32_t k = 0; k < deg[a]; k++)
                    if (adj[(int64_t)a * d + k] == b) { dup = 1; break; }
                if (dup) continue;
                adj[(int64_t)a * d + deg[a]++] = b;
                adj[(int64_t)b * d + deg[b]++] = a;
                if (edges_push(e, base + a, base + b)) { free(pts); free(adj); free(deg); return -1; }
                /* remove points i and j (larger index first) */
                int64_t hi_i = i > j ? i : j, lo_i = i > j ? j : i;
                pts[hi_i] = pts[left - 1]; left--;
                pts[lo_i] = pts[left - 1]; left--;
                joined = 1;
                break;
            }
            if (!joined) { ok = 0; break; }
        }
        if (ok) { free(pts); free(adj); free(deg); return 0; }
    }
    free(pts); free(adj); free(deg);
    /* Dense blocks (d close to n - 1), where the pairing rarely completes: a
     * d-regular graph is the complement of an (n-1-d)-regular one, which the
     * pairing finds easily. Taken only after the pairing failed, so every
     * graph the pairing produces stays as it was. */
    if (2 * d > n - 1 && n <= 4096) {
        gen_edges c;
        memset(&c, 0, sizeof(c));
        int rc = regular_into(&c, 0, n, n - 1 - d, s);
        if (rc) { gen_free(&c); return rc; }
        uint8_t* mat = (uint8_t*)calloc((size_t)n * n, 1);
        if (!mat) { gen_free(&c); return -1; }
        for (int64_t k = 0; k < c.m; k++) {
            mat[(int64_t)c.u[k] * n + c.v[k]] = 1;
            mat[(int64_t)c.v[k] * n + c.u[k]] = 1;
        }
        gen_free(&c);
        e->m = m0;
        for (int32_t a = 0; a < n; a++)
            for (int32_t b = a + 1; b < n; b++)
                if (!mat[(int64_t)a * n + b] && edges_push(e, base + a, base + b)) { free(mat); return -1; }
        free(mat);
        return 0;
    }
    return -3;
}

int gen_regular(int32_t n, int32_t d, uint64_t seed, gen_edges* out) {
    memset(out, 0, sizeof(*out));
    out->n = n;
    uint64_t s = seed;
    return regular_into(out, 0, n, d, &s);
}

/* Two random d-regular blocks [0,na) and [na,na+nb) with integer weights in
 * [lo,hi], joined by `bridges` distinct uniform cross pairs of weight 1. */
int gen_planted(int32_t na, int32_t nb, int32_t d, int32_t bridges, int64_t lo, int64_t hi,
                uint64_t seed, gen_edges* out) {
    memset(out, 0, sizeof(*out));
    out->n = (int64_t)na + nb;
    uint64_t s = seed;
    int rc = regular_into(out, 0, na, d, &s);
    if (rc) return rc;
    rc = regular_into(out, na, nb, d, &s);
    if (rc) return rc;
    int64_t inner = out->m;
    if (gen_weights(out, lo, hi, seed + 17)) return -1;
    int64_t* w = out->w;
    out->w = NULL;
    for (int32_t b = 0; b < bridges; b++) {
        for (;;) {
            int32_t x = (int32_t)rng_below(&s, (uint64_t)na);
            int32_t y = na + (int32_t)rng_below(&s, (uint64_t)nb);
            int dup = 0;
            for (int64_t k = inner; k < out->m; k++)
                if (out->u[k] == x && out->v[k] == y) { dup = 1; break; }
            if (dup) continue;
            if (edges_push(out, x, y)) { free(w); return -1; }
            break;
        }
    }
    out->w = (int64_t*)realloc(w, (size_t)(out->m > 0 ? out->m : 1) * sizeof(int64_t));
    if (!out->w) return -1;
    for (int64_t k = inner; k < out->m; k++) out->w[k] = 1;
    return 0;
}

/* ------------------------------------------------------ Erdos-Renyi (BB) */
int gen_er(int32_t n, double p, uint64_t seed, gen_edges* out) {
    memset(out, 0, sizeof(*out));
    out->n = n;
    if (p <= 0.0 || n < 2) return 0;
    uint64_t s = seed;
    if (p >= 1.0) {
        for (int32_t a = 0; a < n; a++)
            for (int32_t b = a + 1; b < n; b++)
                if (edges_push(out, a, b)) return -1;
        return 0;
    }
    double lq = log(1.0 - p);
    int64_t v = 1, wv = -1;
    while (v < n) {
        double r = rng_unit(&s);
        wv += 1 + (int64_t)floor(log(1.0 - r) / lq);
        while (wv >= v && v < n) { wv -= v; v++; }
        if (v < n && edges_push(out, (int32_t)v, (int32_t)wv)) return -1;
    }
    return 0;
}

/* -------------------------------------------------------- Chung-Lu (MH) */
/* Expected-degree weights c*(i+1)^(-1/(beta-1)) scaled to mean avg_deg and
 * capped at `cap` (<= 0 means sqrt(n*avg_deg)); vertex pairs joined with
 * probability min(1, w_i w_j / sum(w)). */
int gen_chung_lu(int32_t n, double beta, double avg_deg, double cap, uint64_t seed,
                 gen_edges* out) {
    memset(out, 0, sizeof(*out));
    out->n = n;
    if (n < 2) return 0;
    double* wt = (double*)malloc((size_t)n * sizeof(double));
    if (!wt) return -1;
    double ex = -1.0 / (beta - 1.0), sum = 0.0;
    for (int32_t i = 0; i < n; i++) { wt[i] = pow((double)i + 1.0, ex); sum += wt[i]; }
    double scale = avg_deg * (double)n / sum;
    if (cap <= 0.0) cap = sqrt((double)n * avg_deg);
    double S = 0.0;
    for (int32_t i = 0; i < n; i++) { wt[i] *= scale; if (wt[i] > cap) wt[i] = cap; S += wt[i]; }
    if (edges_reserve(out, (int64_t)(0.55 * avg_deg * n) + 1024)) { free(wt); return -1; }
    uint64_t s = seed;
    for (int32_t u = 0; u < n - 1; u++) {
        int64_t v = u + 1;
        double p = wt[u] * wt[v] / S;
        if (p > 1.0) p = 1.0;
        while (v < n && p > 0.0) {
            if (p != 1.0) {
                double r = rng_unit(&s);
                v += (int64_t)floor(log(1.0 - r) / log(1.0 - p));
            }
            if (v < n) {
                double q = wt[u] * wt[v] / S;
                if (q > 1.0) q = 1.0;
                double r = rng_unit(&s);
                if (r < q / p && edges_push(out, u, (int32_t)v)) { free(wt); return -1; }
                p = q;
                v++;
            }
        }
    }
    free(wt);
    return 0;
}

/* --------------------------------------------- random hyperbolic (KPKVB) */
typedef struct { double theta, r, cr, sr; int32_t id; } rhg_pt;
static int rhg_cmp(const void* a, const void* b) {
    double x = ((const rhg_pt*)a)->theta, y = ((const rhg_pt*)b)->theta;
    return (x > y) - (x < y);
}
/* Expected mean degree of the threshold model with disk radius R: (n-1)
 * times the probability that two independent points lie within distance R,
 * integrated on a midpoint grid over the radial quantiles (the angle
 * difference is uniform on [0, pi], so the inner integral is closed form). */
static double rhg_mean_deg(int32_t n, double alpha, double R, int grid) {
    double coshR = cosh(R), acc = 0.0;
    double* cr = (double*)malloc((size_t)grid * sizeof(double));
    double* sr = (double*)malloc((size_t)grid * sizeof(double));
    if (!cr || !sr) { free(cr); free(sr); return 0.0; }
    for (int i = 0; i < grid; i++) {
        double u = (i + 0.5) / grid;
        double r = acosh(1.0 + u * (cosh(alpha * R) - 1.0)) / alpha;
        cr[i] = cosh(r); sr[i] = sinh(r);
    }
    for (int i = 0; i < grid; i++) {
        for (int j = 0; j < grid; j++) {
            double num = cr[i] * cr[j] - coshR, den = sr[i] * sr[j];
            double frac;
            if (den <= 0.0) frac = (num <= 0.0) ? 1.0 : 0.0;
            else if (num >= den) frac = 0.0;
            else if (num <= -den) frac = 1.0;
            else frac = acos(num / den) / M_PI;
            acc += frac;
        }
    }
    free(cr); free(sr);
    return acc / ((double)grid * grid) * (double)(n - 1);
}

int gen_rhg(int32_t n, double avg_deg, double gamma, uint64_t seed, gen_edges* out) {
    memset(out, 0, sizeof(*out));
    out->n = n;
    if (n < 2) return 0;
    double alpha = (gamma - 1.0) / 2.0;
    uint64_t s = seed;
    /* bisection on R for the requested mean degree */
    double lo = 1.0, hi = 2.0 * log((double)n) + 10.0;
    for (int it = 0; it < 40; it++) {
        double mid = 0.5 * (lo + hi);
        double dm = rhg_mean_deg(n, alpha, mid, 1200);
        if (dm > avg_deg) lo = mid; else hi = mid;
    }
    double R = 0.5 * (lo + hi), coshR = cosh(R);
    rhg_pt* p = (rhg_pt*)malloc((size_t)n * sizeof(rhg_pt));
    if (!p) return -1;
    for (int32_t i = 0; i < n; i++) {
        double u = rng_unit(&s);
        p[i].theta = rng_unit(&s) * 2.0 * M_PI;
        p[i].r = acosh(1.0 + u * (cosh(alpha * R) - 1.0)) / alpha;
        p[i].cr = cosh(p[i].r);
        p[i].sr = sinh(p[i].r);
        p[i].id = i;
    }
    /* radial bands of roughly equal hyperbolic width, outermost widest */
    int nb = (int)(log((double)n) / 2.0) + 1;
    if (nb < 2) nb = 2;
    if (nb > 32) nb = 32;
    double bnd[34];
    bnd[0] = 0.0;
    for (int b = 1; b < nb; b++) bnd[b] = R * (double)b / nb;
    bnd[nb] = R + 1e-12;
    int64_t bstart[34];
    rhg_pt* sorted = (rhg_pt*)malloc((size_t)n * sizeof(rhg_pt));
    if (!sorted) { free(p); return -1; }
    int64_t pos = 0;
    for (int b = 0; b < nb; b++) {
        bstart[b] = pos;
        for (int32_t i = 0; i < n; i++)
            if (p[i].r >= bnd[b] && p[i].r < bnd[b + 1]) sorted[pos++] = p[i];
        qsort(sorted + bstart[b], (size_t)(pos - bstart[b]), sizeof(rhg_pt), rhg_cmp);
    }
    bstart[nb] = pos;
    free(p);
    /* for each point, query every band at or outside its own band */
    for (int bq = 0; bq < nb; bq++) {
        for (int64_t i = bstart[bq]; i < bstart[bq + 1]; i++) {
            const rhg_pt* a = &sorted[i];
            for (int b = bq; b < nb; b++) {
                int64_t s0 = bstart[b], s1 = bstart[b + 1];
                if (s0 == s1) continue;
                /* largest angle at which a point of radius >= bnd[b] can connect */
                double rb = bnd[b];
                double dth;
                double num = a->cr * cosh(rb) - coshR, den = a->sr * sinh(rb);
                if (den <= 0.0 || num <= -den) dth = M_PI;
                else if (num >= den) dth = -1.0;
                else dth = acos(num / den);
                if (dth < 0.0) continue;
                double t0 = a->theta - dth, t1 = a->theta + dth;
                /* scan the angular window, split at the 0 / 2pi seam */
                int full = dth >= M_PI;
                for (int pass = 0; pass < 3; pass++) {
                    double lo_t = t0, hi_t = t1;
                    if (full) { if (pass > 0) continue; lo_t = 0.0; hi_t = 2 * M_PI; }
                    else if (pass == 0) { if (lo_t < 0.0) lo_t = 0.0; if (hi_t > 2 * M_PI) hi_t = 2 * M_PI; }
                    else if (pass == 1) { if (t0 >= 0.0) continue; lo_t = t0 + 2 * M_PI; hi_t = 2 * M_PI; }
                    else { if (t1 < 2 * M_PI) continue; lo_t = 0.0; hi_t = t1 - 2 * M_PI; }
                    int64_t l = s0, h = s1;
                    while (l < h) { int64_t mid = (l + h) / 2; if (sorted[mid].theta < lo_t) l = mid + 1; else h = mid; }
                    for (int64_t j = l; j < s1 && sorted[j].theta <= hi_t; j++) {
                        const rhg_pt* c = &sorted[j];
                        if (b == bq && j <= i) continue;
                        double dt = fabs(a->theta - c->theta);
                        if (dt > M_PI) dt = 2 * M_PI - dt;
                        double ch = a->cr * c->cr - a->sr * c->sr * cos(dt);
                        if (ch <= coshR && edges_push(out, a->id, c->id)) { free(sorted); return -1; }
                    }
                }
            }
        }
    }
    free(sorted);
    return 0;
}

/* ------------------------------------------------------ core, LCC, etc. */
static int build_adj(const gen_edges* e, int64_t** off_out, int32_t** adj_out) {
    int64_t n = e->n;
    int64_t* off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* adj = (int32_t*)malloc((size_t)(2 * e->m + 1) * sizeof(int32_t));
    if (!off || !adj) { free(off); free(adj); return -1; }
    for (int64_t i = 0; i < e->m; i++) { off[e->u[i] + 1]++; off[e->v[i] + 1]++; }
    for (int64_t i = 0; i < n; i++) off[i + 1] += off[i];
    int64_t* cur = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    if (!cur) { free(off); free(adj); return -1; }
    memcpy(cur, off, (size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < e->m; i++) { adj[cur[e->u[i]]++] = e->v[i]; adj[cur[e->v[i]]++] = e->u[i]; }
    free(cur);
    *off_out = off;
    *adj_out = adj;
    return 0;
}

/* keep only edges whose endpoints both have keep[x] != 0, relabel survivors
 * densely in increasing id order */
static int filter_relabel(gen_edges* e, const uint8_t* keep) {
    int32_t* nid = (int32_t*)malloc((size_t)(e->n + 1) * sizeof(int32_t));
    if (!nid) return -1;
    int32_t c = 0;
    for (int64_t x = 0; x < e->n; x++) nid[x] = keep[x] ? c++ : -1;
    int64_t k = 0;
    for (int64_t i = 0; i < e->m; i++) {
        if (keep[e->u[i]] && keep[e->v[i]]) {
            e->u[k] = nid[e->u[i]];
            e->v[k] = nid[e->v[i]];
            if (e->w) e->w[k] = e->w[i];
            k++;
        }
    }
    e->m = k;
    e->n = c;
    free(nid);
    return 0;
}

/* reduce to the k-core (Batagelj-Zaversnik peeling) */
int gen_kcore(gen_edges* e, int32_t k) {
    int64_t n = e->n;
    if (n == 0) return 0;
    int64_t* off; int32_t* adj;
    if (build_adj(e, &off, &adj)) return -1;
    int32_t* deg = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    uint8_t* keep = (uint8_t*)malloc((size_t)n);
    int32_t* stack = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!deg || !keep || !stack) { free(off); free(adj); free(deg); free(keep); free(stack); return -1; }
    int64_t top = 0;
    for (int64_t x = 0; x < n; x++) {
        deg[x] = (int32_t)(off[x + 1] - off[x]);
        keep[x] = 1;
        if (deg[x] < k) { keep[x] = 0; stack[top++] = (int32_t)x; }
    }
    while (top > 0) {
        int32_t x = stack[--top];
        for (int64_t j = off[x]; j < off[x + 1]; j++) {
            int32_t y = adj[j];
            if (keep[y] && --deg[y] < k) { keep[y] = 0; stack[top++] = y; }
        }
    }
    int rc = filter_relabel(e, keep);
    free(off); free(adj); free(deg); free(keep); free(stack);
    return rc;
}

/* reduce to the largest connected component (ties: the one holding the
 * smallest vertex id) */
int gen_lcc(gen_edges* e) {
    int64_t n = e->n;
    if (n == 0) return 0;
    int32_t* par = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int64_t* sz = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    uint8_t* keep = (uint8_t*)malloc((size_t)n);
    if (!par || !sz || !keep) { free(par); free(sz); free(keep); return -1; }
    for (int64_t x = 0; x < n; x++) par[x] = (int32_t)x;
    for (int64_t i = 0; i < e->m; i++) {
        int32_t a = e->u[i], b = e->v[i];
        while (par[a] != a) { par[a] = par[par[a]]; a = par[a]; }
        while (par[b] != b) { par[b] = par[par[b]]; b = par[b]; }
        if (a != b) { if (a < b) par[b] = a; else par[a] = b; }
    }
    int32_t best = -1;
    for (int64_t x = 0; x < n; x++) {
        int32_t a = (int32_t)x;
        while (par[a] != a) a = par[a];
        par[x] = a;
        sz[a]++;
    }
    for (int64_t x = 0; x < n; x++) if (par[x] == x && (best < 0 || sz[x] > sz[best])) best = (int32_t)x;
    for (int64_t x = 0; x < n; x++) keep[x] = (par[x] == best);
    int rc = filter_relabel(e, keep);
    free(par); free(sz); free(keep);
    return rc;
}

/* apply a seeded uniform random permutation to the vertex ids */
int gen_shuffle(gen_edges* e, uint64_t seed) {
    int64_t n = e->n;
    int32_t* perm = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!perm) return -1;
    for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
    uint64_t s = seed ^ 0xD1B54A32D192ED03ULL;
    for (int64_t i = n - 1; i > 0; i--) {
        int64_t j = (int64_t)rng_below(&s, (uint64_t)i + 1);
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    for (int64_t i = 0; i < e->m; i++) {
        int32_t a = perm[e->u[i]], b = perm[e->v[i]];
        if (a > b) { int32_t t = a; a = b; b = t; }
        e->u[i] = a; e->v[i] = b;
    }
    free(perm);
    return 0;
}

/* symmetric CSR with every row sorted by target; edge weights must be set */
int gen_to_csr(const gen_edges* e, int32_t* row_ptr, int32_t* col, int64_t* w) {
    int64_t n = e->n;
    memset(row_ptr, 0, (size_t)(n + 1) * sizeof(int32_t));
    for (int64_t i = 0; i < e->m; i++) { row_ptr[e->u[i] + 1]++; row_ptr[e->v[i] + 1]++; }
    for (int64_t x = 0; x < n; x++) row_ptr[x + 1] += row_ptr[x];
    int32_t* cur = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
    if (!cur) return -1;
    memcpy(cur, row_ptr, (size_t)n * sizeof(int32_t));
    /* edges are visited in (u,v) order after a counting sort by the other
     * endpoint, which leaves each row sorted */
    int64_t* ord = (int64_t*)malloc((size_t)(2 * e->m + 1) * sizeof(int64_t));
    int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    if (!ord || !cnt) { free(cur); free(ord); free(cnt); return -1; }
    /* directed entries (src,dst) keyed by dst, then stable-place by src */
    for (int64_t i = 0; i < e->m; i++) { cnt[e->v[i] + 1]++; cnt[e->u[i] + 1]++; }
    for (int64_t x = 0; x < n; x++) cnt[x + 1] += cnt[x];
    for (int64_t i = 0; i < e->m; i++) {
        ord[cnt[e->v[i]]++] = 2 * i;       /* entry u -> v, keyed by v */
        ord[cnt[e->u[i]]++] = 2 * i + 1;   /* entry v -> u, keyed by u */
    }
    for (int64_t k = 0; k < 2 * e->m; k++) {
        int64_t i = ord[k] >> 1;
        int32_t src = (ord[k] & 1) ? e->v[i] : e->u[i];
        int32_t dst = (ord[k] & 1) ? e->u[i] : e->v[i];
        int32_t p = cur[src]++;
        col[p] = dst;
        w[p] = e->w[i];
    }
    free(cur); free(ord); free(cnt);
    return 0;
}
