/*
 * CPU oracle of Hierarchical NSW (Malkov & Yashunin, "Efficient and robust
 * approximate nearest neighbor search using Hierarchical Navigable Small World
 * graphs", arXiv:1603.09320).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header or table with the GPU library.
 *
 * What it implements, each in the paper's order and notation:
 *   - the level draw of Alg. 1, l = floor(-ln(unif(0..1)) * mL),
 *   - SEARCH-LAYER (Alg. 2) with an exact visited set and two binary heaps
 *     (C: nearest first, W: furthest first),
 *   - SELECT-NEIGHBORS-SIMPLE (Alg. 3) and SELECT-NEIGHBORS-HEURISTIC (Alg. 4),
 *     both flags of Alg. 4 included,
 *   - INSERT (Alg. 1), including the connection shrink,
 *   - K-NN-SEARCH (Alg. 5),
 *   - brute-force K-NN, the plain definition of the problem (Sec. 1).
 *
 * Readings taken where the paper is silent (each is listed with its reason in
 * the design notes of the repository):
 *   - Distances: squared L2, or 1 - <q,x> for the inner-product metric (Sec. 5.2
 *     treats cosine as L2 after normalisation).  The sum is accumulated in
 *     double precision; the value that takes part in every comparison is that
 *     sum rounded once to float (the precision of the paper's implementation
 *     and of the GPU kernel), so both sides take each decision in fp32.
 *   - Ties: every "nearest"/"furthest" compares the key (distance, id) in
 *     lexicographic order, a strict total order.
 *   - unif(0..1): U = (r + 1) * 2^-53 with r the top 53 bits of
 *     splitmix64(seed XOR i), so U lies in (0, 1] and ln U is finite.
 *   - Alg. 4's keep-test: candidate e is kept iff dist(e, q) < dist(e, r) for
 *     every r already kept (the rule stated in Sec. 3; the printed test is
 *     garbled).
 *   - Alg. 1: the first element becomes the entry point with no links; a new
 *     element takes M links on every layer it belongs to, layer 0 included;
 *     all of W is the entry set of the next layer; elements are inserted in
 *     id order.
 *   - Alg. 5: ef below K is raised to K; fewer than K results are padded with
 *     id -1 and distance +inf; results are sorted by (distance, id).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OR_EXPORT __attribute__((visibility("default")))
#define OR_NONE 0xFFFFFFFFu

enum { OR_L2 = 0, OR_IP = 1 };

typedef struct {
    float d;
    uint32_t id;
} item;

/* key(a) < key(b) in the (distance, id) order. */
static int key_less(item a, item b) { return a.d < b.d || (a.d == b.d && a.id < b.id); }

/* ---------------------------------------------------------------- distance */

static double dist64(int metric, const float *a, const float *b, uint32_t dim) {
    double s = 0.0;
    if (metric == OR_L2) {
        for (uint32_t j = 0; j < dim; ++j) {
            double t = (double)a[j] - (double)b[j];
            s += t * t;
        }
        return s;
    }
    for (uint32_t j = 0; j < dim; ++j) s += (double)a[j] * (double)b[j];
    return 1.0 - s;
}

/* --------------------------------------------------------------- the graph */

typedef struct {
    uint32_t n, dim, metric;
    uint32_t M, Mmax, Mmax0, efC;
    double mL;
    uint64_t seed;
    int heuristic, extend, keep_pruned;
    int rerank;        /* re-score the final W with the fp32 vectors (Alg. 5's last line) */
    const float *X;    /* [n][dim], borrowed from the caller                */
    const float *XQ;   /* [n][dim] decoded low-precision values, or NULL    */
    const float *SQ;   /* [n] per-vector scale of XQ                         */
    uint8_t *level;    /* [n]                                               */
    uint32_t *cnt0;    /* [n]          layer-0 list lengths                 */
    uint32_t *adj0;    /* [n][Mmax0+1] layer-0 lists                        */
    int64_t *uoff;     /* [n]          row of layer 1 in the upper store, -1 */
    uint32_t *ucnt;    /* [rows]                                            */
    uint32_t *uadj;    /* [rows][Mmax+1]                                    */
    uint64_t rows;
    uint32_t n_inserted;
    int64_t entry;     /* entry point, -1 while empty                       */
    int max_level;     /* L, the level of the entry point                   */
    struct searcher *ws; /* workspace used by INSERT                         */
} graph;

static uint32_t *nbr(const graph *g, uint32_t e, int lc, uint32_t **cnt) {
    if (lc == 0) {
        *cnt = &g->cnt0[e];
        return g->adj0 + (uint64_t)e * (g->Mmax0 + 1);
    }
    uint64_t row = (uint64_t)g->uoff[e] + (uint64_t)(lc - 1);
    *cnt = &g->ucnt[row];
    return g->uadj + row * (g->Mmax + 1);
}

/*
 * Distance to a low-precision copy: the stored value of coordinate j is
 * s * xq_j, formed exactly in double (xq_j is a decoded bf16/fp8 value, s a
 * float), so only the final rounding to float differs from exact arithmetic.
 */
static double dist64_q(int metric, const float *q, const float *xq, double s, uint32_t dim) {
    double acc = 0.0;
    if (metric == OR_L2) {
        for (uint32_t j = 0; j < dim; ++j) {
            double t = (double)q[j] - s * (double)xq[j];
            acc += t * t;
        }
        return acc;
    }
    for (uint32_t j = 0; j < dim; ++j) acc += (double)q[j] * (s * (double)xq[j]);
    return 1.0 - acc;
}

static float dkey(const graph *g, const float *q, uint32_t e) {
    if (g->XQ)
        return (float)dist64_q((int)g->metric, q, g->XQ + (uint64_t)e * g->dim, (double)g->SQ[e], g->dim);
    return (float)dist64((int)g->metric, q, g->X + (uint64_t)e * g->dim, g->dim);
}

/* ----------------------------------------------------------- binary heaps */

typedef struct {
    item *a;
    size_t n, cap;
    int is_max; /* 1: furthest on top (W), 0: nearest on top (C) */
} heap;

static int h_above(const heap *h, item x, item y) { return h->is_max ? key_less(y, x) : key_less(x, y); }

static void h_reserve(heap *h, size_t cap) {
    if (cap <= h->cap) return;
    size_t c = h->cap ? h->cap : 64;
    while (c < cap) c *= 2;
    h->a = (item *)realloc(h->a, c * sizeof(item));
    if (!h->a) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    h->cap = c;
}

static void h_push(heap *h, item x) {
    h_reserve(h, h->n + 1);
    size_t i = h->n++;
    while (i > 0) {
        size_t p = (i - 1) / 2;
        if (!h_above(h, x, h->a[p])) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i] = x;
}

static item h_pop(heap *h) {
    item top = h->a[0];
    item x = h->a[--h->n];
    size_t i = 0;
    for (;;) {
        size_t l = 2 * i + 1, r = l + 1, b = i;
        item bx = x;
        if (l < h->n && h_above(h, h->a[l], bx)) { b = l; bx = h->a[l]; }
        if (r < h->n && h_above(h, h->a[r], bx)) { b = r; bx = h->a[r]; }
        if (b == i) break;
        h->a[i] = h->a[b];
        i = b;
    }
    if (h->n) h->a[i] = x;
    return top;
}

/* ------------------------------------------------------ search workspace */

typedef struct searcher {
    uint32_t *vis; /* visited stamps, one per element                   */
    uint32_t gen;
    uint32_t n;
    heap C, W;
    uint64_t n_dist[64], n_exp[64]; /* per-layer counters of the last search */
} searcher;

static searcher *ws_new(uint32_t n) {
    searcher *s = (searcher *)calloc(1, sizeof(searcher));
    s->vis = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
    s->n = n;
    s->W.is_max = 1;
    return s;
}

static void ws_free(searcher *s) {
    if (!s) return;
    free(s->vis);
    free(s->C.a);
    free(s->W.a);
    free(s);
}

static uint32_t next_gen(searcher *s) {
    if (++s->gen == 0) {
        memset(s->vis, 0, (size_t)s->n * sizeof(uint32_t));
        s->gen = 1;
    }
    return s->gen;
}

/* --------------------------------------------- learned early termination */

/*
 * The learned stop rule (an addition to the paper, which stops only when the
 * nearest candidate is further than the furthest element of W, Alg. 2).
 * Every LT layer-0 expansions (at most LMAX checkpoints) a 24-value feature
 * vector of the search state is formed; a 24-64-64-2 perceptron with BF16
 * weights scores it.  Output 0 is a stop logit: the search ends when it
 * exceeds tau.  Output 1, at the first checkpoint only, asks for j halvings
 * of ef (j = floor(0.5 - out1) clamped to [0, jmax]); W then keeps its ef
 * nearest elements.  All feature arithmetic is IEEE float (add, subtract,
 * multiply, divide); the network multiplies BF16 values (exact in float) and
 * accumulates in float in input order, so the result is reproducible bit for
 * bit.
 */
static int cmp_item(const void *pa, const void *pb);

#define LF 24 /* features */
#define LH 64 /* hidden width */

typedef struct {
    int T, max_ckpt, K, jmax;
    const float *w1, *b1, *w2, *b2, *w3, *b3; /* NULL w1: trace only, no decisions */
    float tau;
    /* per-query outputs (trace arrays may be NULL) */
    float *feat;     /* [max_ckpt][LF]                         */
    int32_t *topk;   /* [max_ckpt][K]                          */
    int n_ckpt;      /* checkpoints reached                    */
    int stopped_at;  /* checkpoint at which the rule stopped, 0 */
    uint32_t ef_end; /* ef after the adaptive step             */
    /* state */
    uint32_t n_exp_upper;
    float d_start, d_best_prev, d_k_prev;
    int32_t prev[64];
    int n_prev;
} learn_ctx;

static float lratio(float a, float b) {
    float den = fabsf(b) + 1e-20f;
    float r = a / den;
    return r > 1e6f ? 1e6f : (r < -1e6f ? -1e6f : r);
}

static float bf16_round(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7FFFu + lsb) & 0xFFFF0000u;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

/* The perceptron on one feature vector: out[0] stop logit, out[1] ef step. */
static void mlp_forward(const learn_ctx *lx, const float *f, float *out) {
    float x[LF], h1[LH], h2[LH];
    for (int i = 0; i < LF; ++i) x[i] = bf16_round(f[i]);
    for (int o = 0; o < LH; ++o) {
        float acc = lx->b1[o];
        for (int i = 0; i < LF; ++i) acc = acc + lx->w1[o * LF + i] * x[i];
        h1[o] = bf16_round(acc > 0.0f ? acc : 0.0f);
    }
    for (int o = 0; o < LH; ++o) {
        float acc = lx->b2[o];
        for (int i = 0; i < LH; ++i) acc = acc + lx->w2[o * LH + i] * h1[i];
        h2[o] = bf16_round(acc > 0.0f ? acc : 0.0f);
    }
    for (int o = 0; o < 2; ++o) {
        float acc = lx->b3[o];
        for (int i = 0; i < LH; ++i) acc = acc + lx->w3[o * LH + i] * h2[i];
        out[o] = acc;
    }
}

/*
 * Checkpoint after `e` layer-0 expansions.  W (max-heap) and C (min-heap) are
 * the state of Alg. 2; the next element Alg. 2 would expand is the top of C
 * when its key does not exceed the furthest key of W.  Returns 1 to stop.
 */
static int checkpoint(learn_ctx *lx, heap *W, heap *C, uint32_t e, uint32_t *ef) {
    int ck = ++lx->n_ckpt;
    size_t n = W->n;
    item *ws = (item *)malloc(sizeof(item) * (n ? n : 1));
    memcpy(ws, W->a, sizeof(item) * n);
    qsort(ws, n, sizeof(item), cmp_item);
    uint32_t K = (uint32_t)lx->K;
    uint32_t kk = n < K ? (uint32_t)n : K;
    float d_best = ws[0].d, d_k = ws[kk - 1].d, d_f = ws[n - 1].d;
    item f = ws[n - 1];
    int has_next = C->n > 0 && !key_less(f, C->a[0]);
    uint32_t pos = (uint32_t)n, n_unexp = 0;
    if (has_next) {
        pos = 0;
        while (pos < n && key_less(ws[pos], C->a[0])) ++pos;
    }
    for (size_t i = 0; i < C->n; ++i) n_unexp += !key_less(f, C->a[i]);
    float d_next = has_next ? ws[pos].d : d_f;
    uint32_t changed = 0;
    for (uint32_t i = 0; i < kk; ++i) {
        int seen = 0;
        for (int j = 0; j < lx->n_prev; ++j) seen |= lx->prev[j] == (int32_t)ws[i].id;
        changed += !seen;
    }
    if (ck == 1) {
        lx->d_best_prev = d_best;
        lx->d_k_prev = d_k;
    }
    float ff[LF];
    float fe = (float)*ef;
    ff[0] = (float)e / fe;
    ff[1] = (float)e / 256.0f;
    ff[2] = (float)lx->n_exp_upper / 16.0f;
    ff[3] = (float)n / fe;
    ff[4] = (float)pos / fe;
    ff[5] = (float)n_unexp / fe;
    ff[6] = (float)changed / (float)K;
    ff[7] = (float)ck / 32.0f;
    ff[8] = lratio(d_best, lx->d_start);
    ff[9] = lratio(d_k, lx->d_start);
    ff[10] = lratio(d_f, lx->d_start);
    ff[11] = lratio(d_next, lx->d_start);
    ff[12] = lratio(d_best, d_k);
    ff[13] = lratio(d_k, d_f);
    ff[14] = lratio(d_next, d_k);
    ff[15] = lratio(lx->d_k_prev, d_k);
    ff[16] = lratio(lx->d_best_prev, d_best);
    ff[17] = lratio(d_k - d_best, d_f - d_best);
    ff[18] = fe / 512.0f;
    ff[19] = (float)K / 100.0f;
    ff[20] = lratio(d_next - d_k, d_f - d_best);
    ff[21] = d_next < d_k ? 1.0f : 0.0f;
    ff[22] = pos < K ? 1.0f : 0.0f;
    ff[23] = 1.0f;
    if (lx->feat) memcpy(lx->feat + (size_t)(ck - 1) * LF, ff, sizeof(ff));
    if (lx->topk)
        for (uint32_t i = 0; i < K; ++i) lx->topk[(size_t)(ck - 1) * K + i] = i < kk ? (int32_t)ws[i].id : -1;
    lx->n_prev = (int)kk;
    for (uint32_t i = 0; i < kk; ++i) lx->prev[i] = (int32_t)ws[i].id;
    lx->d_best_prev = d_best;
    lx->d_k_prev = d_k;
    free(ws);
    if (!lx->w1) return 0;
    float out[2];
    mlp_forward(lx, ff, out);
    if (ck == 1 && lx->jmax > 0) {
        int j = (int)floorf(0.5f - out[1]);
        j = j < 0 ? 0 : (j > lx->jmax ? lx->jmax : j);
        uint32_t ne = *ef >> j;
        if (ne < K) ne = K;
        if (ne < *ef) {
            *ef = ne;
            while (W->n > ne) h_pop(W);
        }
    }
    if (out[0] > lx->tau) {
        lx->stopped_at = ck;
        return 1;
    }
    return 0;
}

/*
 * SEARCH-LAYER (Alg. 2).  On return s->W holds the result (heap order).
 * ep: enter points (ids), q: query vector.
 */
static void search_layer_l(const graph *g, searcher *s, const float *q, const uint32_t *ep, size_t n_ep,
                           uint32_t ef, int lc, learn_ctx *lx) {
    uint32_t gen = next_gen(s);
    s->C.n = 0;
    s->W.n = 0;
    for (size_t i = 0; i < n_ep; ++i) {
        if (s->vis[ep[i]] == gen) continue;
        s->vis[ep[i]] = gen;
        item it = {dkey(g, q, ep[i]), ep[i]};
        s->n_dist[lc]++;
        h_push(&s->C, it);
        h_push(&s->W, it);
    }
    if (lx) lx->d_start = s->W.a[0].d;
    uint32_t n_exp_here = 0;
    while (s->C.n > 0) {
        item c = h_pop(&s->C);        /* nearest element of C            */
        item f = s->W.a[0];           /* furthest element of W           */
        if (key_less(f, c)) break;    /* all elements of W are evaluated */
        s->n_exp[lc]++;
        ++n_exp_here;
        uint32_t *cnt;
        const uint32_t *nb = nbr(g, c.id, lc, &cnt);
        uint32_t m = *cnt;
        for (uint32_t k = 0; k < m; ++k) {
            uint32_t e = nb[k];
            if (s->vis[e] == gen) continue;
            s->vis[e] = gen;
            f = s->W.a[0];
            item it = {dkey(g, q, e), e};
            s->n_dist[lc]++;
            if (key_less(it, f) || s->W.n < ef) {
                h_push(&s->C, it);
                h_push(&s->W, it);
                if (s->W.n > ef) h_pop(&s->W);
            }
        }
        if (lx && n_exp_here % (uint32_t)lx->T == 0 && lx->n_ckpt < lx->max_ckpt &&
            checkpoint(lx, &s->W, &s->C, n_exp_here, &ef))
            break;
    }
    if (lx) lx->ef_end = ef;
}

static void search_layer(const graph *g, searcher *s, const float *q, const uint32_t *ep, size_t n_ep,
                         uint32_t ef, int lc) {
    search_layer_l(g, s, q, ep, n_ep, ef, lc, NULL);
}

static int cmp_item(const void *pa, const void *pb) {
    item a = *(const item *)pa, b = *(const item *)pb;
    return key_less(a, b) ? -1 : (key_less(b, a) ? 1 : 0);
}

/* ------------------------------------------------------ neighbor selection */

/* SELECT-NEIGHBORS-SIMPLE (Alg. 3): the M nearest of cand (distances to the base). */
static size_t select_simple(item *cand, size_t n, uint32_t M, uint32_t *out) {
    qsort(cand, n, sizeof(item), cmp_item);
    size_t m = n < M ? n : M;
    for (size_t i = 0; i < m; ++i) out[i] = cand[i].id;
    return m;
}

/*
 * SELECT-NEIGHBORS-HEURISTIC (Alg. 4).  base: vector of the base element,
 * base_id: its id (excluded when extending), cand: candidates with distances
 * to the base.
 */
static size_t select_heuristic(const graph *g, searcher *s, const float *base, uint32_t base_id, const item *cand,
                               size_t n, uint32_t M, int lc, int extend, int keep_pruned, uint32_t *out) {
    heap Wq = {0}, Wd = {0};
    for (size_t i = 0; i < n; ++i) h_push(&Wq, cand[i]);
    if (extend) {
        uint32_t gen = next_gen(s);
        for (size_t i = 0; i < n; ++i) s->vis[cand[i].id] = gen;
        s->vis[base_id] = gen;
        for (size_t i = 0; i < n; ++i) {
            uint32_t *cnt;
            const uint32_t *nb = nbr(g, cand[i].id, lc, &cnt);
            for (uint32_t k = 0; k < *cnt; ++k) {
                uint32_t e = nb[k];
                if (s->vis[e] == gen) continue;
                s->vis[e] = gen;
                item it = {dkey(g, base, e), e};
                h_push(&Wq, it);
            }
        }
    }
    size_t r = 0;
    while (Wq.n > 0 && r < M) {
        item e = h_pop(&Wq);
        const float *xe = g->X + (uint64_t)e.id * g->dim;
        int keep = 1;
        for (size_t j = 0; j < r; ++j) {
            float der = (float)dist64((int)g->metric, xe, g->X + (uint64_t)out[j] * g->dim, g->dim);
            if (!(e.d < der)) { keep = 0; break; }
        }
        if (keep) out[r++] = e.id;
        else h_push(&Wd, e);
    }
    if (keep_pruned)
        while (Wd.n > 0 && r < M) out[r++] = h_pop(&Wd).id;
    free(Wq.a);
    free(Wd.a);
    return r;
}

static size_t select_neighbors(const graph *g, searcher *s, const float *base, uint32_t base_id, item *cand,
                               size_t n, uint32_t M, int lc, uint32_t *out) {
    if (g->heuristic) return select_heuristic(g, s, base, base_id, cand, n, M, lc, g->extend, g->keep_pruned, out);
    return select_simple(cand, n, M, out);
}

/* ---------------------------------------------------------------- levels */

static uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

/* The level draw of Alg. 1: l = floor(-ln(unif(0..1)) * mL). */
OR_EXPORT void or_levels(uint64_t seed, uint32_t n, double mL, uint8_t *out) {
    for (uint32_t i = 0; i < n; ++i) {
        uint64_t r = splitmix64(seed ^ (uint64_t)i) >> 11;
        double U = (double)(r + 1) * 0x1.0p-53;
        double l = floor(-log(U) * mL);
        if (l > 255.0) l = 255.0;
        out[i] = (uint8_t)l;
    }
}

/* ---------------------------------------------------------------- INSERT */

static void alloc_lists(graph *g) {
    g->cnt0 = (uint32_t *)calloc(g->n ? g->n : 1, sizeof(uint32_t));
    g->adj0 = (uint32_t *)malloc(((size_t)g->n * (g->Mmax0 + 1) + 1) * sizeof(uint32_t));
    g->uoff = (int64_t *)malloc(((size_t)g->n + 1) * sizeof(int64_t));
    uint64_t rows = 0;
    for (uint32_t i = 0; i < g->n; ++i) {
        g->uoff[i] = g->level[i] ? (int64_t)rows : -1;
        rows += g->level[i];
    }
    g->rows = rows;
    g->ucnt = (uint32_t *)calloc(rows ? rows : 1, sizeof(uint32_t));
    g->uadj = (uint32_t *)malloc(((size_t)rows * (g->Mmax + 1) + 1) * sizeof(uint32_t));
    if (!g->cnt0 || !g->adj0 || !g->uoff || !g->ucnt || !g->uadj) {
        fprintf(stderr, "oracle: out of memory\n");
        abort();
    }
}

OR_EXPORT graph *or_create(const float *X, uint32_t n, uint32_t dim, uint32_t metric, uint32_t M, uint32_t Mmax,
                           uint32_t Mmax0, uint32_t efC, double mL, uint64_t seed, int heuristic, int extend,
                           int keep_pruned) {
    graph *g = (graph *)calloc(1, sizeof(graph));
    g->n = n; g->dim = dim; g->metric = metric;
    g->M = M; g->Mmax = Mmax; g->Mmax0 = Mmax0; g->efC = efC;
    g->mL = mL; g->seed = seed;
    g->heuristic = heuristic; g->extend = extend; g->keep_pruned = keep_pruned;
    g->X = X;
    g->level = (uint8_t *)malloc(n ? n : 1);
    or_levels(seed, n, mL, g->level);
    alloc_lists(g);
    g->entry = -1;
    g->max_level = -1;
    g->ws = ws_new(n);
    return g;
}

/* INSERT (Alg. 1) of element q (its id); elements must be inserted in id order. */
static void insert(graph *g, uint32_t qid) {
    searcher *s = g->ws;
    const float *q = g->X + (uint64_t)qid * g->dim;
    int l = g->level[qid];
    if (g->entry < 0) {               /* first element: entry point, no links */
        g->entry = qid;
        g->max_level = l;
        g->n_inserted++;
        return;
    }
    int L = g->max_level;
    uint32_t *ep = (uint32_t *)malloc(sizeof(uint32_t) * ((size_t)g->efC + 1));
    size_t n_ep = 1;
    ep[0] = (uint32_t)g->entry;
    for (int lc = L; lc > l; --lc) {  /* greedy phase, ef = 1 */
        search_layer(g, s, q, ep, n_ep, 1, lc);
        item best = s->W.a[0];
        for (size_t i = 1; i < s->W.n; ++i)
            if (key_less(s->W.a[i], best)) best = s->W.a[i];
        ep[0] = best.id;
        n_ep = 1;
    }
    uint32_t Mcap = g->Mmax0 > g->Mmax ? g->Mmax0 : g->Mmax;
    item *cand = (item *)malloc(sizeof(item) * ((size_t)g->efC + Mcap + 2));
    uint32_t *sel = (uint32_t *)malloc(sizeof(uint32_t) * ((size_t)g->efC + Mcap + 2));
    uint32_t *sel2 = (uint32_t *)malloc(sizeof(uint32_t) * ((size_t)Mcap + 2));
    for (int lc = (L < l ? L : l); lc >= 0; --lc) {
        search_layer(g, s, q, ep, n_ep, g->efC, lc);
        size_t nW = s->W.n;
        for (size_t i = 0; i < nW; ++i) cand[i] = s->W.a[i];
        /* W is also the next layer's entry set */
        for (size_t i = 0; i < nW; ++i) ep[i] = cand[i].id;
        n_ep = nW;
        size_t m = select_neighbors(g, s, q, qid, cand, nW, g->M, lc, sel);
        uint32_t *cq;
        uint32_t *lq = nbr(g, qid, lc, &cq);
        for (size_t i = 0; i < m; ++i) lq[i] = sel[i];
        *cq = (uint32_t)m;
        uint32_t cap = lc == 0 ? g->Mmax0 : g->Mmax;
        for (size_t i = 0; i < m; ++i) {     /* the reverse links */
            uint32_t *ce;
            uint32_t *le = nbr(g, sel[i], lc, &ce);
            le[(*ce)++] = qid;
        }
        for (size_t i = 0; i < m; ++i) {     /* shrink overflowing lists */
            uint32_t e = sel[i];
            uint32_t *ce;
            uint32_t *le = nbr(g, e, lc, &ce);
            if (*ce <= cap) continue;
            const float *xe = g->X + (uint64_t)e * g->dim;
            for (uint32_t k = 0; k < *ce; ++k) {
                cand[k].id = le[k];
                cand[k].d = dkey(g, xe, le[k]);
            }
            size_t mm = select_neighbors(g, s, xe, e, cand, *ce, cap, lc, sel2);
            for (size_t k = 0; k < mm; ++k) le[k] = sel2[k];
            *ce = (uint32_t)mm;
        }
        /* select_neighbors may have reordered cand; ep was saved before. */
    }
    if (l > L) {
        g->entry = qid;
        g->max_level = l;
    }
    g->n_inserted++;
    free(ep);
    free(cand);
    free(sel);
    free(sel2);
}

/* Insert elements [start, end) in id order; returns the number inserted so far. */
OR_EXPORT uint32_t or_insert_range(graph *g, uint32_t start, uint32_t end) {
    if (start != g->n_inserted || end > g->n || start > end) return (uint32_t)-1;
    for (uint32_t i = start; i < end; ++i) insert(g, i);
    return g->n_inserted;
}

OR_EXPORT void or_free(graph *g) {
    if (!g) return;
    free(g->level); free(g->cnt0); free(g->adj0); free(g->uoff); free(g->ucnt); free(g->uadj);
    ws_free(g->ws);
    free(g);
}

/* -------------------------------------------------------- K-NN-SEARCH */

/* K-NN-SEARCH (Alg. 5) of one query using workspace s. */
static void knn_search_l(const graph *g, searcher *s, const float *q, uint32_t K, uint32_t ef, int32_t *ids,
                         float *dists, uint64_t *counters, learn_ctx *lx) {
    memset(s->n_dist, 0, sizeof(s->n_dist));
    memset(s->n_exp, 0, sizeof(s->n_exp));
    uint32_t efe = ef < K ? K : ef;
    size_t nres = 0;
    if (g->entry >= 0) {
        uint32_t ep = (uint32_t)g->entry;
        for (int lc = g->max_level; lc >= 1; --lc) {
            search_layer(g, s, q, &ep, 1, 1, lc);
            item best = s->W.a[0];
            for (size_t i = 1; i < s->W.n; ++i)
                if (key_less(s->W.a[i], best)) best = s->W.a[i];
            ep = best.id;
        }
        if (lx) lx->n_exp_upper = (uint32_t)(s->n_exp[1] + s->n_exp[2] + s->n_exp[3] + s->n_exp[4] + s->n_exp[5] +
                                             s->n_exp[6] + s->n_exp[7] + s->n_exp[8]);
        search_layer_l(g, s, q, &ep, 1, efe, 0, lx);
        nres = s->W.n;
        if (g->rerank) /* K nearest of W by the exact distance to the fp32 vectors */
            for (size_t i = 0; i < nres; ++i)
                s->W.a[i].d = (float)dist64((int)g->metric, q, g->X + (uint64_t)s->W.a[i].id * g->dim, g->dim);
        qsort(s->W.a, nres, sizeof(item), cmp_item);
    }
    for (uint32_t k = 0; k < K; ++k) {
        if (k < nres) { ids[k] = (int32_t)s->W.a[k].id; dists[k] = s->W.a[k].d; }
        else { ids[k] = -1; dists[k] = INFINITY; }
    }
    if (counters) {
        uint64_t dt = 0, et = 0;
        for (int l = 0; l < 64; ++l) { dt += s->n_dist[l]; et += s->n_exp[l]; }
        counters[0] = dt;             /* distance evaluations, all layers */
        counters[1] = et;             /* expansions, all layers            */
        counters[2] = s->n_dist[0];   /* distance evaluations, layer 0     */
        counters[3] = s->n_exp[0];    /* expansions, layer 0               */
    }
}

static void knn_search(const graph *g, searcher *s, const float *q, uint32_t K, uint32_t ef, int32_t *ids,
                       float *dists, uint64_t *counters) {
    knn_search_l(g, s, q, K, ef, ids, dists, counters, NULL);
}

typedef struct {
    const graph *g;
    const float *Q;
    uint32_t K, ef, lo, hi;
    int32_t *ids;
    float *dists;
    uint64_t *counters;
} search_job;

static void *search_worker(void *p) {
    search_job *j = (search_job *)p;
    searcher *s = ws_new(j->g->n);
    for (uint32_t i = j->lo; i < j->hi; ++i)
        knn_search(j->g, s, j->Q + (uint64_t)i * j->g->dim, j->K, j->ef, j->ids + (uint64_t)i * j->K,
                   j->dists + (uint64_t)i * j->K, j->counters ? j->counters + 4ull * i : NULL);
    ws_free(s);
    return NULL;
}

/* Batched K-NN-SEARCH: queries are independent, split over nthreads threads. */
OR_EXPORT void or_search(const graph *g, const float *Q, uint32_t nq, uint32_t K, uint32_t ef, int32_t *ids,
                         float *dists, uint64_t *counters, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    if ((uint32_t)nthreads > nq) nthreads = nq ? (int)nq : 1;
    pthread_t th[256];
    search_job jobs[256];
    if (nthreads > 256) nthreads = 256;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (search_job){g, Q, K, ef, (uint32_t)((uint64_t)nq * t / nthreads),
                               (uint32_t)((uint64_t)nq * (t + 1) / nthreads), ids, dists, counters};
        if (nthreads == 1) search_worker(&jobs[t]);
        else pthread_create(&th[t], NULL, search_worker, &jobs[t]);
    }
    if (nthreads > 1)
        for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* One SEARCH-LAYER call from explicit enter points; W is returned sorted. */
OR_EXPORT uint32_t or_search_layer(const graph *g, const float *q, const uint32_t *ep, uint32_t n_ep, uint32_t ef,
                                   int lc, int32_t *ids, float *dists, uint64_t *n_dist) {
    searcher *s = ws_new(g->n);
    memset(s->n_dist, 0, sizeof(s->n_dist));
    search_layer(g, s, q, ep, n_ep, ef, lc);
    qsort(s->W.a, s->W.n, sizeof(item), cmp_item);
    uint32_t m = (uint32_t)s->W.n;
    for (uint32_t i = 0; i < m; ++i) { ids[i] = (int32_t)s->W.a[i].id; dists[i] = s->W.a[i].d; }
    if (n_dist) *n_dist = s->n_dist[lc];
    ws_free(s);
    return m;
}

/* Alg. 4 on an explicit candidate list, against the graph's vectors and layer lc. */
OR_EXPORT uint32_t or_select_heuristic(const graph *g, uint32_t base_id, const uint32_t *cand_ids, uint32_t n,
                                       uint32_t M, int lc, int extend, int keep_pruned, uint32_t *out) {
    searcher *s = ws_new(g->n);
    const float *base = g->X + (uint64_t)base_id * g->dim;
    item *c = (item *)malloc(sizeof(item) * (n + 1));
    for (uint32_t i = 0; i < n; ++i) c[i] = (item){dkey(g, base, cand_ids[i]), cand_ids[i]};
    size_t m = select_heuristic(g, s, base, base_id, c, n, M, lc, extend, keep_pruned, out);
    free(c);
    ws_free(s);
    return (uint32_t)m;
}

/* ---------------------------------------------------------- brute force */

typedef struct {
    const float *X, *Q;
    uint32_t n, dim, metric, K, lo, hi;
    int by_f32;
    int32_t *ids;
    double *d64;
} bf_job;

typedef struct {
    double d;
    float f;
    uint32_t id;
} bf_item;

static int bf_cmp64(const void *pa, const void *pb) {
    const bf_item *a = (const bf_item *)pa, *b = (const bf_item *)pb;
    if (a->d != b->d) return a->d < b->d ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id);
}

static int bf_cmp32(const void *pa, const void *pb) {
    const bf_item *a = (const bf_item *)pa, *b = (const bf_item *)pb;
    if (a->f != b->f) return a->f < b->f ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id);
}

static void *bf_worker(void *p) {
    bf_job *j = (bf_job *)p;
    bf_item *all = (bf_item *)malloc(sizeof(bf_item) * (j->n ? j->n : 1));
    for (uint32_t qi = j->lo; qi < j->hi; ++qi) {
        const float *q = j->Q + (uint64_t)qi * j->dim;
        for (uint32_t i = 0; i < j->n; ++i) {
            double d = dist64((int)j->metric, q, j->X + (uint64_t)i * j->dim, j->dim);
            all[i] = (bf_item){d, (float)d, i};
        }
        qsort(all, j->n, sizeof(bf_item), j->by_f32 ? bf_cmp32 : bf_cmp64);
        for (uint32_t k = 0; k < j->K; ++k) {
            j->ids[(uint64_t)qi * j->K + k] = k < j->n ? (int32_t)all[k].id : -1;
            j->d64[(uint64_t)qi * j->K + k] = k < j->n ? all[k].d : INFINITY;
        }
    }
    free(all);
    return NULL;
}

/*
 * Exact K-NN by computing all n distances (the problem statement of Sec. 1).
 * by_f32 = 0 orders by the double-precision distance, 1 by the fp32 key.
 */
OR_EXPORT void or_bruteforce(const float *X, uint32_t n, uint32_t dim, uint32_t metric, const float *Q, uint32_t nq,
                             uint32_t K, int by_f32, int32_t *ids, double *d64, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    if ((uint32_t)nthreads > nq) nthreads = nq ? (int)nq : 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    bf_job jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (bf_job){X, Q, n, dim, metric, K, (uint32_t)((uint64_t)nq * t / nthreads),
                           (uint32_t)((uint64_t)nq * (t + 1) / nthreads), by_f32, ids, d64};
        if (nthreads == 1) bf_worker(&jobs[t]);
        else pthread_create(&th[t], NULL, bf_worker, &jobs[t]);
    }
    if (nthreads > 1)
        for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* Exact distances of explicit (query, id) pairs, fp64 and the fp32 key. */
OR_EXPORT void or_pair_dist(const float *X, uint32_t dim, uint32_t metric, const float *Q, const int32_t *ids,
                            uint64_t n_pairs, uint32_t per_query, double *d64) {
    for (uint64_t p = 0; p < n_pairs; ++p) {
        int32_t id = ids[p];
        const float *q = Q + (p / per_query) * dim;
        d64[p] = id < 0 ? INFINITY : dist64((int)metric, q, X + (uint64_t)id * dim, dim);
    }
}

/* ------------------------------------------------------- export / import */

OR_EXPORT void or_info(const graph *g, uint64_t *out) {
    out[0] = g->n; out[1] = g->dim; out[2] = g->metric; out[3] = g->M; out[4] = g->Mmax; out[5] = g->Mmax0;
    out[6] = g->efC; out[7] = (uint64_t)(g->max_level < 0 ? 0 : g->max_level);
    out[8] = (uint64_t)(g->entry < 0 ? 0 : g->entry); out[9] = g->rows; out[10] = g->n_inserted;
    out[11] = g->seed;
}

/*
 * Packed form: levels[n] u8, adj0[n][Mmax0] u32 padded with 0xFFFFFFFF,
 * upper_off[n] i32 (row of layer 1, -1 when the element has level 0),
 * adjU[rows][Mmax] u32 padded; an element's rows for layers 1..level are
 * consecutive.
 */
OR_EXPORT void or_export(const graph *g, uint8_t *levels, uint32_t *adj0, int32_t *upper_off, uint32_t *adjU) {
    memcpy(levels, g->level, g->n);
    for (uint32_t i = 0; i < g->n; ++i) {
        const uint32_t *src = g->adj0 + (uint64_t)i * (g->Mmax0 + 1);
        uint32_t *dst = adj0 + (uint64_t)i * g->Mmax0;
        for (uint32_t k = 0; k < g->Mmax0; ++k) dst[k] = k < g->cnt0[i] ? src[k] : OR_NONE;
        upper_off[i] = (int32_t)g->uoff[i];
    }
    for (uint64_t r = 0; r < g->rows; ++r)
        for (uint32_t k = 0; k < g->Mmax; ++k)
            adjU[r * g->Mmax + k] = k < g->ucnt[r] ? g->uadj[r * (g->Mmax + 1) + k] : OR_NONE;
}

/* Rebuild a searchable graph from the packed form (e.g. read from a file, or a hand-made graph). */
OR_EXPORT graph *or_import(const float *X, uint32_t n, uint32_t dim, uint32_t metric, uint32_t M, uint32_t Mmax,
                           uint32_t Mmax0, int64_t entry, int max_level, const uint8_t *levels, const uint32_t *adj0,
                           const uint32_t *adjU) {
    graph *g = (graph *)calloc(1, sizeof(graph));
    g->n = n; g->dim = dim; g->metric = metric; g->M = M; g->Mmax = Mmax; g->Mmax0 = Mmax0;
    g->X = X;
    g->level = (uint8_t *)malloc(n ? n : 1);
    memcpy(g->level, levels, n);
    alloc_lists(g);
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t c = 0;
        for (uint32_t k = 0; k < Mmax0; ++k) {
            uint32_t v = adj0[(uint64_t)i * Mmax0 + k];
            if (v != OR_NONE) g->adj0[(uint64_t)i * (Mmax0 + 1) + c++] = v;
        }
        g->cnt0[i] = c;
    }
    for (uint64_t r = 0; r < g->rows; ++r) {
        uint32_t c = 0;
        for (uint32_t k = 0; k < Mmax; ++k) {
            uint32_t v = adjU[r * Mmax + k];
            if (v != OR_NONE) g->uadj[r * (Mmax + 1) + c++] = v;
        }
        g->ucnt[r] = c;
    }
    g->entry = entry;
    g->max_level = max_level;
    g->n_inserted = n;
    g->ws = ws_new(n);
    return g;
}

/* Swap the vector store (same shape). */
OR_EXPORT void or_set_vectors(graph *g, const float *X) { g->X = X; }

/*
 * Traverse over a low-precision copy (decoded values XQ [n][dim] and scales
 * SQ [n]) and re-rank the final W with the fp32 vectors; NULL restores the
 * plain search.
 */
OR_EXPORT void or_set_lowp(graph *g, const float *XQ, const float *SQ) {
    g->XQ = XQ;
    g->SQ = SQ;
    g->rerank = XQ != NULL;
}

/* ------------------------------------------------------- quantisation */

/* float -> bfloat16, round to nearest even (NaN kept quiet). */
static uint16_t bf16_rne(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);
    uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

static float bf16_value(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

/*
 * OCP FP8 E4M3: 1 sign, 4 exponent bits (bias 7), 3 mantissa bits; no
 * infinities; S.1111.111 is NaN; largest finite magnitude 448 (S.1111.110);
 * subnormals m * 2^-9.
 */
static float e4m3_value(uint8_t b) {
    int sgn = b >> 7, e = (b >> 3) & 15, m = b & 7;
    double v = e == 0 ? ldexp((double)m, -9) : ldexp(1.0 + m / 8.0, e - 7);
    if (e == 15 && m == 7) v = NAN;
    return (float)(sgn ? -v : v);
}

/* Nearest E4M3 code to a finite float, ties to the even code, saturating at +-448. */
static uint8_t e4m3_rne(float f) {
    uint8_t sgn = signbit(f) ? 0x80 : 0; /* E4M3 encodes -0 as S=1, all else 0 */
    double a = fabs((double)f);
    if (a >= 448.0) return sgn | 0x7E;
    /* scan the 127 non-negative finite codes: they increase with the code */
    uint8_t best = 0;
    for (int c = 1; c <= 0x7E; ++c) {
        double v = (double)e4m3_value((uint8_t)c);
        if (v <= a) best = (uint8_t)c;
    }
    double lo = (double)e4m3_value(best);
    if (best < 0x7E) {
        double hi = (double)e4m3_value((uint8_t)(best + 1));
        double dl = a - lo, dh = hi - a;
        if (dh < dl || (dh == dl && (best & 1))) best = (uint8_t)(best + 1);
    }
    return (uint8_t)(sgn | best);
}

OR_EXPORT void or_quantize_bf16(const float *X, uint64_t n, uint32_t dim, uint16_t *out, float *decoded) {
    for (uint64_t i = 0; i < n * dim; ++i) {
        out[i] = bf16_rne(X[i]);
        if (decoded) decoded[i] = bf16_value(out[i]);
    }
}

/*
 * Per-vector scaled FP8: s = max_j |x_j| / 448 (s = 1 for an all-zero row),
 * code_j = E4M3 nearest to x_j / s (both divisions in float).
 */
OR_EXPORT void or_quantize_fp8(const float *X, uint64_t n, uint32_t dim, uint8_t *out, float *scale, float *decoded) {
    for (uint64_t i = 0; i < n; ++i) {
        const float *x = X + i * dim;
        float mx = 0.0f;
        for (uint32_t j = 0; j < dim; ++j) mx = fabsf(x[j]) > mx ? fabsf(x[j]) : mx;
        float s = mx > 0.0f ? mx / 448.0f : 1.0f;
        scale[i] = s;
        for (uint32_t j = 0; j < dim; ++j) {
            uint8_t c = e4m3_rne(x[j] / s);
            out[i * dim + j] = c;
            if (decoded) decoded[i * dim + j] = e4m3_value(c);
        }
    }
}

OR_EXPORT float or_e4m3_value(uint8_t b) { return e4m3_value(b); }
OR_EXPORT uint8_t or_e4m3_rne(float f) { return e4m3_rne(f); }
OR_EXPORT uint16_t or_bf16_rne(float f) { return bf16_rne(f); }

/* ---------------------------------------------- learned search, traces */

typedef struct {
    const graph *g;
    const float *Q;
    uint32_t K, ef, lo, hi;
    learn_ctx proto;
    int32_t *ids;
    float *dists;
    uint64_t *counters;
    float *feat;     /* [nq][max_ckpt][LF] or NULL */
    int32_t *topk;   /* [nq][max_ckpt][K] or NULL  */
    int32_t *info;   /* [nq][3]: checkpoints, stopped_at, ef at the end */
} learn_job;

static void *learn_worker(void *p) {
    learn_job *j = (learn_job *)p;
    searcher *s = ws_new(j->g->n);
    for (uint32_t i = j->lo; i < j->hi; ++i) {
        learn_ctx lx = j->proto;
        lx.feat = j->feat ? j->feat + (size_t)i * lx.max_ckpt * LF : NULL;
        lx.topk = j->topk ? j->topk + (size_t)i * lx.max_ckpt * lx.K : NULL;
        knn_search_l(j->g, s, j->Q + (uint64_t)i * j->g->dim, j->K, j->ef, j->ids + (uint64_t)i * j->K,
                     j->dists + (uint64_t)i * j->K, j->counters ? j->counters + 4ull * i : NULL, &lx);
        if (j->info) {
            j->info[3 * i] = lx.n_ckpt;
            j->info[3 * i + 1] = lx.stopped_at;
            j->info[3 * i + 2] = (int32_t)lx.ef_end;
        }
    }
    ws_free(s);
    return NULL;
}

/*
 * K-NN-SEARCH with the learned stop rule (net != NULL) or with a trace of
 * the checkpoint features and top-K lists only (net == NULL).
 * net: w1[64][24], b1[64], w2[64][64], b2[64], w3[2][64], b3[2] as floats
 * (weights already BF16 values), concatenated.
 */
OR_EXPORT void or_search_learned(const graph *g, const float *Q, uint32_t nq, uint32_t K, uint32_t ef, int T,
                                 int max_ckpt, const float *net, float tau, int jmax, int32_t *ids, float *dists,
                                 uint64_t *counters, float *feat, int32_t *topk, int32_t *info, int nthreads) {
    learn_ctx proto;
    memset(&proto, 0, sizeof(proto));
    proto.T = T;
    proto.max_ckpt = max_ckpt;
    proto.K = (int)K;
    proto.jmax = jmax;
    proto.tau = tau;
    if (net) {
        proto.w1 = net;
        proto.b1 = proto.w1 + LH * LF;
        proto.w2 = proto.b1 + LH;
        proto.b2 = proto.w2 + LH * LH;
        proto.w3 = proto.b2 + LH;
        proto.b3 = proto.w3 + 2 * LH;
    }
    if (nthreads < 1) nthreads = 1;
    if ((uint32_t)nthreads > nq) nthreads = nq ? (int)nq : 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    learn_job jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (learn_job){g, Q, K, ef, (uint32_t)((uint64_t)nq * t / nthreads),
                              (uint32_t)((uint64_t)nq * (t + 1) / nthreads), proto, ids, dists, counters, feat, topk,
                              info};
        if (nthreads == 1) learn_worker(&jobs[t]);
        else pthread_create(&th[t], NULL, learn_worker, &jobs[t]);
    }
    if (nthreads > 1)
        for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* The perceptron alone on n feature vectors (for tests of the network arithmetic). */
OR_EXPORT void or_mlp_forward(const float *net, const float *feat, uint32_t n, float *out) {
    learn_ctx lx;
    memset(&lx, 0, sizeof(lx));
    lx.w1 = net;
    lx.b1 = lx.w1 + LH * LF;
    lx.w2 = lx.b1 + LH;
    lx.b2 = lx.w2 + LH * LH;
    lx.w3 = lx.b2 + LH;
    lx.b3 = lx.w3 + 2 * LH;
    for (uint32_t i = 0; i < n; ++i) mlp_forward(&lx, feat + (size_t)i * LF, out + 2 * i);
}
