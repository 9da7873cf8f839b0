/*
 * mls.c — multi-try k-way local search (MLS), oracle-only (test
 * infrastructure; see oracle.h). Sequential form of §III-C, used to measure
 * what the GPU path's LP-only refinement leaves on the table, and a batched
 * form of §IV-C's parallel MLS (orc_mls_batched): a batch takes seeds in
 * queue order while their closed neighbourhoods are disjoint; its searches
 * start from the same partition and marks, then their kept prefixes are
 * replayed in seed order with recomputed gains; a batch of one is the
 * sequential search.
 *
 * What the paper fixes (§III-C, Algorithm 1 of §IV-C for the iteration
 * control):
 *  - a global iteration puts the boundary vertices into a todo list T and
 *    visits them in random order; every vertex starts unmarked;
 *  - a search starts at an unmarked vertex v: v and its neighbours are marked
 *    and inserted into a priority queue keyed by gain; the search repeatedly
 *    moves the vertex of largest gain (moves must respect L_max), marks and
 *    inserts unmarked neighbours of the moved vertex and updates the keys of
 *    neighbours already queued; it stops on an empty queue or by the stopping
 *    rule, and the best partition seen during the search is restored;
 *  - after a local iteration (T exhausted) the moved vertices form the next
 *    todo list (shuffled); another local iteration follows while its gain
 *    exceeds alpha (10%) of the gain of the global iteration so far,
 *    otherwise the next global iteration starts from all boundary vertices;
 *    three global iterations.
 *
 * Readings where the paper is silent (see the design notes):
 *  - gain(v) = max over blocks b adjacent to v, b != block(v), with
 *    B[b] + c(v) <= L_max, of conn(v, b) - conn(v, block(v)); ties -> lowest
 *    b; a vertex with no such block is not queued (and leaves the queue);
 *  - queue order: larger gain first, ties -> lower vertex id; a popped entry
 *    whose gain changed (block weights move with every move) is re-queued
 *    with its current gain;
 *  - the adaptive stopping rule (cited by the paper from another work) is
 *    replaced by a fixed one: stop after max_idle moves without a new best;
 *  - the best partition of a search is the shortest prefix of its moves with
 *    the largest cumulative gain (> 0, else nothing is kept); moved-back
 *    vertices stay marked for the rest of the local iteration;
 *  - random orders are a splitmix64 hash order: key(v) = sm(h ^ v) with
 *    h = sm(sm(sm(seed) ^ (g + 1)) ^ (l + 1)) for global iteration g, local
 *    iteration l; ties by vertex id.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

#define VW(g, v) ((g)->vwgt ? (int64_t)(g)->vwgt[v] : (int64_t)1)
#define EW(g, e) ((g)->adjwgt ? (int64_t)(g)->adjwgt[e] : (int64_t)1)

static void *xcalloc(size_t count, size_t size) {
    void *p = calloc(count ? count : 1, size ? size : 1);
    if (!p) abort();
    return p;
}

static uint64_t mix64(uint64_t x) {  /* splitmix64 finaliser of x + golden gamma */
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

/* gain of moving v (see the readings); returns 0 and sets *ok = 0 when no block qualifies */
static int64_t gain_of(const orc_graph *g, const int32_t *part, const int64_t *B, int32_t k, int64_t lmax, int32_t v,
                       int64_t *conn, int32_t *target, int *ok) {
    const int32_t own = part[v];
    for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) conn[part[g->adjncy[e]]] += EW(g, e);
    int32_t best = -1;
    int64_t best_conn = 0;
    for (int32_t b = 0; b < k; b++) {
        if (b == own || conn[b] <= 0 || B[b] + VW(g, v) > lmax) continue;
        if (best < 0 || conn[b] > best_conn) {
            best = b;
            best_conn = conn[b];
        }
    }
    const int64_t own_conn = conn[own];
    for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) conn[part[g->adjncy[e]]] = 0;
    *ok = best >= 0;
    *target = best;
    return best >= 0 ? best_conn - own_conn : 0;
}

int64_t orc_mls_gain(const orc_graph *g, const int32_t *part, const int64_t *B, int32_t k, int64_t lmax, int32_t v,
                     int32_t *target) {
    int64_t *conn = (int64_t *)xcalloc((size_t)k, sizeof(int64_t));
    int ok = 0;
    const int64_t gn = gain_of(g, part, B, k, lmax, v, conn, target, &ok);
    free(conn);
    if (!ok) *target = -1;
    return gn;
}

/* binary max-heap of (gain, vertex), larger gain first, ties -> lower vertex; pos[v] = slot or -1 */
typedef struct {
    int64_t *key;
    int32_t *ver;
    int32_t *pos;
    int32_t size;
} heap_t;

static int above(const heap_t *h, int32_t i, int32_t j) {
    return h->key[i] > h->key[j] || (h->key[i] == h->key[j] && h->ver[i] < h->ver[j]);
}
static void swap_slots(heap_t *h, int32_t i, int32_t j) {
    int64_t tk = h->key[i];
    int32_t tv = h->ver[i];
    h->key[i] = h->key[j];
    h->ver[i] = h->ver[j];
    h->key[j] = tk;
    h->ver[j] = tv;
    h->pos[h->ver[i]] = i;
    h->pos[h->ver[j]] = j;
}
static void sift_up(heap_t *h, int32_t i) {
    while (i > 0 && above(h, i, (i - 1) / 2)) {
        swap_slots(h, i, (i - 1) / 2);
        i = (i - 1) / 2;
    }
}
static void sift_down(heap_t *h, int32_t i) {
    for (;;) {
        int32_t m = i, l = 2 * i + 1, r = l + 1;
        if (l < h->size && above(h, l, m)) m = l;
        if (r < h->size && above(h, r, m)) m = r;
        if (m == i) return;
        swap_slots(h, i, m);
        i = m;
    }
}
static void heap_push(heap_t *h, int64_t key, int32_t v) {
    int32_t i = h->size++;
    h->key[i] = key;
    h->ver[i] = v;
    h->pos[v] = i;
    sift_up(h, i);
}
static void heap_remove(heap_t *h, int32_t v) {
    int32_t i = h->pos[v];
    h->pos[v] = -1;
    int32_t last = --h->size;
    if (i == last) return;
    h->key[i] = h->key[last];
    h->ver[i] = h->ver[last];
    h->pos[h->ver[i]] = i;
    sift_up(h, i);
    sift_down(h, h->pos[h->ver[i]]);
}
static void heap_update(heap_t *h, int32_t v, int64_t key) {
    int32_t i = h->pos[v];
    h->key[i] = key;
    sift_up(h, i);
    sift_down(h, h->pos[v]);
}

typedef struct {
    uint64_t key;
    int32_t v;
} order_t;
static int cmp_order(const void *a, const void *b) {
    const order_t *x = (const order_t *)a, *y = (const order_t *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->v < y->v ? -1 : (x->v > y->v);
}
static void hash_order(int32_t *list, int32_t len, uint64_t seed, int32_t gi, int32_t li) {
    const uint64_t h = mix64(mix64(mix64(seed) ^ (uint64_t)(gi + 1)) ^ (uint64_t)(li + 1));
    order_t *o = (order_t *)xcalloc((size_t)len, sizeof(order_t));
    for (int32_t i = 0; i < len; i++) {
        o[i].v = list[i];
        o[i].key = mix64(h ^ (uint64_t)(uint32_t)list[i]);
    }
    qsort(o, (size_t)len, sizeof(order_t), cmp_order);
    for (int32_t i = 0; i < len; i++) list[i] = o[i].v;
    free(o);
}

/* state shared by the searches of one call */
typedef struct {
    const orc_graph *g;
    int32_t k;
    int64_t lmax;
    int32_t *part;
    int64_t *B;
    int64_t *conn;
    uint8_t *marked;
    int32_t *marklist;
    int32_t nmark;
    int32_t *logv, *logf;
    heap_t h;
    int32_t max_idle;
    int32_t max_queue;  /* 0: unbounded; q > 0: a search queues at most q vertices */
} mls_ctx;

/*
 * One search from seed s on (part, B): queue s and its unmarked neighbours,
 * move the vertex of largest gain while the stopping rule allows, then
 * restore the best prefix. Returns its gain; logv/logf[0 .. *nbest) hold the
 * kept moves (vertex, block it left). Vertices it queued are appended to
 * marklist.
 */
static int64_t mls_search(mls_ctx *c, int32_t s, int32_t *nbest) {
    const orc_graph *g = c->g;
    heap_t *h = &c->h;
    int32_t *part = c->part;
    int64_t *B = c->B;
    int32_t queued = 0;  /* vertices this search marked (a vertex past the bound stays unmarked) */
    for (int32_t q = -1; q < g->xadj[s + 1] - g->xadj[s]; q++) {
        const int32_t u = q < 0 ? s : g->adjncy[g->xadj[s] + q];
        if (c->marked[u]) continue;
        if (c->max_queue > 0 && queued >= c->max_queue) break;
        queued++;
        c->marked[u] = 1;
        c->marklist[c->nmark++] = u;
        int32_t t;
        int ok;
        const int64_t gn = gain_of(g, part, B, c->k, c->lmax, u, c->conn, &t, &ok);
        if (ok) heap_push(h, gn, u);
    }
    int32_t nlog = 0, bestlen = 0, idle = 0;
    int64_t cum = 0, best = 0;
    while (h->size > 0) {
        const int32_t w = h->ver[0];
        const int64_t key = h->key[0];
        int32_t t;
        int ok;
        const int64_t gn = gain_of(g, part, B, c->k, c->lmax, w, c->conn, &t, &ok);
        if (!ok) {
            heap_remove(h, w);
            continue;
        }
        if (gn != key) {
            heap_update(h, w, gn);
            continue;
        }
        heap_remove(h, w);
        c->logv[nlog] = w;
        c->logf[nlog] = part[w];
        nlog++;
        B[part[w]] -= VW(g, w);
        B[t] += VW(g, w);
        part[w] = t;
        cum += gn;
        if (cum > best) {
            best = cum;
            bestlen = nlog;
            idle = 0;
        } else if (++idle >= c->max_idle) {
            break;
        }
        for (int32_t e = g->xadj[w]; e < g->xadj[w + 1]; e++) {
            const int32_t u = g->adjncy[e];
            if (h->pos[u] >= 0) {
                int32_t tu;
                int oku;
                const int64_t gu = gain_of(g, part, B, c->k, c->lmax, u, c->conn, &tu, &oku);
                if (oku) heap_update(h, u, gu);
                else heap_remove(h, u);
            } else if (!c->marked[u] && (c->max_queue <= 0 || queued < c->max_queue)) {
                queued++;
                c->marked[u] = 1;
                c->marklist[c->nmark++] = u;
                int32_t tu;
                int oku;
                const int64_t gu = gain_of(g, part, B, c->k, c->lmax, u, c->conn, &tu, &oku);
                if (oku) heap_push(h, gu, u);
            }
        }
    }
    while (h->size > 0) heap_remove(h, h->ver[0]);
    for (int32_t i = nlog - 1; i >= bestlen; i--) {
        const int32_t w = c->logv[i];
        B[part[w]] -= VW(g, w);
        B[c->logf[i]] += VW(g, w);
        part[w] = c->logf[i];
    }
    *nbest = bestlen;
    return best;
}

/* growable int32 array */
typedef struct {
    int32_t *a;
    int64_t len, cap;
} vec32;
static void vpush(vec32 *v, int32_t x) {
    if (v->len == v->cap) {
        v->cap = v->cap ? 2 * v->cap : 1024;
        v->a = (int32_t *)realloc(v->a, sizeof(int32_t) * (size_t)v->cap);
        if (!v->a) abort();
    }
    v->a[v->len++] = x;
}

int64_t orc_mls_batched(const orc_graph *g, int32_t k, int64_t lmax, int32_t *part, uint64_t seed,
                        int32_t global_iters, double alpha, int32_t max_idle, int32_t batch, int32_t max_queue,
                        orc_mls_stats *st) {
    const int32_t n = g->n;
    mls_ctx c;
    c.g = g;
    c.k = k;
    c.lmax = lmax;
    c.part = part;
    c.B = (int64_t *)xcalloc((size_t)k, sizeof(int64_t));
    for (int32_t v = 0; v < n; v++) c.B[part[v]] += VW(g, v);
    c.conn = (int64_t *)xcalloc((size_t)k, sizeof(int64_t));
    c.marked = (uint8_t *)xcalloc((size_t)n, 1);
    c.marklist = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    c.nmark = 0;
    c.logv = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    c.logf = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    c.h.key = (int64_t *)xcalloc((size_t)n, sizeof(int64_t));
    c.h.ver = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    c.h.pos = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    c.h.size = 0;
    c.max_idle = max_idle;
    c.max_queue = max_queue;
    for (int32_t v = 0; v < n; v++) c.h.pos[v] = -1;
    int64_t *B = c.B;
    int32_t *todo = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    int32_t *next = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    int32_t *seeds = (int32_t *)xcalloc((size_t)(batch > 0 ? batch : 1), sizeof(int32_t));
    int64_t *mstart = (int64_t *)xcalloc((size_t)(batch > 0 ? batch : 1) + 1, sizeof(int64_t));
    vec32 bmarks = {0}, mv_v = {0}, mv_f = {0}, mv_t = {0}, claims = {0};
    uint8_t *claimed = (uint8_t *)xcalloc((size_t)n, 1);
    int64_t total = 0, searches = 0, kept_moves = 0, local_iters = 0;

    for (int32_t gi = 0; gi < global_iters; gi++) {
        int32_t ntodo = 0;
        for (int32_t v = 0; v < n; v++) {
            int boundary = 0;
            for (int32_t e = g->xadj[v]; e < g->xadj[v + 1] && !boundary; e++) boundary = part[g->adjncy[e]] != part[v];
            if (boundary) todo[ntodo++] = v;
        }
        hash_order(todo, ntodo, seed, gi, 0);
        int64_t gtotal = 0;
        for (int32_t li = 0;; li++) {
            local_iters++;
            int32_t nnext = 0;
            int64_t lgain = 0;
            c.nmark = 0;
            if (batch <= 0) {
                /* sequential: every search sees the moves and marks of the ones before */
                for (int32_t ti = 0; ti < ntodo; ti++) {
                    const int32_t s = todo[ti];
                    if (c.marked[s]) continue;
                    searches++;
                    int32_t bl;
                    const int64_t best = mls_search(&c, s, &bl);
                    for (int32_t i = 0; i < bl; i++) next[nnext++] = c.logv[i];
                    lgain += best;
                    kept_moves += bl;
                }
            } else {
                /* batches of `batch` searches from the same state and marks; their
                   kept prefixes are then applied in seed order with recomputed gains */
                int32_t ti = 0;
                while (ti < ntodo) {
                    int32_t ns = 0;
                    while (ti < ntodo && ns < batch) {
                        const int32_t s = todo[ti];
                        if (c.marked[s]) {
                            ti++;
                            continue;
                        }
                        /* the batch ends at the first seed whose closed neighbourhood
                           meets one already taken (it starts the next batch) */
                        int clash = claimed[s];
                        for (int32_t e = g->xadj[s]; e < g->xadj[s + 1] && !clash; e++) clash = claimed[g->adjncy[e]];
                        if (clash && ns > 0) break;
                        claimed[s] = 1;
                        vpush(&claims, s);
                        for (int32_t e = g->xadj[s]; e < g->xadj[s + 1]; e++) {
                            if (!claimed[g->adjncy[e]]) {
                                claimed[g->adjncy[e]] = 1;
                                vpush(&claims, g->adjncy[e]);
                            }
                        }
                        seeds[ns++] = s;
                        ti++;
                    }
                    for (int64_t i = 0; i < claims.len; i++) claimed[claims.a[i]] = 0;
                    claims.len = 0;
                    if (ns == 0) break;
                    bmarks.len = mv_v.len = mv_f.len = mv_t.len = 0;
                    for (int32_t j = 0; j < ns; j++) {
                        searches++;
                        const int32_t mark0 = c.nmark;
                        int32_t bl;
                        (void)mls_search(&c, seeds[j], &bl);
                        mstart[j] = mv_v.len;
                        for (int32_t i = 0; i < bl; i++) {
                            vpush(&mv_v, c.logv[i]);
                            vpush(&mv_f, c.logf[i]);
                            vpush(&mv_t, part[c.logv[i]]);
                        }
                        /* back to the batch's state, and its marks kept aside */
                        for (int32_t i = bl - 1; i >= 0; i--) {
                            const int32_t w = c.logv[i];
                            B[part[w]] -= VW(g, w);
                            B[c.logf[i]] += VW(g, w);
                            part[w] = c.logf[i];
                        }
                        for (int32_t i = mark0; i < c.nmark; i++) {
                            c.marked[c.marklist[i]] = 0;
                            vpush(&bmarks, c.marklist[i]);
                        }
                        c.nmark = mark0;
                    }
                    mstart[ns] = mv_v.len;
                    for (int64_t i = 0; i < bmarks.len; i++) {
                        const int32_t u = bmarks.a[i];
                        if (!c.marked[u]) {
                            c.marked[u] = 1;
                            c.marklist[c.nmark++] = u;
                        }
                    }
                    for (int32_t j = 0; j < ns; j++) {
                        int64_t cum = 0, best = 0;
                        int32_t na = 0, bestlen = 0;
                        for (int64_t m = mstart[j]; m < mstart[j + 1]; m++) {
                            const int32_t v = mv_v.a[m], f = mv_f.a[m], t = mv_t.a[m];
                            if (part[v] != f || B[t] + VW(g, v) > lmax) break;
                            int64_t ct = 0, cf = 0;
                            for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
                                const int32_t pu = part[g->adjncy[e]];
                                if (pu == t) ct += EW(g, e);
                                else if (pu == f) cf += EW(g, e);
                            }
                            B[f] -= VW(g, v);
                            B[t] += VW(g, v);
                            part[v] = t;
                            na++;
                            cum += ct - cf;
                            if (cum > best) {
                                best = cum;
                                bestlen = na;
                            }
                        }
                        for (int32_t i = na - 1; i >= bestlen; i--) {
                            const int64_t m = mstart[j] + i;
                            const int32_t v = mv_v.a[m];
                            B[part[v]] -= VW(g, v);
                            B[mv_f.a[m]] += VW(g, v);
                            part[v] = mv_f.a[m];
                        }
                        for (int32_t i = 0; i < bestlen; i++) next[nnext++] = mv_v.a[mstart[j] + i];
                        lgain += best;
                        kept_moves += bestlen;
                    }
                }
            }
            for (int32_t i = 0; i < c.nmark; i++) c.marked[c.marklist[i]] = 0;
            total += lgain;
            /* another local iteration around the moved vertices while it pays */
            if (lgain > 0 && (double)lgain > alpha * (double)gtotal) {
                gtotal += lgain;
                memcpy(todo, next, sizeof(int32_t) * (size_t)nnext);
                ntodo = nnext;
                hash_order(todo, ntodo, seed, gi, li + 1);
                if (ntodo == 0) break;
            } else {
                break;
            }
        }
    }
    if (st) {
        st->gain = total;
        st->searches = searches;
        st->moves = kept_moves;
        st->local_iters = local_iters;
    }
    free(c.B);
    free(c.conn);
    free(c.marked);
    free(c.marklist);
    free(c.logv);
    free(c.logf);
    free(c.h.key);
    free(c.h.ver);
    free(c.h.pos);
    free(todo);
    free(next);
    free(seeds);
    free(mstart);
    free(bmarks.a);
    free(mv_v.a);
    free(mv_f.a);
    free(mv_t.a);
    free(claims.a);
    free(claimed);
    return total;
}

int64_t orc_mls(const orc_graph *g, int32_t k, int64_t lmax, int32_t *part, uint64_t seed, int32_t global_iters,
                double alpha, int32_t max_idle, orc_mls_stats *st) {
    return orc_mls_batched(g, k, lmax, part, seed, global_iters, alpha, max_idle, 0, 0, st);
}
