/*
 * oracle.c — plain CPU oracle (test infrastructure; see oracle.h).
 *
 * Paper: Akhremtsev, Sanders, Schulz, "High-Quality Shared-Memory Graph
 * Partitioning" (arXiv 1710.08231). Sections cited: §II-A (problem statement,
 * L_max, cut, size-constrained clustering, quotient graph), §III-A
 * (coarsening, contraction, size-constrained label propagation), §III-B
 * (initial partitioning by recursive bisection, best of I tries), §III-C
 * (projection, LP as local search with U = L_max), §IV-A (parallel LP: a move
 * is made only if the target is still feasible; parallel contraction by
 * prefix-sum relabelling), §VI (10 / 25 LP iterations, 4 initial tries).
 *
 * The LP here is the round-synchronous reading of §III-A/§IV-A: every vertex
 * proposes from the labels and label weights of the round start, ties go to
 * the lowest label, and the moves to one target are admitted in ascending
 * vertex order while the running weight stays within U. Even rounds only
 * allow moves to smaller labels and odd rounds only to larger ones
 * ("direction alternation"), which rules out the two-cycles a synchronous
 * round would otherwise fall into.
 *
 * Everything is written as the plain definition: dense scratch arrays,
 * explicit loops, no blocking or fusion.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define VW(g, v) ((g)->vwgt ? (int64_t)(g)->vwgt[v] : (int64_t)1)
#define EW(g, e) ((g)->adjwgt ? (int64_t)(g)->adjwgt[e] : (int64_t)1)

static void *xcalloc(size_t count, size_t size) {
    void *p = calloc(count ? count : 1, size);
    if (!p) abort();
    return p;
}

/* §II-A: L_max = (1+eps) * ceil(c(V)/k), read as the floor of the binary64 product. */
int64_t orc_lmax(int64_t total_vwgt, int32_t k, double eps) {
    int64_t q = total_vwgt / k + (total_vwgt % k != 0);
    return (int64_t)floor((1.0 + eps) * (double)q);
}

int64_t orc_total_vwgt(const orc_graph *g) {
    int64_t s = 0;
    for (int32_t v = 0; v < g->n; v++) s += VW(g, v);
    return s;
}

/*
 * One synchronous LP round (§III-A clustering rule, §IV-A admission).
 *   1. conn[L] = total weight of v's edges to vertices labelled L.
 *   2. candidates: L != C[v], allowed by the direction of round r, and
 *      eligible, i.e. W[L] + c(v) <= U (a cluster is overloaded only when it
 *      exceeds its bound).
 *   3. best = max conn, ties -> smallest L; propose iff conn[best] > conn[C[v]].
 *   4. admission per target in ascending v: admitted iff W[t] + (sum of c over
 *      the proposers to t up to and including v) <= U.
 *   5. apply all admitted moves; W follows.
 */
/*
 * Active-set rounds (the paper's Q/Q' of §III-A and §IV-A, made synchronous):
 * act[v] counts the evaluations v still owes. A vertex with act[v] == 0 makes
 * no proposal and its edges are not visited. Every evaluated vertex owes one
 * evaluation less afterwards. A vertex whose proposal is refused by the
 * admission owes at least one more (it is blocked by capacity, not
 * settled). Every neighbour of an admitted mover owes `renew` evaluations:
 * 2 with direction alternation (one per direction, since a round sees only
 * one direction), else 1. All vertices start owing `renew`.
 */
/* Proposal of vertex v (steps 1-3) from the labels C and weights W of the
 * round start: the best eligible label, or -1 to stay. conn, seen and touched
 * are scratch arrays of nlabels entries, all zero on entry and on return. */
static int32_t propose_vertex(const orc_graph *g, const int32_t *C, const int64_t *W, int64_t U, int32_t r,
                              int32_t dir_alternate, int32_t v, int64_t *conn, int32_t *seen, int32_t *touched) {
    int32_t ntouched = 0;
    for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
        int32_t L = C[g->adjncy[e]];
        if (!seen[L]) { seen[L] = 1; touched[ntouched++] = L; }
        conn[L] += EW(g, e);
    }
    int32_t own = C[v];
    int64_t conn_own = seen[own] ? conn[own] : 0;
    int32_t best = -1;
    int64_t best_conn = 0;
    for (int32_t i = 0; i < ntouched; i++) {
        int32_t L = touched[i];
        if (L == own) continue;
        if (dir_alternate) {
            if ((r % 2) == 0 && !(L < own)) continue;
            if ((r % 2) == 1 && !(L > own)) continue;
        }
        if (W[L] + VW(g, v) > U) continue;
        if (best < 0 || conn[L] > best_conn || (conn[L] == best_conn && L < best)) {
            best = L;
            best_conn = conn[L];
        }
    }
    for (int32_t i = 0; i < ntouched; i++) { conn[touched[i]] = 0; seen[touched[i]] = 0; }
    return (best >= 0 && best_conn > conn_own) ? best : -1;
}

/* Threads of the proposal loop of full rounds and of a colour class (1 unless
 * orc_set_threads says otherwise). Every proposal reads only the labels and
 * weights as they stand before the loop and writes only its own entry, so the
 * result does not depend on the thread count. */
static int orc_threads = 1;

void orc_set_threads(int32_t t) { orc_threads = t > 0 ? t : 1; }

static int64_t lp_round_act(const orc_graph *g, int32_t *C, int64_t *W, int32_t nlabels, int64_t U,
                            int32_t r, int32_t dir_alternate, int32_t *prop_out, uint8_t *act, int64_t *visits) {
    int32_t n = g->n;
    int64_t *conn = (int64_t *)xcalloc((size_t)nlabels, sizeof(int64_t));
    int32_t *prop = prop_out ? prop_out : (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    const uint8_t renew = dir_alternate ? 2 : 1;

    if (act || orc_threads <= 1) {
        int32_t *seen = (int32_t *)xcalloc((size_t)nlabels, sizeof(int32_t));
        int32_t *touched = (int32_t *)xcalloc((size_t)nlabels, sizeof(int32_t));
        for (int32_t v = 0; v < n; v++) {
            if (act && act[v] == 0) {
                prop[v] = -1;
                continue;
            }
            if (act) act[v]--;
            if (visits) *visits += g->xadj[v + 1] - g->xadj[v];
            prop[v] = propose_vertex(g, C, W, U, r, dir_alternate, v, conn, seen, touched);
        }
        free(seen);
        free(touched);
    } else {
        if (visits) *visits += g->xadj[n];
#pragma omp parallel num_threads(orc_threads)
        {
            int64_t *tconn = (int64_t *)xcalloc((size_t)nlabels, sizeof(int64_t));
            int32_t *tseen = (int32_t *)xcalloc((size_t)nlabels, sizeof(int32_t));
            int32_t *ttouched = (int32_t *)xcalloc((size_t)nlabels, sizeof(int32_t));
#pragma omp for schedule(dynamic, 1024)
            for (int32_t v = 0; v < n; v++)
                prop[v] = propose_vertex(g, C, W, U, r, dir_alternate, v, tconn, tseen, ttouched);
            free(tconn);
            free(tseen);
            free(ttouched);
        }
    }

    /* admission: running proposal weight per target, vertices in ascending order */
    int64_t *acc = conn; /* all zero again */
    uint8_t *admitted = (uint8_t *)xcalloc((size_t)n, 1);
    for (int32_t v = 0; v < n; v++) {
        if (prop[v] < 0) continue;
        int32_t t = prop[v];
        acc[t] += VW(g, v);
        admitted[v] = (W[t] + acc[t] <= U);
        if (act && !admitted[v] && act[v] < 1) act[v] = 1;
    }
    int64_t moves = 0;
    for (int32_t v = 0; v < n; v++) {
        if (!admitted[v]) continue;
        int32_t t = prop[v];
        W[t] += VW(g, v);
        W[C[v]] -= VW(g, v);
        C[v] = t;
        moves++;
        if (act)
            for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) act[g->adjncy[e]] = renew;
    }
    free(admitted);
    free(conn);
    if (!prop_out) free(prop);
    return moves;
}

int64_t orc_lp_round(const orc_graph *g, int32_t *C, int64_t *W, int32_t nlabels, int64_t U,
                     int32_t r, int32_t dir_alternate, int32_t *prop_out) {
    return lp_round_act(g, C, W, nlabels, U, r, dir_alternate, prop_out, NULL, NULL);
}

/* Round loop shared by clustering and refinement; stop after two idle rounds
 * in a row. flags: ORC_LP_DIR_ALTERNATE, ORC_LP_ACTIVE_SET. */
static void lp_rounds(const orc_graph *g, int32_t *C, int64_t *W, int32_t nlabels, int64_t U,
                      int32_t rounds, int32_t flags, orc_lp_stats *st) {
    const int32_t dirs = (flags & ORC_LP_DIR_ALTERNATE) != 0;
    uint8_t *act = NULL;
    if (flags & ORC_LP_ACTIVE_SET) {
        act = (uint8_t *)xcalloc((size_t)g->n + 1, 1);
        memset(act, dirs ? 2 : 1, (size_t)g->n);
    }
    int64_t prev = -1, total = 0, visits = 0;
    int32_t run = 0;
    for (int32_t r = 0; r < rounds; r++) {
        int64_t m = lp_round_act(g, C, W, nlabels, U, r, dirs, NULL, act, &visits);
        total += m;
        run = r + 1;
        if (r >= 1 && m == 0 && prev == 0) break;
        prev = m;
    }
    free(act);
    if (st) {
        st->rounds_run = run;
        st->moves = total;
        st->edge_visits = visits;
    }
}

/*
 * Colour-class LP (oracle-only comparison mode; lp_async = 2 in orc_params for
 * clustering and refinement, 3 for clustering only).
 * A schedule between the synchronous rounds and the paper's sequential queue
 * (§III-A) that keeps the parallelism a GPU needs: vertices are split into
 * classes of pairwise non-adjacent vertices, and a round visits the classes
 * one after the other.
 *  - Colouring: in decreasing order of the priority sm64(v) (ties: larger id
 *    first), each vertex takes the smallest colour that no already coloured
 *    neighbour holds (first fit). The same colouring comes out of the
 *    parallel rule "colour v once all neighbours of higher priority are
 *    coloured" (Jones and Plassmann 1993).
 *  - Round: for each colour in increasing order, every vertex of the class
 *    proposes from the current labels and weights (steps 1-3; no direction
 *    rule, since no two proposers of a class are adjacent), the proposals are
 *    admitted per target in ascending id (step 4), and applied (step 5)
 *    before the next class proposes. Stop after two idle rounds in a row.
 */
typedef struct {
    uint64_t p;
    int32_t v;
} prio_t;

static int cmp_prio_desc(const void *a, const void *b) {
    const prio_t *x = (const prio_t *)a, *y = (const prio_t *)b;
    if (x->p != y->p) return x->p < y->p ? 1 : -1;
    return (x->v < y->v) - (x->v > y->v);
}

static uint64_t sm64(uint64_t x);

int32_t orc_colour_classes(const orc_graph *g, int32_t *colour) {
    const int32_t n = g->n;
    if (n == 0) return 0;
    prio_t *order = (prio_t *)xcalloc((size_t)n, sizeof(prio_t));
    int32_t dmax = 0;
    for (int32_t v = 0; v < n; v++) {
        order[v].p = sm64((uint64_t)v);
        order[v].v = v;
        colour[v] = -1;
        if (g->xadj[v + 1] - g->xadj[v] > dmax) dmax = g->xadj[v + 1] - g->xadj[v];
    }
    qsort(order, (size_t)n, sizeof(prio_t), cmp_prio_desc);
    int32_t *stamp = (int32_t *)xcalloc((size_t)dmax + 2, sizeof(int32_t));
    int32_t ncol = 0;
    for (int32_t i = 0; i < n; i++) {
        const int32_t v = order[i].v;
        for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
            const int32_t c = colour[g->adjncy[e]];
            if (c >= 0 && c <= dmax) stamp[c] = i + 1;
        }
        int32_t c = 0;
        while (stamp[c] == i + 1) c++;
        colour[v] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    free(stamp);
    free(order);
    return ncol;
}

static void lp_colour(const orc_graph *g, int32_t *C, int64_t *W, int32_t nlabels, int64_t U, int32_t rounds,
                      orc_lp_stats *st) {
    const int32_t n = g->n;
    int32_t *colour = (int32_t *)xcalloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    const int32_t ncol = orc_colour_classes(g, colour);
    /* classes in ascending id: counting sort by colour */
    int32_t *start = (int32_t *)xcalloc((size_t)ncol + 2, sizeof(int32_t));
    int32_t *cls = (int32_t *)xcalloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    for (int32_t v = 0; v < n; v++) start[colour[v] + 1]++;
    for (int32_t c = 0; c < ncol; c++) start[c + 1] += start[c];
    for (int32_t v = 0; v < n; v++) cls[start[colour[v]]++] = v;
    for (int32_t c = ncol; c > 0; c--) start[c] = start[c - 1];
    start[0] = 0;
    int64_t *conn = (int64_t *)xcalloc((size_t)nlabels, sizeof(int64_t));
    int32_t *seen = (int32_t *)xcalloc((size_t)nlabels, sizeof(int32_t));
    int32_t *touched = (int32_t *)xcalloc((size_t)nlabels, sizeof(int32_t));
    int64_t *acc = (int64_t *)xcalloc((size_t)nlabels, sizeof(int64_t));
    int32_t *prop = (int32_t *)xcalloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    uint8_t *admitted = (uint8_t *)xcalloc((size_t)(n > 0 ? n : 1), 1);
    /* per-thread proposal scratch (all zero between proposals), allocated once */
    const int nthr = orc_threads;
    int64_t **tconn = NULL;
    int32_t **tseen = NULL, **ttouched = NULL;
    if (nthr > 1) {
        tconn = (int64_t **)xcalloc((size_t)nthr, sizeof(int64_t *));
        tseen = (int32_t **)xcalloc((size_t)nthr, sizeof(int32_t *));
        ttouched = (int32_t **)xcalloc((size_t)nthr, sizeof(int32_t *));
        for (int t = 0; t < nthr; t++) {
            tconn[t] = (int64_t *)xcalloc((size_t)nlabels, sizeof(int64_t));
            tseen[t] = (int32_t *)xcalloc((size_t)nlabels, sizeof(int32_t));
            ttouched[t] = (int32_t *)xcalloc((size_t)nlabels, sizeof(int32_t));
        }
    }
    int64_t prev = -1, total = 0, visits = 0;
    int32_t run = 0;
    for (int32_t r = 0; r < rounds; r++) {
        int64_t m = 0;
        for (int32_t c = 0; c < ncol; c++) {
            const int32_t b = start[c], e = start[c + 1];
            for (int32_t j = b; j < e; j++) visits += g->xadj[cls[j] + 1] - g->xadj[cls[j]];
            if (nthr > 1 && e - b >= 4096) {
                /* proposals of one class read C and W and write only their own entry */
#pragma omp parallel num_threads(nthr)
                {
                    const int t = omp_get_thread_num();
#pragma omp for schedule(dynamic, 1024)
                    for (int32_t j = b; j < e; j++)
                        prop[j] = propose_vertex(g, C, W, U, r, 0, cls[j], tconn[t], tseen[t], ttouched[t]);
                }
            } else {
                for (int32_t j = b; j < e; j++) prop[j] = propose_vertex(g, C, W, U, r, 0, cls[j], conn, seen, touched);
            }
            for (int32_t j = b; j < e; j++) {
                if (prop[j] < 0) continue;
                acc[prop[j]] += VW(g, cls[j]);
                admitted[j] = (W[prop[j]] + acc[prop[j]] <= U);
            }
            for (int32_t j = b; j < e; j++) {
                if (prop[j] < 0) continue;
                acc[prop[j]] = 0;
                if (!admitted[j]) continue;
                const int32_t v = cls[j], t = prop[j];
                W[t] += VW(g, v);
                W[C[v]] -= VW(g, v);
                C[v] = t;
                admitted[j] = 0;
                m++;
            }
        }
        total += m;
        run = r + 1;
        if (r >= 1 && m == 0 && prev == 0) break;
        prev = m;
    }
    if (st) {
        st->rounds_run = run;
        st->moves = total;
        st->edge_visits = visits;
    }
    for (int t = 0; t < nthr && tconn; t++) {
        free(tconn[t]);
        free(tseen[t]);
        free(ttouched[t]);
    }
    free(tconn);
    free(tseen);
    free(ttouched);
    free(colour);
    free(start);
    free(cls);
    free(conn);
    free(seen);
    free(touched);
    free(acc);
    free(prop);
    free(admitted);
}

int orc_lp_cluster_colour(const orc_graph *g, int64_t U, int32_t rounds, int32_t *labels_out, orc_lp_stats *st) {
    int32_t n = g->n;
    int64_t *W = (int64_t *)xcalloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    for (int32_t v = 0; v < n; v++) { labels_out[v] = v; W[v] = VW(g, v); }
    lp_colour(g, labels_out, W, n > 0 ? n : 1, U, rounds, st);
    free(W);
    return 0;
}

int orc_lp_refine_colour(const orc_graph *g, int32_t k, int64_t lmax, int32_t rounds, int32_t *part,
                         orc_lp_stats *st) {
    int64_t *W = (int64_t *)xcalloc((size_t)k, sizeof(int64_t));
    for (int32_t v = 0; v < g->n; v++) W[part[v]] += VW(g, v);
    lp_colour(g, part, W, k, lmax, rounds, st);
    free(W);
    return 0;
}

/* §III-A: size-constrained LP clustering from singletons, C[v] = v, bound U. */
int orc_lp_cluster(const orc_graph *g, int64_t U, int32_t rounds, int32_t flags,
                   int32_t *labels_out, orc_lp_stats *st) {
    int32_t n = g->n;
    int64_t *W = (int64_t *)xcalloc((size_t)n, sizeof(int64_t));
    for (int32_t v = 0; v < n; v++) { labels_out[v] = v; W[v] = VW(g, v); }
    lp_rounds(g, labels_out, W, n, U, rounds, flags, st);
    free(W);
    return 0;
}

/* §III-C: LP as local search from a k-way partition with U = L_max. */
int orc_lp_refine(const orc_graph *g, int32_t k, int64_t lmax, int32_t rounds,
                  int32_t flags, int32_t *part, orc_lp_stats *st) {
    int64_t *W = (int64_t *)xcalloc((size_t)k, sizeof(int64_t));
    for (int32_t v = 0; v < g->n; v++) W[part[v]] += VW(g, v);
    lp_rounds(g, part, W, k, lmax, rounds, flags, st);
    free(W);
    return 0;
}

/*
 * §III-A sequential size-constrained LP in the paper's own form (oracle-only,
 * to measure what the round-synchronous reading costs in quality):
 *  - all vertices start in queue Q in increasing order of degree (ties: id);
 *  - visiting v moves it at once to the eligible cluster (W[L] + c(v) <= U)
 *    with the strongest connection; its own cluster competes and wins ties,
 *    other ties go to the smallest label (the paper leaves ties open);
 *  - when v changes cluster, every neighbour not yet queued for the next
 *    iteration is appended to Q' (in the order they are met);
 *  - Q and Q' swap after each iteration; stop after `rounds` iterations or
 *    when Q is empty.
 * C and W are updated in place.
 */
static void lp_async(const orc_graph *g, int32_t *C, int64_t *W, int32_t nlabels, int64_t U, int32_t rounds,
                     orc_lp_stats *st) {
    int32_t n = g->n;
    int32_t *Q = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    int32_t *Q2 = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    uint8_t *queued = (uint8_t *)xcalloc((size_t)n, 1);
    int64_t *conn = (int64_t *)xcalloc((size_t)nlabels, sizeof(int64_t));
    int32_t *touched = (int32_t *)xcalloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    /* counting sort by degree keeps ascending ids inside a degree */
    int32_t dmax = 0;
    for (int32_t v = 0; v < n; v++) if (g->xadj[v + 1] - g->xadj[v] > dmax) dmax = g->xadj[v + 1] - g->xadj[v];
    int32_t *cnt = (int32_t *)xcalloc((size_t)dmax + 2, sizeof(int32_t));
    for (int32_t v = 0; v < n; v++) cnt[g->xadj[v + 1] - g->xadj[v] + 1]++;
    for (int32_t d = 0; d <= dmax; d++) cnt[d + 1] += cnt[d];
    for (int32_t v = 0; v < n; v++) Q[cnt[g->xadj[v + 1] - g->xadj[v]]++] = v;
    free(cnt);
    int32_t qn = n, it = 0;
    int64_t moves = 0, visits = 0;
    for (; it < rounds && qn > 0; it++) {
        int32_t q2n = 0;
        for (int32_t qi = 0; qi < qn; qi++) {
            const int32_t v = Q[qi];
            if (C[v] < 0) continue; /* takes no part */
            const int32_t own = C[v];
            const int64_t cv = VW(g, v);
            int32_t nt = 0;
            for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
                const int32_t L = C[g->adjncy[e]];
                if (L < 0) continue;
                if (conn[L] == 0) touched[nt++] = L;
                conn[L] += EW(g, e);
            }
            visits += g->xadj[v + 1] - g->xadj[v];
            int32_t best = own;
            int64_t bc = conn[own];
            for (int32_t i = 0; i < nt; i++) {
                const int32_t L = touched[i];
                if (L == own || W[L] + cv > U) continue;
                if (conn[L] > bc || (conn[L] == bc && best != own && L < best)) {
                    best = L;
                    bc = conn[L];
                }
            }
            for (int32_t i = 0; i < nt; i++) conn[touched[i]] = 0;
            if (best != own) {
                C[v] = best;
                W[own] -= cv;
                W[best] += cv;
                moves++;
                for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
                    const int32_t u = g->adjncy[e];
                    if (!queued[u]) {
                        queued[u] = 1;
                        Q2[q2n++] = u;
                    }
                }
            }
        }
        for (int32_t i = 0; i < q2n; i++) queued[Q2[i]] = 0;
        int32_t *t = Q;
        Q = Q2;
        Q2 = t;
        qn = q2n;
    }
    if (st) {
        st->rounds_run = it;
        st->moves = moves;
        st->edge_visits = visits;
    }
    free(Q);
    free(Q2);
    free(queued);
    free(conn);
    free(touched);
}

int orc_lp_cluster_async(const orc_graph *g, int64_t U, int32_t rounds, int32_t *labels_out, orc_lp_stats *st) {
    int32_t n = g->n;
    int64_t *W = (int64_t *)xcalloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    for (int32_t v = 0; v < n; v++) { labels_out[v] = v; W[v] = VW(g, v); }
    lp_async(g, labels_out, W, n, U, rounds, st);
    free(W);
    return 0;
}

int orc_lp_refine_async(const orc_graph *g, int32_t k, int64_t lmax, int32_t rounds, int32_t *part,
                        orc_lp_stats *st) {
    int64_t *W = (int64_t *)xcalloc((size_t)k, sizeof(int64_t));
    for (int32_t v = 0; v < g->n; v++) if (part[v] >= 0) W[part[v]] += VW(g, v);
    lp_async(g, part, W, k, lmax, rounds, st);
    free(W);
    return 0;
}

static int cmp_i32(const void *a, const void *b) {
    const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * §III-A / §IV-A contraction. Coarse ids: prefix sum over "label is used"
 * indicators, so coarse id = rank of the label among the used labels.
 * c'(i) = sum of c over cluster i; w'(i,j) = sum of w over fine edges between
 * clusters i != j. Rows ascending by i, columns ascending by j.
 */
int orc_contract(const orc_graph *g, const int32_t *labels, int32_t *xadj_c, int32_t *adjncy_c,
                 int32_t *adjwgt_c, int32_t *vwgt_c, int32_t *f2c, int32_t *n_c_out,
                 int32_t *nnz_c_out) {
    int32_t n = g->n;
    int32_t *used = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    int32_t *id = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    for (int32_t v = 0; v < n; v++) used[labels[v]] = 1;
    int32_t nc = 0;
    for (int32_t L = 0; L < n; L++) { id[L] = nc; nc += used[L]; }
    for (int32_t v = 0; v < n; v++) f2c[v] = id[labels[v]];

    /* members of each coarse vertex, ascending fine id */
    int32_t *mstart = (int32_t *)xcalloc((size_t)nc + 1, sizeof(int32_t));
    int32_t *members = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    for (int32_t v = 0; v < n; v++) mstart[f2c[v] + 1]++;
    for (int32_t i = 0; i < nc; i++) mstart[i + 1] += mstart[i];
    int32_t *fill = (int32_t *)xcalloc((size_t)nc + 1, sizeof(int32_t));
    memcpy(fill, mstart, sizeof(int32_t) * (size_t)nc);
    for (int32_t v = 0; v < n; v++) members[fill[f2c[v]]++] = v;
    free(fill);

    int64_t *acc = (int64_t *)xcalloc((size_t)nc, sizeof(int64_t));
    int32_t *seen = (int32_t *)xcalloc((size_t)nc, sizeof(int32_t));
    int32_t *cols = (int32_t *)xcalloc((size_t)nc, sizeof(int32_t));
    int64_t nnz = 0;
    xadj_c[0] = 0;
    for (int32_t i = 0; i < nc; i++) {
        int64_t cw = 0;
        int32_t ncols = 0;
        for (int32_t m = mstart[i]; m < mstart[i + 1]; m++) {
            int32_t v = members[m];
            cw += VW(g, v);
            for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
                int32_t j = f2c[g->adjncy[e]];
                if (j == i) continue;
                if (!seen[j]) { seen[j] = 1; cols[ncols++] = j; }
                acc[j] += EW(g, e);
            }
        }
        /* ascending columns */
        qsort(cols, (size_t)ncols, sizeof(int32_t), cmp_i32);
        for (int32_t a = 0; a < ncols; a++) {
            int32_t j = cols[a];
            adjncy_c[nnz] = j;
            adjwgt_c[nnz] = (int32_t)acc[j];
            nnz++;
            acc[j] = 0;
            seen[j] = 0;
        }
        xadj_c[i + 1] = (int32_t)nnz;
        vwgt_c[i] = (int32_t)cw;
    }
    *n_c_out = nc;
    *nnz_c_out = (int32_t)nnz;
    free(used); free(id); free(mstart); free(members); free(acc); free(seen); free(cols);
    return 0;
}

/* §III-C: a fine vertex takes the block of its coarse representative. */
void orc_project(int32_t n, const int32_t *f2c, const int32_t *part_coarse, int32_t *part_fine) {
    for (int32_t v = 0; v < n; v++) part_fine[v] = part_coarse[f2c[v]];
}

/* §II-A: cut = weight of edges between different blocks, each undirected edge once. */
int64_t orc_cut(const orc_graph *g, const int32_t *part) {
    int64_t s = 0;
    for (int32_t v = 0; v < g->n; v++)
        for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++)
            if (part[v] != part[g->adjncy[e]]) s += EW(g, e);
    return s / 2;
}

void orc_block_weights(const orc_graph *g, const int32_t *part, int32_t k, int64_t *B) {
    for (int32_t b = 0; b < k; b++) B[b] = 0;
    for (int32_t v = 0; v < g->n; v++) B[part[v]] += VW(g, v);
}

/* splitmix64 finaliser applied to x + gamma (Steele, Lea & Flood 2014). */
static uint64_t sm64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Start-vertex hash of the initial bisection: chained splitmix64 over four words. */
uint64_t orc_mix4(uint64_t seed, uint64_t a, uint64_t base, uint64_t ks) {
    return sm64(sm64(sm64(sm64(seed) ^ a) ^ base) ^ ks);
}

/*
 * Recursive bisection (§III-B: split into ceil(k/2) and floor(k/2) blocks and
 * recurse). One bisection of the set S (ascending ids) with k_S blocks:
 * target = ceil(c(S) * k_L / k_S) with k_L = ceil(k_S/2). Grow the left side
 * by FIFO breadth-first search inside S from a hashed start vertex; vertices
 * are marked when enqueued, appended to the left side when dequeued, and the
 * search stops once the left side weighs at least `target`. When the queue
 * runs dry, the smallest unmarked vertex of S is enqueued.
 */
typedef struct {
    const orc_graph *g;
    uint64_t seed;
    int32_t attempt;
    int32_t *part;
    int32_t *inset;  /* inset[v] == set tag while v belongs to the current S */
    int32_t *marked;
    int32_t *queue;
    int32_t tag;
    int64_t lmax;      /* block bound; a side that will hold j blocks may weigh j * lmax */
    int32_t fm_passes; /* 0: no local search after a bisection */
    int32_t *side;     /* 0 left, 1 right, for the vertices of the current S */
    int32_t *locked;
    int32_t *log;
    int64_t *gain;
} rb_ctx;

/*
 * 2-way FM local search after a bisection (§III-B: the bisection is improved
 * by local search; the paper's KaHIP uses Fiduccia-Mattheyses). Only edges
 * with both ends in S count. One pass: every vertex of S unlocked, gain(v) =
 * (weight of v's edges to the other side) - (weight to its own side); move the
 * unlocked vertex of largest gain whose move keeps the receiving side within
 * its bound (ties -> lowest id), lock it, update its neighbours' gains; stop
 * when no vertex may move or after ORC_FM_IDLE moves without a new best
 * running gain; keep the shortest prefix of moves with the best running gain
 * and undo the rest. Passes repeat until one gains nothing (at most
 * fm_passes).
 */
#define ORC_FM_IDLE 50

static void fm2(rb_ctx *cx, const int32_t *S, int32_t size, int32_t tag, int64_t U0, int64_t U1) {
    const orc_graph *g = cx->g;
    const int64_t U[2] = {U0, U1};
    int32_t *side = cx->side;
    for (int32_t pass = 0; pass < cx->fm_passes; pass++) {
        int64_t Wt[2] = {0, 0};
        for (int32_t i = 0; i < size; i++) {
            int32_t v = S[i];
            Wt[side[v]] += VW(g, v);
            cx->locked[v] = 0;
            int64_t gn = 0;
            for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
                int32_t u = g->adjncy[e];
                if (u == v || cx->inset[u] != tag) continue;
                gn += side[u] != side[v] ? EW(g, e) : -EW(g, e);
            }
            cx->gain[v] = gn;
        }
        int64_t run = 0, best = 0;
        int32_t len = 0, best_len = 0, idle = 0;
        for (;;) {
            int32_t bv = -1;
            for (int32_t i = 0; i < size; i++) {
                int32_t v = S[i];
                if (cx->locked[v] || Wt[1 - side[v]] + VW(g, v) > U[1 - side[v]]) continue;
                if (bv < 0 || cx->gain[v] > cx->gain[bv]) bv = v;
            }
            if (bv < 0) break;
            int32_t to = 1 - side[bv];
            Wt[side[bv]] -= VW(g, bv);
            Wt[to] += VW(g, bv);
            side[bv] = to;
            cx->locked[bv] = 1;
            run += cx->gain[bv];
            cx->log[len++] = bv;
            for (int32_t e = g->xadj[bv]; e < g->xadj[bv + 1]; e++) {
                int32_t u = g->adjncy[e];
                if (u == bv || cx->inset[u] != tag) continue;
                cx->gain[u] += side[u] == to ? -2 * EW(g, e) : 2 * EW(g, e);
            }
            if (run > best) {
                best = run;
                best_len = len;
                idle = 0;
            } else if (++idle >= ORC_FM_IDLE) {
                break;
            }
        }
        for (int32_t i = len - 1; i >= best_len; i--) side[cx->log[i]] ^= 1;
        if (best <= 0) break;
    }
}

static void rb(rb_ctx *cx, int32_t *S, int32_t size, int32_t ks, int32_t base) {
    const orc_graph *g = cx->g;
    if (size == 0) return;
    if (ks == 1) {
        for (int32_t i = 0; i < size; i++) cx->part[S[i]] = base;
        return;
    }
    int32_t kl = (ks + 1) / 2;
    int64_t cs = 0;
    for (int32_t i = 0; i < size; i++) cs += VW(g, S[i]);
    __int128 num = (__int128)cs * kl;
    int64_t target = (int64_t)((num + ks - 1) / ks);

    int32_t tag = ++cx->tag;
    for (int32_t i = 0; i < size; i++) { cx->inset[S[i]] = tag; cx->marked[S[i]] = 0; }
    uint64_t h = orc_mix4(cx->seed, (uint64_t)cx->attempt, (uint64_t)base, (uint64_t)ks);
    int32_t s = S[h % (uint64_t)size];

    int32_t *left = (int32_t *)xcalloc((size_t)size, sizeof(int32_t));
    int32_t nleft = 0, head = 0, tail = 0, scan = 0;
    int64_t cleft = 0;
    cx->marked[s] = 1;
    cx->queue[tail++] = s;
    for (;;) {
        if (head == tail) {
            while (scan < size && cx->marked[S[scan]]) scan++;
            if (scan == size) break; /* cannot happen: target <= c(S) */
            cx->marked[S[scan]] = 1;
            cx->queue[tail++] = S[scan];
        }
        int32_t v = cx->queue[head++];
        left[nleft++] = v;
        cleft += VW(g, v);
        if (cleft >= target) break;
        for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
            int32_t u = g->adjncy[e];
            if (cx->inset[u] == tag && !cx->marked[u]) {
                cx->marked[u] = 1;
                cx->queue[tail++] = u;
            }
        }
    }
    /* sides: the grown part is the left side; optional local search; both
       sides in ascending order */
    for (int32_t i = 0; i < size; i++) cx->side[S[i]] = 1;
    for (int32_t i = 0; i < nleft; i++) cx->side[left[i]] = 0;
    if (cx->fm_passes > 0) fm2(cx, S, size, tag, (int64_t)kl * cx->lmax, (int64_t)(ks - kl) * cx->lmax);
    int32_t *right = (int32_t *)xcalloc((size_t)size, sizeof(int32_t));
    int32_t nright = 0;
    nleft = 0;
    for (int32_t i = 0; i < size; i++) {
        if (cx->side[S[i]] == 0) left[nleft++] = S[i];
        else right[nright++] = S[i];
    }
    rb(cx, left, nleft, kl, base);
    rb(cx, right, nright, ks - kl, base + kl);
    free(left);
    free(right);
}

void orc_recursive_bisection(const orc_graph *g, int32_t k, uint64_t seed, int32_t attempt, int64_t lmax,
                             int32_t fm_passes, int32_t *part_out) {
    int32_t n = g->n;
    rb_ctx cx;
    cx.g = g;
    cx.seed = seed;
    cx.attempt = attempt;
    cx.part = part_out;
    cx.inset = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    cx.marked = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    cx.queue = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    cx.tag = 0;
    cx.lmax = lmax;
    cx.fm_passes = fm_passes;
    cx.side = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    cx.locked = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    cx.log = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    cx.gain = (int64_t *)xcalloc((size_t)n, sizeof(int64_t));
    int32_t *S = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    for (int32_t v = 0; v < n; v++) S[v] = v;
    rb(&cx, S, n, k, 0);
    free(S);
    free(cx.inset);
    free(cx.marked);
    free(cx.queue);
    free(cx.side);
    free(cx.locked);
    free(cx.log);
    free(cx.gain);
}

/*
 * Greedy rebalance (project-defined; the paper delegates this to KaHIP's
 * local search). While a block exceeds L_max, apply the single move (v, t)
 * with v in an overloaded block, t != P(v), B[t] + c(v) <= L_max, of maximum
 * gain conn(v,t) - conn(v,P(v)) (§II-A gain); ties -> lowest v, then lowest t.
 */
int orc_rebalance(const orc_graph *g, int32_t k, int64_t lmax, int32_t *part) {
    int64_t *B = (int64_t *)xcalloc((size_t)k, sizeof(int64_t));
    int64_t *conn = (int64_t *)xcalloc((size_t)k, sizeof(int64_t));
    orc_block_weights(g, part, k, B);
    int balanced = 0;
    for (;;) {
        int over = 0;
        for (int32_t b = 0; b < k; b++) over |= (B[b] > lmax);
        if (!over) { balanced = 1; break; }
        int32_t bv = -1, bt = -1;
        int64_t bgain = 0;
        for (int32_t v = 0; v < g->n; v++) {
            int32_t pv = part[v];
            if (B[pv] <= lmax) continue;
            for (int32_t b = 0; b < k; b++) conn[b] = 0;
            for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) conn[part[g->adjncy[e]]] += EW(g, e);
            for (int32_t t = 0; t < k; t++) {
                if (t == pv || B[t] + VW(g, v) > lmax) continue;
                int64_t gain = conn[t] - conn[pv];
                if (bv < 0 || gain > bgain) { bv = v; bt = t; bgain = gain; }
            }
        }
        if (bv < 0) break;
        B[part[bv]] -= VW(g, bv);
        B[bt] += VW(g, bv);
        part[bv] = bt;
    }
    free(B);
    free(conn);
    return balanced;
}

/* §III-B / §IV-B: best of `attempts` tries by (imbalanced, cut, attempt index). */
int orc_initial_partition(const orc_graph *g, int32_t k, int64_t lmax, uint64_t seed,
                          int32_t attempts, int32_t rounds_refine, int32_t dir_alternate, int32_t fm_passes,
                          int32_t *part_out) {
    int32_t n = g->n;
    int32_t *P = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    int best = -1, best_bal = 0;
    int64_t best_cut = 0;
    for (int32_t a = 0; a < attempts; a++) {
        orc_recursive_bisection(g, k, seed, a, lmax, fm_passes, P);
        orc_lp_refine(g, k, lmax, rounds_refine, dir_alternate, P, NULL);
        int bal = orc_rebalance(g, k, lmax, P);
        int64_t cut = orc_cut(g, P);
        int better = best < 0 || (bal && !best_bal) || (bal == best_bal && cut < best_cut);
        if (better) {
            best = a;
            best_bal = bal;
            best_cut = cut;
            memcpy(part_out, P, sizeof(int32_t) * (size_t)n);
        }
    }
    free(P);
    return best;
}

/* Isolated vertices (no neighbours), ascending id, each into the lightest block (ties -> lowest). */
void orc_fill_isolated(const orc_graph *g, int32_t k, int32_t *part, int64_t *B) {
    for (int32_t v = 0; v < g->n; v++) {
        if (g->xadj[v + 1] != g->xadj[v]) continue;
        int32_t b = 0;
        for (int32_t t = 1; t < k; t++)
            if (B[t] < B[b]) b = t;
        part[v] = b;
        B[b] += VW(g, v);
    }
}

typedef struct {
    orc_graph g;
    int32_t *xadj, *adjncy, *adjwgt, *vwgt, *f2c; /* f2c maps this level to the next */
} level_t;

typedef struct {
    level_t *lev;
    int32_t L; /* index of the coarsest level */
    int32_t *newid;
    int64_t lmax, ucl, ev_cluster;
} hierarchy_t;

/*
 * §III-A coarsening with the project's stop rules:
 *  - U_c = max(c_max, L_max - ceil(W/k)) during coarsening (the paper only
 *    names "a given upper bound U");
 *  - vertices without neighbours are set aside before coarsening (level 0 is
 *    the graph of the other vertices, renumbered in ascending order);
 *  - coarsen while n > coarsest_per_k * k; discard a level that did not
 *    shrink; stop after a level with stall_den * n' > stall_num * n.
 */
/* direction flag of the coarsening and uncoarsening rounds; active-set rounds
 * are added per phase (initial partitioning always runs full rounds) */
static int32_t lp_flags(const orc_params *p) {
    return p->dir_alternate ? ORC_LP_DIR_ALTERNATE : 0;
}

static void coarsen(const orc_graph *g, int32_t k, double eps, const orc_params *p, hierarchy_t *h) {
    int32_t n = g->n;
    int64_t W = orc_total_vwgt(g);
    int64_t lmax = orc_lmax(W, k, eps);
    int64_t cmax = 0;
    for (int32_t v = 0; v < n; v++) if (VW(g, v) > cmax) cmax = VW(g, v);
    int64_t ceil_wk = W / k + (W % k != 0);
    int64_t ucl = lmax - ceil_wk;
    if (ucl < cmax) ucl = cmax;

    int32_t *newid = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    int32_t n0 = 0;
    for (int32_t v = 0; v < n; v++) newid[v] = (g->xadj[v + 1] > g->xadj[v]) ? n0++ : -1;
    int32_t nnz = g->xadj[n];

    int32_t maxlev = 64; /* grows as needed: the number of levels is not bounded */
    level_t *lev = (level_t *)xcalloc((size_t)maxlev, sizeof(level_t));
    lev[0].xadj = (int32_t *)xcalloc((size_t)n0 + 1, sizeof(int32_t));
    lev[0].adjncy = (int32_t *)xcalloc((size_t)nnz, sizeof(int32_t));
    lev[0].adjwgt = (int32_t *)xcalloc((size_t)nnz, sizeof(int32_t));
    lev[0].vwgt = (int32_t *)xcalloc((size_t)n0, sizeof(int32_t));
    {
        int32_t pos = 0;
        for (int32_t v = 0; v < n; v++) {
            if (newid[v] < 0) continue;
            int32_t i = newid[v];
            lev[0].vwgt[i] = (int32_t)VW(g, v);
            for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
                lev[0].adjncy[pos] = newid[g->adjncy[e]];
                lev[0].adjwgt[pos] = (int32_t)EW(g, e);
                pos++;
            }
            lev[0].xadj[i + 1] = pos;
        }
    }
    lev[0].g = (orc_graph){n0, lev[0].xadj, lev[0].adjncy, lev[0].adjwgt, lev[0].vwgt};

    int64_t ev_cluster = 0;
    int32_t L = 0;
    while (lev[L].g.n > (int64_t)p->coarsest_per_k * k) {
        if (L + 1 == maxlev) {
            lev = (level_t *)realloc(lev, sizeof(level_t) * (size_t)maxlev * 2);
            if (!lev) abort();
            memset(lev + maxlev, 0, sizeof(level_t) * (size_t)maxlev);
            maxlev *= 2;
        }
        level_t *f = &lev[L], *c = &lev[L + 1];
        int32_t fn = f->g.n, fnnz = f->g.xadj[fn];
        int32_t *labels = (int32_t *)xcalloc((size_t)fn, sizeof(int32_t));
        orc_lp_stats st;
        if (p->lp_async == 2 || p->lp_async == 3) orc_lp_cluster_colour(&f->g, ucl, p->rounds_coarsen, labels, &st);
        else if (p->lp_async == 1) orc_lp_cluster_async(&f->g, ucl, p->rounds_coarsen, labels, &st);
        else orc_lp_cluster(&f->g, ucl, p->rounds_coarsen,
                            lp_flags(p) | ((p->active_set & 1) ? ORC_LP_ACTIVE_SET : 0), labels, &st);
        ev_cluster += st.edge_visits;
        c->xadj = (int32_t *)xcalloc((size_t)fn + 1, sizeof(int32_t));
        c->adjncy = (int32_t *)xcalloc((size_t)fnnz, sizeof(int32_t));
        c->adjwgt = (int32_t *)xcalloc((size_t)fnnz, sizeof(int32_t));
        c->vwgt = (int32_t *)xcalloc((size_t)fn, sizeof(int32_t));
        f->f2c = (int32_t *)xcalloc((size_t)fn, sizeof(int32_t));
        int32_t nc, nnzc;
        orc_contract(&f->g, labels, c->xadj, c->adjncy, c->adjwgt, c->vwgt, f->f2c, &nc, &nnzc);
        free(labels);
        c->g = (orc_graph){nc, c->xadj, c->adjncy, c->adjwgt, c->vwgt};
        if (nc == fn) {
            free(c->xadj); free(c->adjncy); free(c->adjwgt); free(c->vwgt); free(f->f2c);
            memset(c, 0, sizeof(*c));
            f->f2c = NULL;
            break;
        }
        L++;
        if ((int64_t)p->stall_den * nc > (int64_t)p->stall_num * fn) break;
    }
    h->lev = lev;
    h->L = L;
    h->newid = newid;
    h->lmax = lmax;
    h->ucl = ucl;
    h->ev_cluster = ev_cluster;
}

static void free_hierarchy(hierarchy_t *h) {
    for (int32_t l = 0; l <= h->L; l++) {
        free(h->lev[l].xadj); free(h->lev[l].adjncy); free(h->lev[l].adjwgt); free(h->lev[l].vwgt);
        free(h->lev[l].f2c);
    }
    free(h->lev);
    free(h->newid);
}

/*
 * Initial partition of the coarsest graph (§III-B), with the project's
 * learned proposal when asked for: the network's logits are decoded under
 * the block bound (orc_mpnn_decode); that proposal goes through the same LP
 * refinement and rebalance as every bisection try and is kept iff it is
 * balanced and either the plain result is not balanced or it cuts no more
 * edge weight (ties keep the proposal). A proposal with a non-finite logit is
 * discarded before decoding.
 */
static void initial_with_judge(const orc_graph *gc, int32_t k, int64_t lmax, const orc_params *p, int32_t *P,
                               orc_result *res) {
    int32_t nc = gc->n;
    if (nc > 0)
        orc_initial_partition(gc, k, lmax, p->seed, p->attempts, p->rounds_refine, p->dir_alternate, p->init_fm,
                              P);
    int32_t tried = 0, kept = 0;
    int64_t pcut = -1, lcut = -1;
    if (p->init_mode == 1 && nc > 0 && nc <= p->mpnn_max_n && p->mpnn_params) {
        tried = 1;
        pcut = orc_cut(gc, P);
        int64_t *B = (int64_t *)xcalloc((size_t)k, sizeof(int64_t));
        orc_block_weights(gc, P, k, B);
        int pbal = 1;
        for (int32_t b = 0; b < k; b++) if (B[b] > lmax) pbal = 0;
        free(B);
        float *Z = (float *)xcalloc((size_t)nc * k, sizeof(float));
        int32_t *Pl = (int32_t *)xcalloc((size_t)nc, sizeof(int32_t));
        orc_mpnn_infer(gc, k, p->mpnn_params, p->mpnn_seed, Z, Pl);
        int finite = 1;
        for (int64_t i = 0; i < (int64_t)nc * k; i++) if (!isfinite(Z[i])) finite = 0;
        if (finite) {
            orc_mpnn_decode(gc, k, Z, lmax, Pl);
            orc_lp_refine(gc, k, lmax, p->rounds_refine, p->dir_alternate, Pl, NULL);
            int lbal = orc_rebalance(gc, k, lmax, Pl);
            lcut = orc_cut(gc, Pl);
            if (lbal && (!pbal || lcut <= pcut)) {
                kept = 1;
                memcpy(P, Pl, sizeof(int32_t) * (size_t)nc);
            }
        }
        free(Z);
        free(Pl);
    }
    if (res) {
        res->learned_tried = tried;
        res->learned_kept = kept;
        res->plain_cut_coarsest = pcut;
        res->learned_cut_coarsest = lcut;
    }
}

int orc_coarsest(const orc_graph *g, int32_t k, double eps, const orc_params *p, int32_t *xadj_c,
                 int32_t *adjncy_c, int32_t *adjwgt_c, int32_t *vwgt_c, int32_t *part_c, int32_t *n_c,
                 int32_t *nnz_c) {
    hierarchy_t h;
    coarsen(g, k, eps, p, &h);
    const orc_graph *gc = &h.lev[h.L].g;
    int32_t nc = gc->n, nnzc = gc->xadj[nc];
    memcpy(xadj_c, gc->xadj, sizeof(int32_t) * ((size_t)nc + 1));
    memcpy(adjncy_c, gc->adjncy, sizeof(int32_t) * (size_t)nnzc);
    memcpy(adjwgt_c, gc->adjwgt, sizeof(int32_t) * (size_t)nnzc);
    memcpy(vwgt_c, gc->vwgt, sizeof(int32_t) * (size_t)nc);
    initial_with_judge(gc, k, h.lmax, p, part_c, NULL);
    *n_c = nc;
    *nnz_c = nnzc;
    free_hierarchy(&h);
    return 0;
}

/*
 * §III multilevel scheme: coarsen (above), initial partition of the coarsest
 * level, then project and refine every level with U = L_max (§III-C); the
 * vertices without neighbours are filled in at the end.
 */
int orc_partition(const orc_graph *g, int32_t k, double eps, const orc_params *p,
                  int32_t *part_out, orc_result *res) {
    int32_t n = g->n;
    hierarchy_t h;
    coarsen(g, k, eps, p, &h);
    level_t *lev = h.lev;
    int32_t L = h.L;
    int64_t lmax = h.lmax;

    int32_t *P = (int32_t *)xcalloc((size_t)lev[L].g.n, sizeof(int32_t));
    orc_result tmp;
    memset(&tmp, 0, sizeof(tmp));
    initial_with_judge(&lev[L].g, k, lmax, p, P, &tmp);
    int64_t ev_refine = 0;
    for (int32_t l = L; l >= 0; l--) {
        if (l < L) {
            int32_t *Pf = (int32_t *)xcalloc((size_t)lev[l].g.n, sizeof(int32_t));
            orc_project(lev[l].g.n, lev[l].f2c, P, Pf);
            free(P);
            P = Pf;
        }
        orc_lp_stats st;
        if (p->lp_async == 2) orc_lp_refine_colour(&lev[l].g, k, lmax, p->rounds_refine, P, &st);
        else if (p->lp_async == 1) orc_lp_refine_async(&lev[l].g, k, lmax, p->rounds_refine, P, &st);
        else orc_lp_refine(&lev[l].g, k, lmax, p->rounds_refine,
                           lp_flags(p) | ((p->active_set & 2) ? ORC_LP_ACTIVE_SET : 0), P, &st);
        ev_refine += st.edge_visits;
        if (p->mls > 0) orc_mls_batched(&lev[l].g, k, lmax, P, p->seed, p->mls, 0.1, 50, p->mls_batch,
                                        p->mls_queue, NULL);
    }

    /* back to original ids, then place the isolated vertices */
    int64_t *B = (int64_t *)xcalloc((size_t)k, sizeof(int64_t));
    int32_t niso = 0;
    for (int32_t v = 0; v < n; v++) {
        int32_t i = h.newid[v];
        if (i >= 0) { part_out[v] = P[i]; B[P[i]] += VW(g, v); }
        else { part_out[v] = -1; niso++; }
    }
    orc_fill_isolated(g, k, part_out, B);

    int64_t maxb = 0;
    for (int32_t b = 0; b < k; b++) if (B[b] > maxb) maxb = B[b];
    if (res) {
        *res = tmp;
        res->cut = orc_cut(g, part_out);
        res->max_block_w = maxb;
        res->lmax = lmax;
        res->ucl = h.ucl;
        res->balanced = maxb <= lmax;
        res->levels = L + 1;
        res->edge_visits_cluster = h.ev_cluster;
        res->edge_visits_refine = ev_refine;
        res->coarsest_n = lev[L].g.n;
        res->n_isolated = niso;
    }
    free_hierarchy(&h);
    free(P);
    free(B);
    return (maxb <= lmax) ? 0 : 1;
}
