/*
 * mpnn.c — plain CPU oracle of the learned initial partition's network
 * (test infrastructure; see oracle.h).
 *
 * The paper computes the initial partition of the coarsest graph with
 * recursive bisection (§III-B). The project adds a message-passing network
 * that proposes that k-way assignment; the plain initial partitioner stays the
 * judge. This file is the binary32 inference, written as its definition:
 *
 *   features   X[v] = ( c(v)/c_max, deg(v)/max_deg, y_8[v][0..15] )
 *              y_0[v][j] = +-1 from a seeded splitmix64 stream,
 *              y_{t+1} = (y_t + D^-1 A y_t) / 2        (lazy random walk, A weighted)
 *   layer      h'[v] = ReLU(b + Ws h[v] + Wn m[v]),  m[v] = (sum_u w(v,u) h[u]) / sum_u w(v,u)
 *   head       z[v] = bh + Wh h3[v],  block(v) = argmax_c z[v][c], ties -> lowest c
 *
 * Exactness contract (so that a GPU implementation can match bit for bit):
 *  - weights are used after rounding to bfloat16 (round to nearest, ties to
 *    even), as binary32 values;
 *  - every sum is a chain of fused multiply-adds (fmaf) in a fixed order:
 *    neighbours in CSR order starting from 0, then inputs in index order
 *    starting from the bias (self inputs first, then aggregated inputs);
 *  - the reciprocal 1/sum_u w(v,u) and the two ratio features are computed in
 *    binary64 and rounded once to binary32; edge weights enter as (float)w;
 *  - vertices without neighbours keep y (walk) and get m = 0 (layers).
 * The file is compiled with -ffp-contract=off so that no other product or sum
 * is fused.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define NPROBE 16
#define NWALK 8
#define NFEAT (2 + NPROBE)
#define HID 64

static void *xmalloc(size_t bytes) {
    void *p = malloc(bytes ? bytes : 1);
    if (!p) abort();
    return p;
}

/* Parameter layout (binary32, flat): for layers l = 1..3 with input width
 * d_1 = 18, d_2 = d_3 = 64: Ws_l [64][d_l], Wn_l [64][d_l], b_l [64]; then
 * Wh [k][64], bh [k]. Matrices are row-major with the output index first. */
int32_t orc_mpnn_param_count(int32_t k) {
    return (2 * HID * NFEAT + HID) + 2 * (2 * HID * HID + HID) + HID * k + k;
}

/* Round a binary32 value to the nearest bfloat16 (ties to even), returned as binary32. */
float orc_bf16(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu) != 0) {
        u = (u & 0xffff0000u) | 0x00400000u; /* NaN stays a (quiet) NaN */
    } else {
        uint32_t lsb = (u >> 16) & 1u;
        u = (u + 0x7fffu + lsb) & 0xffff0000u;
    }
    float r;
    memcpy(&r, &u, 4);
    return r;
}

static uint64_t splitmix(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static float edge_w(const orc_graph *g, int32_t e) { return g->adjwgt ? (float)g->adjwgt[e] : 1.0f; }

/* 1 / sum of the edge weights at v, binary64 then binary32; 0 when v has no neighbour. */
static float inv_wdeg(const orc_graph *g, int32_t v) {
    int64_t s = 0;
    for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) s += g->adjwgt ? g->adjwgt[e] : 1;
    return s > 0 ? (float)(1.0 / (double)s) : 0.0f;
}

void orc_mpnn_features(const orc_graph *g, uint64_t seed, float *X) {
    const int32_t n = g->n;
    int64_t cmax = 0, dmax = 0;
    for (int32_t v = 0; v < n; v++) {
        int64_t c = g->vwgt ? g->vwgt[v] : 1, d = g->xadj[v + 1] - g->xadj[v];
        if (c > cmax) cmax = c;
        if (d > dmax) dmax = d;
    }
    float *y = (float *)xmalloc(sizeof(float) * (size_t)n * NPROBE);
    float *y2 = (float *)xmalloc(sizeof(float) * (size_t)n * NPROBE);
    const uint64_t base = splitmix(seed);
    for (int32_t v = 0; v < n; v++)
        for (int j = 0; j < NPROBE; j++) {
            uint64_t h = splitmix(base ^ ((uint64_t)v * NPROBE + (uint64_t)j));
            y[(size_t)v * NPROBE + j] = (h >> 63) ? -1.0f : 1.0f;
        }
    for (int t = 0; t < NWALK; t++) {
        for (int32_t v = 0; v < n; v++) {
            const float r = inv_wdeg(g, v);
            const int has = g->xadj[v + 1] > g->xadj[v];
            for (int j = 0; j < NPROBE; j++) {
                float acc = 0.0f;
                for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++)
                    acc = fmaf(edge_w(g, e), y[(size_t)g->adjncy[e] * NPROBE + j], acc);
                const float self = y[(size_t)v * NPROBE + j];
                y2[(size_t)v * NPROBE + j] = has ? (self + acc * r) * 0.5f : self;
            }
        }
        float *tmp = y;
        y = y2;
        y2 = tmp;
    }
    for (int32_t v = 0; v < n; v++) {
        int64_t c = g->vwgt ? g->vwgt[v] : 1, d = g->xadj[v + 1] - g->xadj[v];
        X[(size_t)v * NFEAT + 0] = (float)((double)c / (double)cmax);
        X[(size_t)v * NFEAT + 1] = dmax > 0 ? (float)((double)d / (double)dmax) : 0.0f;
        for (int j = 0; j < NPROBE; j++) X[(size_t)v * NFEAT + 2 + j] = y[(size_t)v * NPROBE + j];
    }
    free(y);
    free(y2);
}

/* One message-passing layer: H [n][din] -> O [n][64]. W points at Ws (bf16-rounded copy). */
static void layer(const orc_graph *g, int32_t din, const float *W, const float *H, float *O) {
    const float *Ws = W, *Wn = W + HID * din, *b = W + 2 * HID * din;
    float *m = (float *)xmalloc(sizeof(float) * (size_t)din);
    for (int32_t v = 0; v < g->n; v++) {
        const float r = inv_wdeg(g, v);
        const int has = g->xadj[v + 1] > g->xadj[v];
        for (int32_t i = 0; i < din; i++) {
            float acc = 0.0f;
            for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++)
                acc = fmaf(edge_w(g, e), H[(size_t)g->adjncy[e] * din + i], acc);
            m[i] = has ? acc * r : 0.0f;
        }
        for (int32_t o = 0; o < HID; o++) {
            float acc = b[o];
            for (int32_t i = 0; i < din; i++) acc = fmaf(Ws[o * din + i], H[(size_t)v * din + i], acc);
            for (int32_t i = 0; i < din; i++) acc = fmaf(Wn[o * din + i], m[i], acc);
            O[(size_t)v * HID + o] = acc > 0.0f ? acc : 0.0f;
        }
    }
    free(m);
}

void orc_mpnn_infer(const orc_graph *g, int32_t k, const float *params, uint64_t seed, float *Z, int32_t *part) {
    const int32_t n = g->n, P = orc_mpnn_param_count(k);
    float *W = (float *)xmalloc(sizeof(float) * (size_t)P);
    for (int32_t i = 0; i < P; i++) W[i] = orc_bf16(params[i]);
    float *X = (float *)xmalloc(sizeof(float) * (size_t)n * NFEAT);
    float *Ha = (float *)xmalloc(sizeof(float) * (size_t)n * HID);
    float *Hb = (float *)xmalloc(sizeof(float) * (size_t)n * HID);
    orc_mpnn_features(g, seed, X);
    const float *w = W;
    layer(g, NFEAT, w, X, Ha);
    w += 2 * HID * NFEAT + HID;
    layer(g, HID, w, Ha, Hb);
    w += 2 * HID * HID + HID;
    layer(g, HID, w, Hb, Ha);
    w += 2 * HID * HID + HID;
    const float *Wh = w, *bh = w + HID * k;
    for (int32_t v = 0; v < n; v++) {
        int32_t best = 0;
        for (int32_t c = 0; c < k; c++) {
            float acc = bh[c];
            for (int32_t i = 0; i < HID; i++) acc = fmaf(Wh[c * HID + i], Ha[(size_t)v * HID + i], acc);
            Z[(size_t)v * k + c] = acc;
            if (c > 0 && acc > Z[(size_t)v * k + best]) best = c;
        }
        if (part) part[v] = best;
    }
    free(W);
    free(X);
    free(Ha);
    free(Hb);
}

/*
 * Capacity-respecting decoding of the logits (project-defined): the network's
 * preferences are admitted under the same rule as a label-propagation move
 * (§IV-A: a vertex joins a block only while the block stays within its
 * bound). Every vertex ranks the blocks by logit, highest first (ties ->
 * lower block). In round r = 0..k-1 every vertex not yet placed proposes its
 * r-th block; the proposers to block t are admitted in ascending vertex id
 * while B[t] + (weight of all proposers to t up to and including v) <= L_max.
 * Vertices still unplaced after k rounds go, in ascending id, to the block
 * that is lightest at that moment (ties -> lowest block).
 */
void orc_mpnn_decode(const orc_graph *g, int32_t k, const float *Z, int64_t lmax, int32_t *part) {
    const int32_t n = g->n;
    int32_t *pref = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)n * (size_t)k);
    for (int32_t v = 0; v < n; v++) {
        const float *z = Z + (size_t)v * k;
        for (int32_t c = 0; c < k; c++) {
            int32_t rank = 0;
            for (int32_t d = 0; d < k; d++)
                if (z[d] > z[c] || (z[d] == z[c] && d < c)) rank++;
            pref[(size_t)v * k + rank] = c;
        }
        part[v] = -1;
    }
    int64_t *B = (int64_t *)calloc((size_t)k, sizeof(int64_t));
    int64_t *run = (int64_t *)calloc((size_t)k, sizeof(int64_t));
    if (!B || !run) abort();
    for (int32_t r = 0; r < k; r++) {
        for (int32_t t = 0; t < k; t++) run[t] = B[t];
        for (int32_t v = 0; v < n; v++) {
            if (part[v] >= 0) continue;
            const int32_t t = pref[(size_t)v * k + r];
            const int64_t c = g->vwgt ? g->vwgt[v] : 1;
            run[t] += c;
            if (run[t] <= lmax) part[v] = -2 - t; /* admitted this round, applied below */
        }
        for (int32_t v = 0; v < n; v++)
            if (part[v] <= -2) {
                part[v] = -2 - part[v];
                B[part[v]] += g->vwgt ? g->vwgt[v] : 1;
            }
    }
    for (int32_t v = 0; v < n; v++) {
        if (part[v] >= 0) continue;
        int32_t b = 0;
        for (int32_t t = 1; t < k; t++)
            if (B[t] < B[b]) b = t;
        part[v] = b;
        B[b] += g->vwgt ? g->vwgt[v] : 1;
    }
    free(pref);
    free(B);
    free(run);
}
