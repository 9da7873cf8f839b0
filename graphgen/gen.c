/*
 * graphgen — seeded synthetic input graphs (symmetric int32 CSR).
 *
 * This module only builds inputs. It contains none of the partitioner's
 * arithmetic; both the CPU oracle and the GPU library consume what it writes.
 *
 * Random numbers: counter-based splitmix64 (Steele, Lea & Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014). The i-th output of
 * stream `seed` is the splitmix64 finaliser applied to seed + (i+1)*gamma.
 * A uniform double in [0,1) is (x >> 11) * 2^-53.
 *
 * Families (all symmetric, no self-loops, no duplicate edges, rows ascending):
 *   rgg2d : n points in the unit square, point i = (U(2i), U(2i+1)); edge iff
 *           squared Euclidean distance < r^2 (the random geometric graph
 *           family of the paper's instance section, radius 0.55*sqrt(ln n/n)).
 *   rmat  : R-MAT with probabilities (a,b,c,d); edge e draws one uniform per
 *           level l (counter e*scale+l), quadrant a=(0,0) b=(0,1) c=(1,0)
 *           d=(1,1), most significant bit first; then symmetrise, dedup,
 *           drop self-loops. No noise, no permutation.
 *   grid3d: X*Y*Z six-neighbour grid, id = x + X*y + X*Y*z; optional edge
 *           weights 1 + (R(3*min(u,v)+axis) mod wmax).
 *
 * Memory: every array returned through an out-pointer is malloc'ed here and
 * must be released with gg_free().
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define GG_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t gg_fin(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* i-th output of the splitmix64 stream started at `seed`. */
uint64_t gg_rand(uint64_t seed, uint64_t i) { return gg_fin(seed + (i + 1) * GG_GAMMA); }

static inline double gg_u01(uint64_t seed, uint64_t i) {
    return (double)(gg_rand(seed, i) >> 11) * (1.0 / 9007199254740992.0);
}

void gg_free(void *p) { free(p); }

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static void sort_row(int32_t *a, int64_t len) {
    if (len <= 32) {
        for (int64_t i = 1; i < len; i++) {
            int32_t x = a[i];
            int64_t j = i - 1;
            while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; j--; }
            a[j + 1] = x;
        }
    } else {
        qsort(a, (size_t)len, sizeof(int32_t), cmp_i32);
    }
}

/*
 * Build a symmetric CSR from an undirected edge list (src[e], dst[e]).
 * Self-loops are dropped, both directions are inserted, rows are sorted and
 * duplicates removed. Returns nnz (directed entries) or -1 on overflow /
 * allocation failure.
 */
static int64_t build_csr(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                         int32_t **xadj_out, int32_t **adj_out) {
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; e++) {
        int32_t u = src[e], v = dst[e];
        if (u == v) continue;
#pragma omp atomic
        cnt[u + 1]++;
#pragma omp atomic
        cnt[v + 1]++;
    }
    for (int64_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
    int64_t total = cnt[n];
    int32_t *tmp = (int32_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
    int64_t *cur = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!tmp || !cur) { free(cnt); free(tmp); free(cur); return -1; }
    memcpy(cur, cnt, (size_t)n * sizeof(int64_t));
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; e++) {
        int32_t u = src[e], v = dst[e];
        if (u == v) continue;
        int64_t pu, pv;
#pragma omp atomic capture
        pu = cur[u]++;
#pragma omp atomic capture
        pv = cur[v]++;
        tmp[pu] = v;
        tmp[pv] = u;
    }
    free(cur);
    int64_t *deg = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!deg) { free(cnt); free(tmp); return -1; }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < n; v++) {
        int32_t *row = tmp + cnt[v];
        int64_t len = cnt[v + 1] - cnt[v];
        sort_row(row, len);
        int64_t w = 0;
        for (int64_t i = 0; i < len; i++)
            if (w == 0 || row[i] != row[w - 1]) row[w++] = row[i];
        deg[v] = w;
    }
    int64_t nnz = 0;
    for (int64_t v = 0; v < n; v++) nnz += deg[v];
    if (nnz >= 2147483647LL) { free(cnt); free(tmp); free(deg); return -1; }
    int32_t *xadj = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
    int32_t *adj = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    if (!xadj || !adj) { free(cnt); free(tmp); free(deg); free(xadj); free(adj); return -1; }
    xadj[0] = 0;
    for (int64_t v = 0; v < n; v++) xadj[v + 1] = (int32_t)(xadj[v] + deg[v]);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < n; v++)
        memcpy(adj + xadj[v], tmp + cnt[v], (size_t)deg[v] * sizeof(int32_t));
    free(cnt); free(tmp); free(deg);
    *xadj_out = xadj;
    *adj_out = adj;
    return nnz;
}

/* 2-D random geometric graph; edge iff dx^2+dy^2 < r^2 (binary64). */
int64_t gg_rgg2d(int64_t n, uint64_t seed, double r, int32_t **xadj, int32_t **adj) {
    if (n < 0 || n >= 2147483647LL || !(r > 0.0)) return -1;
    double *px = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *py = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!px || !py) { free(px); free(py); return -1; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        px[i] = gg_u01(seed, (uint64_t)(2 * i));
        py[i] = gg_u01(seed, (uint64_t)(2 * i + 1));
    }
    /* bucket points into square cells of side >= r */
    int64_t g = (int64_t)floor(1.0 / r);
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    int64_t ncell = g * g;
    int64_t *cstart = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int32_t *order = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t *cellof = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!cstart || !order || !cellof) { free(px); free(py); free(cstart); free(order); free(cellof); return -1; }
    for (int64_t i = 0; i < n; i++) {
        int64_t cx = (int64_t)(px[i] * (double)g), cy = (int64_t)(py[i] * (double)g);
        if (cx >= g) cx = g - 1;
        if (cy >= g) cy = g - 1;
        cellof[i] = cx + g * cy;
        cstart[cellof[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; c++) cstart[c + 1] += cstart[c];
    {
        int64_t *fill = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
        if (!fill) { free(px); free(py); free(cstart); free(order); free(cellof); return -1; }
        memcpy(fill, cstart, (size_t)ncell * sizeof(int64_t));
        for (int64_t i = 0; i < n; i++) order[fill[cellof[i]]++] = (int32_t)i;
        free(fill);
    }
    /* count, then emit each edge once as (i, j) with i < j */
    double r2 = r * r;
    int64_t *ecnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *es = NULL, *ed = NULL;
    if (!ecnt) { free(px); free(py); free(cstart); free(order); free(cellof); return -1; }
    for (int pass = 0; pass < 2; pass++) {
        if (pass == 1) {
            for (int64_t i = 0; i < n; i++) ecnt[i + 1] += ecnt[i];
            es = (int32_t *)malloc((size_t)(ecnt[n] > 0 ? ecnt[n] : 1) * sizeof(int32_t));
            ed = (int32_t *)malloc((size_t)(ecnt[n] > 0 ? ecnt[n] : 1) * sizeof(int32_t));
            if (!es || !ed) break;
        }
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; i++) {
            int64_t cx = cellof[i] % g, cy = cellof[i] / g;
            int64_t w = pass == 1 ? ecnt[i] : 0, c = 0;
            for (int64_t dy = -1; dy <= 1; dy++)
                for (int64_t dx = -1; dx <= 1; dx++) {
                    int64_t x = cx + dx, y = cy + dy;
                    if (x < 0 || y < 0 || x >= g || y >= g) continue;
                    int64_t cell = x + g * y;
                    for (int64_t p = cstart[cell]; p < cstart[cell + 1]; p++) {
                        int32_t j = order[p];
                        if (j <= i) continue;
                        double ddx = px[i] - px[j], ddy = py[i] - py[j];
                        if (ddx * ddx + ddy * ddy < r2) {
                            if (pass == 0) c++;
                            else { es[w] = (int32_t)i; ed[w] = j; w++; }
                        }
                    }
                }
            if (pass == 0) ecnt[i + 1] = c;
        }
    }
    int64_t m = ecnt[n];
    int ok = es && ed;
    free(px); free(py); free(cstart); free(order); free(cellof); free(ecnt);
    int64_t nnz = ok ? build_csr(n, m, es, ed, xadj, adj) : -1;
    free(es); free(ed);
    return nnz;
}

/* R-MAT with (a, b, c, 1-a-b-c) and m edge draws on 2^scale vertices. */
int64_t gg_rmat_m(int32_t scale, int64_t m, double a, double b, double c, uint64_t seed, int32_t **xadj,
                  int32_t **adj) {
    if (scale < 1 || scale > 30 || m < 0) return -1;
    int64_t n = (int64_t)1 << scale;
    int32_t *src = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int32_t *dst = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    if (!src || !dst) { free(src); free(dst); return -1; }
    double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; e++) {
        uint32_t u = 0, v = 0;
        for (int32_t l = 0; l < scale; l++) {
            double x = gg_u01(seed, (uint64_t)e * (uint64_t)scale + (uint64_t)l);
            uint32_t bu, bv;
            if (x < a) { bu = 0; bv = 0; }
            else if (x < ab) { bu = 0; bv = 1; }
            else if (x < abc) { bu = 1; bv = 0; }
            else { bu = 1; bv = 1; }
            u = (u << 1) | bu;
            v = (v << 1) | bv;
        }
        src[e] = (int32_t)u;
        dst[e] = (int32_t)v;
    }
    int64_t nnz = build_csr(n, m, src, dst, xadj, adj);
    free(src); free(dst);
    return nnz;
}

/* R-MAT with m = edge_factor * 2^scale draws. */
int64_t gg_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c, uint64_t seed,
                int32_t **xadj, int32_t **adj) {
    if (edge_factor < 1) return -1;
    return gg_rmat_m(scale, (int64_t)edge_factor << scale, a, b, c, seed, xadj, adj);
}

/* Six-neighbour grid. If wmax > 0, *adjwgt receives weights 1 + (R mod wmax). */
int64_t gg_grid3d(int32_t X, int32_t Y, int32_t Z, uint64_t seed, int32_t wmax,
                  int32_t **xadj_o, int32_t **adj_o, int32_t **wgt_o) {
    int64_t n = (int64_t)X * Y * Z;
    if (X < 1 || Y < 1 || Z < 1 || n >= 2147483647LL) return -1;
    int32_t *xadj = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
    if (!xadj) return -1;
    int64_t XY = (int64_t)X * Y;
    xadj[0] = 0;
    for (int64_t id = 0; id < n; id++) {
        int64_t x = id % X, y = (id / X) % Y, z = id / XY;
        int d = (z > 0) + (y > 0) + (x > 0) + (x < X - 1) + (y < Y - 1) + (z < Z - 1);
        if ((int64_t)xadj[id] + d >= 2147483647LL) { free(xadj); return -1; }
        xadj[id + 1] = xadj[id] + d;
    }
    int64_t nnz = xadj[n];
    int32_t *adj = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    int32_t *wgt = wmax > 0 ? (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t)) : NULL;
    if (!adj || (wmax > 0 && !wgt)) { free(xadj); free(adj); free(wgt); return -1; }
#pragma omp parallel for schedule(static)
    for (int64_t id = 0; id < n; id++) {
        int64_t x = id % X, y = (id / X) % Y, z = id / XY;
        int64_t p = xadj[id];
        /* neighbours in ascending id order: -XY, -X, -1, +1, +X, +XY */
        int64_t nb[6]; int ax[6]; int cnt = 0;
        if (z > 0) { nb[cnt] = id - XY; ax[cnt++] = 2; }
        if (y > 0) { nb[cnt] = id - X; ax[cnt++] = 1; }
        if (x > 0) { nb[cnt] = id - 1; ax[cnt++] = 0; }
        if (x < X - 1) { nb[cnt] = id + 1; ax[cnt++] = 0; }
        if (y < Y - 1) { nb[cnt] = id + X; ax[cnt++] = 1; }
        if (z < Z - 1) { nb[cnt] = id + XY; ax[cnt++] = 2; }
        for (int q = 0; q < cnt; q++) {
            adj[p + q] = (int32_t)nb[q];
            if (wgt) {
                int64_t lo = nb[q] < id ? nb[q] : id;
                wgt[p + q] = 1 + (int32_t)(gg_rand(seed, (uint64_t)(3 * lo + ax[q])) % (uint64_t)wmax);
            }
        }
    }
    *xadj_o = xadj;
    *adj_o = adj;
    if (wgt_o) *wgt_o = wgt;
    else free(wgt);
    return nnz;
}
