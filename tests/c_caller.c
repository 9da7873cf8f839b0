/*
 * A plain C caller of the partitioner's C ABI (include/gp.h): no Python and no
 * torch, only the HIP runtime for device memory.
 *
 * GRAPH is a binary file: int32 n, int32 nnz, int32 xadj[n + 1],
 * int32 adjncy[nnz] (a symmetric CSR graph with unit weights, §II-A).
 *
 * c_caller partition GRAPH K PART
 *   Partitions the graph twice with the default parameters and eps = 0.03:
 *   on the library's cached scratch (ws = NULL), then on a caller workspace of
 *   exactly the size the first call reports; both must agree. Writes
 *   int32 part[n] to PART and prints "ok cut=... max_block_w=... lmax=...
 *   levels=... ws=...".
 *
 * c_caller steps GRAPH K U OUT
 *   One level of the multilevel scheme (§III) by hand, every call on one
 *   caller workspace sized by gp_workspace_bytes: clustering with bound U
 *   (10 rounds), contraction, refinement of the coarse graph from the
 *   partition i mod K (25 rounds), projection, refinement of the fine graph,
 *   cut and block weights. Writes OUT/labels.bin [n], OUT/coarse.bin
 *   (n_c, nnz_c, xadj_c, adjncy_c, adjwgt_c, vwgt_c), OUT/f2c.bin [n],
 *   OUT/partc.bin [n_c] and OUT/partf.bin [n]; prints "ok cut=... moves_c=...
 *   moves_rc=... moves_rf=... B=b0,b1,...".
 *
 * Exit codes: 0 ok, 1 usage or file error, 2 HIP error, 3 library error,
 * 4 the two partition calls disagree.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gp.h"

#define HIP_OK(x)                                                                  \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));         \
            return 2;                                                              \
        }                                                                          \
    } while (0)

#define GP_OK_OR_EXIT(call)                                                        \
    do {                                                                           \
        int rc_ = (call);                                                          \
        if (rc_ < 0) {                                                             \
            fprintf(stderr, "%s: %s: %s\n", #call, gp_strerror(rc_), gp_last_error()); \
            return 3;                                                              \
        }                                                                          \
    } while (0)

static size_t nz(size_t count) { return count ? count : 1; }

static int32_t *read_ints(FILE *f, size_t count) {
    int32_t *p = (int32_t *)malloc(nz(count) * sizeof(int32_t));
    if (p && count && fread(p, sizeof(int32_t), count, f) != count) {
        free(p);
        return NULL;
    }
    return p;
}

static int write_ints(const char *dir, const char *name, const int32_t *const *parts, const size_t *counts,
                      int nparts) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "wb");
    if (!f) return 1;
    for (int i = 0; i < nparts; i++)
        if (counts[i] && fwrite(parts[i], sizeof(int32_t), counts[i], f) != counts[i]) {
            fclose(f);
            return 1;
        }
    fclose(f);
    return 0;
}

/* device array [count] -> new host array */
static int32_t *to_host(const int32_t *d, size_t count) {
    int32_t *h = (int32_t *)malloc(nz(count) * sizeof(int32_t));
    if (h && count && hipMemcpy(h, d, count * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) {
        free(h);
        return NULL;
    }
    return h;
}

static int run_partition(const gp_graph *g, int32_t k, const char *out_path) {
    const int32_t n = g->n;
    int32_t *d_part = NULL, *d_part2 = NULL;
    HIP_OK(hipMalloc((void **)&d_part, sizeof(int32_t) * nz((size_t)n)));
    HIP_OK(hipMalloc((void **)&d_part2, sizeof(int32_t) * nz((size_t)n)));
    gp_params p;
    gp_default_params(&p);
    gp_result r, r2;
    GP_OK_OR_EXIT(gp_partition(g, k, 0.03, &p, d_part, &r, NULL, 0, NULL));

    /* the same call on a caller workspace of the reported size: no allocation by the library */
    void *ws = NULL;
    const size_t ws_bytes = nz((size_t)r.workspace_bytes);
    HIP_OK(hipMalloc(&ws, ws_bytes));
    GP_OK_OR_EXIT(gp_partition(g, k, 0.03, &p, d_part2, &r2, ws, ws_bytes, NULL));

    int32_t *part = to_host(d_part, (size_t)n), *part2 = to_host(d_part2, (size_t)n);
    if (!part || !part2) return 2;
    if (memcmp(part, part2, sizeof(int32_t) * (size_t)n) != 0 || r.cut != r2.cut || r.max_block_w != r2.max_block_w) {
        fprintf(stderr, "the workspace call differs from the cached call\n");
        return 4;
    }
    FILE *o = fopen(out_path, "wb");
    if (!o || (n && fwrite(part, sizeof(int32_t), (size_t)n, o) != (size_t)n)) {
        fprintf(stderr, "cannot write %s\n", out_path);
        return 1;
    }
    fclose(o);
    printf("ok cut=%lld max_block_w=%lld lmax=%lld levels=%d ws=%zu\n", (long long)r.cut, (long long)r.max_block_w,
           (long long)r.lmax, r.levels, (size_t)r.workspace_bytes);
    HIP_OK(hipFree(ws));
    HIP_OK(hipFree(d_part));
    HIP_OK(hipFree(d_part2));
    free(part);
    free(part2);
    return 0;
}

static size_t max_sz(size_t a, size_t b) { return a > b ? a : b; }

static int run_steps(const gp_graph *g, int32_t k, int64_t U, const char *dir) {
    const int32_t n = g->n, nnz = g->nnz;
    const int32_t dirs = GP_LP_DIR_ALTERNATE;
    const int64_t lmax = gp_lmax(n, k, 0.03); /* unit weights: c(V) = n at every level */

    /* one workspace for every call, sized for the fine graph */
    size_t need = gp_workspace_bytes(GP_OP_LP_CLUSTER, n, nnz, 1, dirs);
    need = max_sz(need, gp_workspace_bytes(GP_OP_CONTRACT, n, nnz, 1, 0));
    need = max_sz(need, gp_workspace_bytes(GP_OP_LP_REFINE, n, nnz, k, dirs));
    need = max_sz(need, gp_workspace_bytes(GP_OP_CUT, n, nnz, k, 0));
    if (need == 0) {
        fprintf(stderr, "gp_workspace_bytes: %s\n", gp_last_error());
        return 3;
    }
    void *ws = NULL;
    HIP_OK(hipMalloc(&ws, need));

    int32_t *labels, *xc, *ac, *wc, *vc, *f2c, *partc, *partf;
    int64_t *B;
    HIP_OK(hipMalloc((void **)&labels, sizeof(int32_t) * nz((size_t)n)));
    HIP_OK(hipMalloc((void **)&xc, sizeof(int32_t) * ((size_t)n + 1)));
    HIP_OK(hipMalloc((void **)&ac, sizeof(int32_t) * nz((size_t)nnz)));
    HIP_OK(hipMalloc((void **)&wc, sizeof(int32_t) * nz((size_t)nnz)));
    HIP_OK(hipMalloc((void **)&vc, sizeof(int32_t) * nz((size_t)n)));
    HIP_OK(hipMalloc((void **)&f2c, sizeof(int32_t) * nz((size_t)n)));
    HIP_OK(hipMalloc((void **)&partc, sizeof(int32_t) * nz((size_t)n)));
    HIP_OK(hipMalloc((void **)&partf, sizeof(int32_t) * nz((size_t)n)));
    HIP_OK(hipMalloc((void **)&B, sizeof(int64_t) * (size_t)k));

    /* clustering (§III-A) and contraction */
    gp_lp_stats sc, src, srf;
    GP_OK_OR_EXIT(gp_lp_cluster(g, U, 10, dirs, labels, &sc, ws, need, NULL));
    int32_t n_c = 0, nnz_c = 0;
    GP_OK_OR_EXIT(gp_contract(g, labels, xc, ac, wc, vc, f2c, &n_c, &nnz_c, ws, need, NULL));
    const gp_graph cg = {n_c, nnz_c, xc, ac, wc, vc};

    /* refinement of the coarse graph from i mod k (§III-C, U = L_max) */
    int32_t *h = (int32_t *)malloc(nz((size_t)n_c) * sizeof(int32_t));
    if (!h) return 1;
    for (int32_t i = 0; i < n_c; i++) h[i] = i % k;
    if (n_c) HIP_OK(hipMemcpy(partc, h, sizeof(int32_t) * (size_t)n_c, hipMemcpyHostToDevice));
    free(h);
    const size_t need_c = gp_workspace_bytes(GP_OP_LP_REFINE, n_c, nnz_c, k, dirs);
    if (need_c == 0 || need_c > need) {
        fprintf(stderr, "coarse refinement needs %zu bytes, the workspace holds %zu\n", need_c, need);
        return 3;
    }
    GP_OK_OR_EXIT(gp_lp_refine(&cg, k, lmax, 25, dirs, partc, &src, ws, need, NULL));

    /* projection and refinement of the fine graph, then cut and block weights */
    GP_OK_OR_EXIT(gp_project(n, f2c, partc, partf, NULL));
    GP_OK_OR_EXIT(gp_lp_refine(g, k, lmax, 25, dirs, partf, &srf, ws, need, NULL));
    int64_t cut = 0;
    GP_OK_OR_EXIT(gp_cut_and_blocks(g, k, partf, &cut, B, ws, need, NULL));
    HIP_OK(hipDeviceSynchronize());

    int32_t *h_lab = to_host(labels, (size_t)n), *h_f2c = to_host(f2c, (size_t)n);
    int32_t *h_xc = to_host(xc, (size_t)n_c + 1), *h_ac = to_host(ac, (size_t)nnz_c);
    int32_t *h_wc = to_host(wc, (size_t)nnz_c), *h_vc = to_host(vc, (size_t)n_c);
    int32_t *h_pc = to_host(partc, (size_t)n_c), *h_pf = to_host(partf, (size_t)n);
    int64_t *h_B = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    if (!h_lab || !h_f2c || !h_xc || !h_ac || !h_wc || !h_vc || !h_pc || !h_pf || !h_B) return 2;
    HIP_OK(hipMemcpy(h_B, B, sizeof(int64_t) * (size_t)k, hipMemcpyDeviceToHost));
    const int32_t sizes[2] = {n_c, nnz_c};
    {
        const int32_t *parts[] = {h_lab};
        const size_t counts[] = {(size_t)n};
        if (write_ints(dir, "labels.bin", parts, counts, 1)) return 1;
    }
    {
        const int32_t *parts[] = {sizes, h_xc, h_ac, h_wc, h_vc};
        const size_t counts[] = {2, (size_t)n_c + 1, (size_t)nnz_c, (size_t)nnz_c, (size_t)n_c};
        if (write_ints(dir, "coarse.bin", parts, counts, 5)) return 1;
    }
    {
        const int32_t *parts[] = {h_f2c};
        const size_t counts[] = {(size_t)n};
        if (write_ints(dir, "f2c.bin", parts, counts, 1)) return 1;
    }
    {
        const int32_t *parts[] = {h_pc};
        const size_t counts[] = {(size_t)n_c};
        if (write_ints(dir, "partc.bin", parts, counts, 1)) return 1;
    }
    {
        const int32_t *parts[] = {h_pf};
        const size_t counts[] = {(size_t)n};
        if (write_ints(dir, "partf.bin", parts, counts, 1)) return 1;
    }
    printf("ok cut=%lld moves_c=%lld moves_rc=%lld moves_rf=%lld B=", (long long)cut, (long long)sc.moves,
           (long long)src.moves, (long long)srf.moves);
    for (int32_t b = 0; b < k; b++) printf(b ? ",%lld" : "%lld", (long long)h_B[b]);
    printf("\n");

    free(h_lab);
    free(h_f2c);
    free(h_xc);
    free(h_ac);
    free(h_wc);
    free(h_vc);
    free(h_pc);
    free(h_pf);
    free(h_B);
    HIP_OK(hipFree(labels));
    HIP_OK(hipFree(xc));
    HIP_OK(hipFree(ac));
    HIP_OK(hipFree(wc));
    HIP_OK(hipFree(vc));
    HIP_OK(hipFree(f2c));
    HIP_OK(hipFree(partc));
    HIP_OK(hipFree(partf));
    HIP_OK(hipFree(B));
    HIP_OK(hipFree(ws));
    return 0;
}

int main(int argc, char **argv) {
    const int steps = argc == 6 && strcmp(argv[1], "steps") == 0;
    if (!steps && !(argc == 5 && strcmp(argv[1], "partition") == 0)) {
        fprintf(stderr, "usage: %s partition GRAPH K PART | %s steps GRAPH K U OUT\n", argv[0], argv[0]);
        return 1;
    }
    const int32_t k = atoi(argv[3]);
    FILE *f = fopen(argv[2], "rb");
    int32_t hdr[2];
    if (!f || fread(hdr, sizeof(int32_t), 2, f) != 2 || hdr[0] < 0 || hdr[1] < 0) {
        fprintf(stderr, "cannot read %s\n", argv[2]);
        return 1;
    }
    const int32_t n = hdr[0], nnz = hdr[1];
    int32_t *xadj = read_ints(f, (size_t)n + 1), *adjncy = read_ints(f, (size_t)nnz);
    fclose(f);
    if (!xadj || !adjncy) {
        fprintf(stderr, "short file %s\n", argv[2]);
        return 1;
    }
    int32_t *d_xadj = NULL, *d_adjncy = NULL;
    HIP_OK(hipMalloc((void **)&d_xadj, sizeof(int32_t) * ((size_t)n + 1)));
    HIP_OK(hipMalloc((void **)&d_adjncy, sizeof(int32_t) * nz((size_t)nnz)));
    HIP_OK(hipMemcpy(d_xadj, xadj, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice));
    if (nnz) HIP_OK(hipMemcpy(d_adjncy, adjncy, sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice));
    const gp_graph g = {n, nnz, d_xadj, d_adjncy, NULL, NULL};

    const int rc = steps ? run_steps(&g, k, (int64_t)atoll(argv[4]), argv[5]) : run_partition(&g, k, argv[4]);
    if (rc != 0) return rc;
    HIP_OK(hipFree(d_xadj));
    HIP_OK(hipFree(d_adjncy));
    if (gp_release_cache() < 0) return 3;
    free(xadj);
    free(adjncy);
    return 0;
}
