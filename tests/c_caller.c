/*
 * A plain C caller of the partitioner's C ABI (include/gp.h): no Python and no
 * torch, only the HIP runtime for device memory.
 *
 * Usage: c_caller GRAPH K PART
 *   GRAPH: binary file int32 n, int32 nnz, int32 xadj[n + 1], int32 adjncy[nnz]
 *          (a symmetric CSR graph with unit weights, §II-A)
 *   PART:  written as int32 part[n], the k-way partition of gp_partition
 *
 * The graph is partitioned twice with the default parameters and eps = 0.03:
 * first on the library's cached scratch (ws = NULL), then on a caller
 * workspace of exactly the size the first call reports. Both partitions must
 * agree. Prints one line "ok cut=... max_block_w=... lmax=... levels=...".
 * Exit codes: 0 ok, 1 usage or input error, 2 HIP error, 3 library error,
 * 4 the two calls disagree.
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

static int32_t *read_ints(FILE *f, size_t count) {
    int32_t *p = (int32_t *)malloc(count ? count * sizeof(int32_t) : 1);
    if (p && count && fread(p, sizeof(int32_t), count, f) != count) {
        free(p);
        return NULL;
    }
    return p;
}

int main(int argc, char **argv) {
    if (argc != 4) {
        fprintf(stderr, "usage: %s GRAPH K PART\n", argv[0]);
        return 1;
    }
    const int32_t k = atoi(argv[2]);
    FILE *f = fopen(argv[1], "rb");
    int32_t hdr[2];
    if (!f || fread(hdr, sizeof(int32_t), 2, f) != 2 || hdr[0] < 0 || hdr[1] < 0) {
        fprintf(stderr, "cannot read %s\n", argv[1]);
        return 1;
    }
    const int32_t n = hdr[0], nnz = hdr[1];
    int32_t *xadj = read_ints(f, (size_t)n + 1), *adjncy = read_ints(f, (size_t)nnz);
    fclose(f);
    if (!xadj || !adjncy) {
        fprintf(stderr, "short file %s\n", argv[1]);
        return 1;
    }

    int32_t *d_xadj = NULL, *d_adjncy = NULL, *d_part = NULL, *d_part2 = NULL;
    HIP_OK(hipMalloc((void **)&d_xadj, sizeof(int32_t) * ((size_t)n + 1)));
    HIP_OK(hipMalloc((void **)&d_adjncy, sizeof(int32_t) * (nnz ? (size_t)nnz : 1)));
    HIP_OK(hipMalloc((void **)&d_part, sizeof(int32_t) * (n ? (size_t)n : 1)));
    HIP_OK(hipMalloc((void **)&d_part2, sizeof(int32_t) * (n ? (size_t)n : 1)));
    HIP_OK(hipMemcpy(d_xadj, xadj, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice));
    if (nnz) HIP_OK(hipMemcpy(d_adjncy, adjncy, sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice));

    const gp_graph g = {n, nnz, d_xadj, d_adjncy, NULL, NULL};
    gp_params p;
    gp_default_params(&p);
    gp_result r, r2;
    int rc = gp_partition(&g, k, 0.03, &p, d_part, &r, NULL, 0, NULL);
    if (rc < 0) {
        fprintf(stderr, "gp_partition: %s: %s\n", gp_strerror(rc), gp_last_error());
        return 3;
    }

    /* the same call on a caller workspace of the reported size: no allocation by the library */
    void *ws = NULL;
    const size_t ws_bytes = (size_t)r.workspace_bytes;
    HIP_OK(hipMalloc(&ws, ws_bytes ? ws_bytes : 1));
    rc = gp_partition(&g, k, 0.03, &p, d_part2, &r2, ws, ws_bytes ? ws_bytes : 1, NULL);
    if (rc < 0) {
        fprintf(stderr, "gp_partition (workspace): %s: %s\n", gp_strerror(rc), gp_last_error());
        return 3;
    }

    int32_t *part = (int32_t *)malloc(sizeof(int32_t) * (n ? (size_t)n : 1));
    int32_t *part2 = (int32_t *)malloc(sizeof(int32_t) * (n ? (size_t)n : 1));
    if (!part || !part2) return 1;
    if (n) {
        HIP_OK(hipMemcpy(part, d_part, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(part2, d_part2, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost));
    }
    if ((n && memcmp(part, part2, sizeof(int32_t) * (size_t)n) != 0) || r.cut != r2.cut ||
        r.max_block_w != r2.max_block_w) {
        fprintf(stderr, "the workspace call differs from the cached call\n");
        return 4;
    }
    FILE *o = fopen(argv[3], "wb");
    if (!o || (n && fwrite(part, sizeof(int32_t), (size_t)n, o) != (size_t)n)) {
        fprintf(stderr, "cannot write %s\n", argv[3]);
        return 1;
    }
    fclose(o);
    printf("ok cut=%lld max_block_w=%lld lmax=%lld levels=%d ws=%zu\n", (long long)r.cut, (long long)r.max_block_w,
           (long long)r.lmax, r.levels, ws_bytes);

    HIP_OK(hipFree(ws));
    HIP_OK(hipFree(d_xadj));
    HIP_OK(hipFree(d_adjncy));
    HIP_OK(hipFree(d_part));
    HIP_OK(hipFree(d_part2));
    if (gp_release_cache() < 0) return 3;
    free(xadj);
    free(adjncy);
    free(part);
    free(part2);
    return 0;
}
