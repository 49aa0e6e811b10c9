/*
 * The C ABI driven from plain C (no Python, no torch): device buffers from
 * hipMalloc, a CSR graph, its ALIAS table, a PPR walk, the end-vertex counts
 * and their top 10.  Test input and output are raw little-endian files in
 * one directory:
 *   in : meta.txt ("n m nq max_len seed stop_q32"), row_ptr, col, weight, sources
 *   out: lengths, status, paths (nq rows of max_len + 1 int32), counts, top_ids, top_vals
 * Exit status 0 on success; any failing call prints trw_last_error().
 */
#define __HIP_PLATFORM_AMD__
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "trw.h"

static char dir[4096];

static void *read_file(const char *name, size_t bytes) {
    char path[4200];
    snprintf(path, sizeof(path), "%s/%s", dir, name);
    FILE *f = fopen(path, "rb");
    void *buf = malloc(bytes ? bytes : 1);
    if (!f || !buf || fread(buf, 1, bytes, f) != bytes) {
        fprintf(stderr, "cannot read %s\n", path);
        exit(2);
    }
    fclose(f);
    return buf;
}

static void write_file(const char *name, const void *buf, size_t bytes) {
    char path[4200];
    snprintf(path, sizeof(path), "%s/%s", dir, name);
    FILE *f = fopen(path, "wb");
    if (!f || fwrite(buf, 1, bytes, f) != bytes) {
        fprintf(stderr, "cannot write %s\n", path);
        exit(2);
    }
    fclose(f);
}

#define HIP(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { \
    fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_)); return 3; } } while (0)
#define TRW(x) do { trw_status s_ = (x); if (s_ != TRW_OK) { \
    fprintf(stderr, "%s: status %d: %s\n", #x, (int)s_, trw_last_error()); return 4; } } while (0)

static void *dalloc(size_t bytes) {
    void *p = NULL;
    if (hipMalloc(&p, bytes ? bytes : 256) != hipSuccess) {
        fprintf(stderr, "hipMalloc(%zu) failed\n", bytes);
        exit(3);
    }
    return p;
}

int main(int argc, char **argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s <dir>\n", argv[0]);
        return 1;
    }
    snprintf(dir, sizeof(dir), "%s", argv[1]);
    long long n, m, nq;
    unsigned max_len, stop;
    unsigned long long seed;
    char path[4200];
    snprintf(path, sizeof(path), "%s/meta.txt", dir);
    FILE *mf = fopen(path, "r");
    if (!mf || fscanf(mf, "%lld %lld %lld %u %llu %u", &n, &m, &nq, &max_len, &seed, &stop) != 6) return 2;
    fclose(mf);

    int32_t *h_rp = read_file("row_ptr", sizeof(int32_t) * (size_t)(n + 1));
    int32_t *h_col = read_file("col", sizeof(int32_t) * (size_t)m);
    uint32_t *h_w = read_file("weight", sizeof(uint32_t) * (size_t)m);
    int32_t *h_src = read_file("sources", sizeof(int32_t) * (size_t)nq);

    int32_t *d_rp = dalloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *d_col = dalloc(sizeof(int32_t) * (size_t)m);
    uint32_t *d_w = dalloc(sizeof(uint32_t) * (size_t)m);
    int32_t *d_src = dalloc(sizeof(int32_t) * (size_t)nq);
    HIP(hipMemcpy(d_rp, h_rp, sizeof(int32_t) * (size_t)(n + 1), hipMemcpyHostToDevice));
    HIP(hipMemcpy(d_col, h_col, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice));
    HIP(hipMemcpy(d_w, h_w, sizeof(uint32_t) * (size_t)m, hipMemcpyHostToDevice));
    HIP(hipMemcpy(d_src, h_src, sizeof(int32_t) * (size_t)nq, hipMemcpyHostToDevice));

    trw_graph g;
    TRW(trw_graph_create(n, m, d_rp, d_col, d_w, NULL, 0, &g));
    void *d_scratch = dalloc(256);
    uint64_t n_bad = 0;
    TRW(trw_graph_validate(g, d_scratch, 256, NULL, &n_bad));

    size_t tbytes = 0;
    TRW(trw_table_bytes(g, TRW_S_ALIAS, &tbytes));
    void *d_table = dalloc(tbytes);
    trw_table alias;
    TRW(trw_table_build(g, TRW_S_ALIAS, d_table, tbytes, NULL, &alias));

    trw_walk_params p;
    memset(&p, 0, sizeof(p));
    p.algo = TRW_A_PPR;
    p.sampler = TRW_S_ALIAS;
    p.max_len = max_len;
    p.stop_q32 = stop;
    p.seed = seed;
    const uint64_t stride = max_len + 1;
    size_t wsb = 0;
    TRW(trw_walk_workspace_bytes(g, &p, (uint64_t)nq, TRW_M_PERSISTENT, &wsb));
    void *d_ws = dalloc(wsb);
    int32_t *d_paths = dalloc(sizeof(int32_t) * (size_t)nq * stride);
    uint32_t *d_len = dalloc(sizeof(uint32_t) * (size_t)nq);
    uint8_t *d_st = dalloc((size_t)nq);
    TRW(trw_walk(g, alias, &p, d_src, (uint64_t)nq, 0, d_paths, stride, d_len, d_st, TRW_M_PERSISTENT, NULL, d_ws,
                 wsb, NULL));

    uint32_t *d_counts = dalloc(sizeof(uint32_t) * (size_t)n);
    HIP(hipMemset(d_counts, 0, sizeof(uint32_t) * (size_t)n));
    TRW(trw_ppr_end_counts(g, d_paths, stride, d_len, d_st, (uint64_t)nq, 0, d_counts, (uint64_t)n, NULL, NULL));
    const uint32_t k = n < 10 ? (uint32_t)n : 10;
    size_t kb = 0;
    TRW(trw_topk_workspace_bytes((uint64_t)n, k, &kb));
    void *d_kws = dalloc(kb);
    int32_t *d_ids = dalloc(sizeof(int32_t) * k);
    uint32_t *d_vals = dalloc(sizeof(uint32_t) * k);
    TRW(trw_topk(d_counts, (uint64_t)n, k, d_ids, d_vals, d_kws, kb, NULL));
    HIP(hipDeviceSynchronize());

    int32_t *h_paths = malloc(sizeof(int32_t) * (size_t)nq * stride);
    uint32_t *h_len = malloc(sizeof(uint32_t) * (size_t)nq);
    uint8_t *h_st = malloc((size_t)nq);
    uint32_t *h_counts = malloc(sizeof(uint32_t) * (size_t)n);
    int32_t h_ids[10];
    uint32_t h_vals[10];
    HIP(hipMemcpy(h_paths, d_paths, sizeof(int32_t) * (size_t)nq * stride, hipMemcpyDeviceToHost));
    HIP(hipMemcpy(h_len, d_len, sizeof(uint32_t) * (size_t)nq, hipMemcpyDeviceToHost));
    HIP(hipMemcpy(h_st, d_st, (size_t)nq, hipMemcpyDeviceToHost));
    HIP(hipMemcpy(h_counts, d_counts, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToHost));
    HIP(hipMemcpy(h_ids, d_ids, sizeof(int32_t) * k, hipMemcpyDeviceToHost));
    HIP(hipMemcpy(h_vals, d_vals, sizeof(uint32_t) * k, hipMemcpyDeviceToHost));
    write_file("paths", h_paths, sizeof(int32_t) * (size_t)nq * stride);
    write_file("lengths", h_len, sizeof(uint32_t) * (size_t)nq);
    write_file("status", h_st, (size_t)nq);
    write_file("counts", h_counts, sizeof(uint32_t) * (size_t)n);
    write_file("top_ids", h_ids, sizeof(int32_t) * k);
    write_file("top_vals", h_vals, sizeof(uint32_t) * k);

    TRW(trw_table_destroy(alias));
    TRW(trw_graph_destroy(g));
    printf("walked %lld queries from C\n", nq);
    return 0;
}
