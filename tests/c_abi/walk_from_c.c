/*
 * The C ABI driven from plain C (no Python, no torch): device buffers from
 * hipMalloc, a CSR graph, its ALIAS table, a PPR walk, the end-vertex counts
 * and their top 10; the same walk streamed to a file by the library's file
 * sink; a server given six requests of three kinds (one with host
 * buffers); and the walk again from the graph written to a CSR file.  Test input and output are raw little-endian files in one
 * directory:
 *   in : meta.txt ("n m nq max_len seed stop_q32"), row_ptr, col, weight, sources
 *   out: lengths, status, paths (nq rows of max_len + 1 int32), counts, top_ids, top_vals,
 *        stream.bin (trw_chunk_to_fd records), srv<i>_{paths,lengths,status} for request i
 *        (sources [i nq / 6, (i + 1) nq / 6), qid_base its first index; kinds PPR ALIAS,
 *        DeepWalk ALIAS, Node2Vec O-REJ in turn; max_len, 40 and 40; path_stride
 *        max_len + 1; request 3 with host buffers), graph.csr (the graph as a CSR file) and
 *        disk_{paths,lengths,status} (the PPR walk from that file, 2 of its partitions resident)
 * Exit status 0 on success; any failing call prints trw_last_error().
 */
#define __HIP_PLATFORM_AMD__
#include <hip/hip_runtime_api.h>
#include <fcntl.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

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

    /* The same walk streamed to disk by the library's file sink. */
    {
        const uint32_t chunk = 4097;
        size_t sdb = 0, shb = 0;
        TRW(trw_walk_stream_bytes(g, &p, chunk, &sdb, &shb));
        void *d_sws = dalloc(sdb);
        void *h_pin = NULL;
        HIP(hipHostMalloc(&h_pin, shb, hipHostMallocDefault));
        snprintf(path, sizeof(path), "%s/stream.bin", dir);
        int fd = open(path, O_WRONLY | O_CREAT | O_TRUNC, 0644);
        if (fd < 0) return 2;
        TRW(trw_walk_stream(g, alias, &p, d_src, (uint64_t)nq, 0, chunk, NULL, d_sws, sdb, h_pin, shb,
                            trw_chunk_to_fd, &fd, NULL));
        close(fd);
        HIP(hipHostFree(h_pin));
        HIP(hipFree(d_sws));
    }

    /* A server: six requests of three kinds; request 3 with host buffers. */
    {
        size_t eb = 0;
        TRW(trw_edge_index_bytes(g, &eb));
        void *d_eidx = dalloc(eb);
        trw_table eidx;
        TRW(trw_edge_index_build(g, d_eidx, eb, NULL, &eidx));
        trw_server_cfg cfg;
        memset(&cfg, 0, sizeof(cfg));
        cfg.use_hipgraph = 1;
        size_t ab = 0;
        TRW(trw_server_arena_bytes(&cfg, (size_t)64 << 20, &ab));
        void *d_arena = dalloc(ab);
        trw_server srv;
        TRW(trw_server_create(g, alias, eidx, &cfg, d_arena, ab, &srv));
        enum { R = 6 };
        trw_request req[R];
        void *outs[R][3];
        uint64_t ids[R];
        for (int i = 0; i < R; ++i) {
            const long long lo = nq * i / R, hi = nq * (i + 1) / R;
            const int kind = i % 3;
            trw_request *r = &req[i];
            memset(r, 0, sizeof(*r));
            r->params.algo = kind == 0 ? TRW_A_PPR : kind == 1 ? TRW_A_DEEPWALK : TRW_A_NODE2VEC;
            r->params.sampler = kind == 2 ? TRW_S_OREJ : TRW_S_ALIAS;
            r->params.max_len = kind == 0 ? max_len : 40;
            r->params.stop_q32 = kind == 0 ? stop : 0;
            r->params.n2v_thr_q16[0] = 16384;      /* p = 2, q = 0.5: 1/p, 1, 1/q over their maximum 2 */
            r->params.n2v_thr_q16[1] = 32768;
            r->params.n2v_thr_q16[2] = 65536;
            r->params.seed = seed + (unsigned long long)i;
            r->nq = (uint32_t)(hi - lo);
            r->qid_base = (uint64_t)lo;
            r->path_stride = r->params.max_len + 1;
            const size_t pb = sizeof(int32_t) * r->nq * r->path_stride, lb = sizeof(uint32_t) * r->nq;
            if (i == 3) {
                r->flags = TRW_REQ_HOST;
                r->sources = h_src + lo;
                outs[i][0] = malloc(pb); outs[i][1] = malloc(lb); outs[i][2] = malloc(r->nq);
            } else {
                r->sources = d_src + lo;
                outs[i][0] = dalloc(pb); outs[i][1] = dalloc(lb); outs[i][2] = dalloc(r->nq);
            }
            r->paths = outs[i][0];
            r->lengths = outs[i][1];
            r->status = outs[i][2];
            TRW(trw_server_submit(srv, r, &ids[i]));
        }
        int done = 0;
        trw_completion comp[R];
        for (int tries = 0; done < R && tries < 600; ++tries) {
            uint32_t got = 0;
            trw_status st = trw_server_poll(srv, comp, R, &got, 100);
            if (st != TRW_OK && st != TRW_E_TIMEOUT) TRW(st);
            for (uint32_t c = 0; c < got; ++c) {
                if (comp[c].status != TRW_OK) {
                    fprintf(stderr, "request %llu ended with %d\n", (unsigned long long)comp[c].request_id,
                            (int)comp[c].status);
                    return 5;
                }
            }
            done += (int)got;
        }
        if (done < R) {
            fprintf(stderr, "the server completed %d of %d requests\n", done, R);
            return 5;
        }
        for (int i = 0; i < R; ++i) {
            const trw_request *r = &req[i];
            const size_t pb = sizeof(int32_t) * r->nq * r->path_stride, lb = sizeof(uint32_t) * r->nq;
            void *hp = outs[i][0], *hl = outs[i][1], *hs = outs[i][2];
            if (i != 3) {
                hp = malloc(pb); hl = malloc(lb); hs = malloc(r->nq);
                HIP(hipMemcpy(hp, outs[i][0], pb, hipMemcpyDeviceToHost));
                HIP(hipMemcpy(hl, outs[i][1], lb, hipMemcpyDeviceToHost));
                HIP(hipMemcpy(hs, outs[i][2], r->nq, hipMemcpyDeviceToHost));
            }
            char name[64];
            snprintf(name, sizeof(name), "srv%d_paths", i); write_file(name, hp, pb);
            snprintf(name, sizeof(name), "srv%d_lengths", i); write_file(name, hl, lb);
            snprintf(name, sizeof(name), "srv%d_status", i); write_file(name, hs, r->nq);
            if (i != 3) {
                for (int k = 0; k < 3; ++k) HIP(hipFree(outs[i][k]));
            }
            free(hp); free(hl); free(hs);
        }
        TRW(trw_server_destroy(srv));
        TRW(trw_table_destroy(eidx));
        HIP(hipFree(d_arena));
        HIP(hipFree(d_eidx));
    }

    /* The graph written to a CSR file and walked from it: partitions of m / 5
     * edges, two resident at once. */
    {
        int64_t *rp64 = malloc(sizeof(int64_t) * (size_t)(n + 1));
        for (long long v = 0; v <= n; ++v) rp64[v] = h_rp[v];
        snprintf(path, sizeof(path), "%s/graph.csr", dir);
        TRW(trw_disk_graph_write(path, n, m, rp64, h_col, h_w, NULL));
        free(rp64);
        trw_disk_graph dg;
        TRW(trw_disk_graph_open(path, (uint64_t)(m / 5), &dg));
        uint32_t parts = 0;
        TRW(trw_disk_graph_info(dg, NULL, NULL, NULL, &parts));
        size_t ddb = 0, dhb = 0;
        TRW(trw_disk_walk_bytes(dg, &p, (uint64_t)nq, 2, &ddb, &dhb));
        void *d_dws = dalloc(ddb);
        void *h_dpin = NULL;
        HIP(hipHostMalloc(&h_dpin, dhb, hipHostMallocDefault));
        int32_t *d_dpaths = dalloc(sizeof(int32_t) * (size_t)nq * stride);
        uint32_t *d_dlen = dalloc(sizeof(uint32_t) * (size_t)nq);
        uint8_t *d_dst = dalloc((size_t)nq);
        trw_disk_walk_stats ds;
        TRW(trw_disk_walk(dg, &p, d_src, (uint64_t)nq, 0, d_dpaths, stride, d_dlen, d_dst, 2, d_dws, ddb, h_dpin, dhb,
                          &ds, NULL));
        HIP(hipMemcpy(h_paths, d_dpaths, sizeof(int32_t) * (size_t)nq * stride, hipMemcpyDeviceToHost));
        HIP(hipMemcpy(h_len, d_dlen, sizeof(uint32_t) * (size_t)nq, hipMemcpyDeviceToHost));
        HIP(hipMemcpy(h_st, d_dst, (size_t)nq, hipMemcpyDeviceToHost));
        write_file("disk_paths", h_paths, sizeof(int32_t) * (size_t)nq * stride);
        write_file("disk_lengths", h_len, sizeof(uint32_t) * (size_t)nq);
        write_file("disk_status", h_st, (size_t)nq);
        printf("disk walk: %u partitions, %llu rounds, %llu loads, %llu bytes read\n", parts,
               (unsigned long long)ds.runs, (unsigned long long)ds.loads, (unsigned long long)ds.bytes_read);
        TRW(trw_disk_graph_close(dg));
        HIP(hipHostFree(h_dpin));
        HIP(hipFree(d_dws));
        HIP(hipFree(d_dpaths));
        HIP(hipFree(d_dlen));
        HIP(hipFree(d_dst));
    }

    TRW(trw_table_destroy(alias));
    TRW(trw_graph_destroy(g));
    printf("walked %lld queries from C (batch, streamed to disk, served, from a graph file)\n", nq);
    return 0;
}
