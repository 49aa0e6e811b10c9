/*
 * Seeded synthetic inputs for the random-walk engine and its oracle.
 *
 * This module generates *inputs only*: R-MAT graphs in CSR form, per-edge
 * weights and labels, query sources and MetaPath schemas.  It holds none of
 * the walk method's arithmetic (no sampling, no Philox, no tables).  Both the
 * oracle and the HIP path consume what it writes, as data.
 *
 * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): every edge sample picks one
 * of four adjacency-matrix quadrants per level with probabilities (a,b,c,d),
 * for `scale` levels, which yields the source and destination bits.  The
 * paper's workloads are real graphs with power-law degrees and edge weights /
 * labels attached uniformly at random (Experimental Setup, "Workloads"); R-MAT
 * with a seeded vertex permutation stands in for them.
 *
 * Randomness: a stateless 64-bit mixer (SplitMix64 finaliser, Steele, Lea and
 * Flood, OOPSLA 2014) applied to (seed, index), so results do not depend on
 * the number of threads.
 *
 * Pipeline:
 *   1. samples i in [0, S): quadrant walk -> (u, v); a seeded permutation of
 *      the vertex ids is applied; self-loops are dropped.
 *   2. symmetric graphs emit (u,v) and (v,u); directed graphs emit (u,v).
 *   3. counting sort by source into rows, sort each row, drop duplicates.
 *   4. weights w in [1,255] and labels in [0,L) as a hash of the edge key
 *      (the unordered pair on symmetric graphs, so both directions agree).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

static inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline uint64_t hash2(uint64_t seed, uint64_t i) {
    return mix64(mix64(seed) ^ (i * 0xD1B54A32D192ED03ull));
}

/* Seeded Fisher-Yates permutation of [0, n). */
int synth_permutation(int64_t n, uint64_t seed, int32_t *perm) {
    for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; i--) {
        uint64_t r = hash2(seed ^ 0x5045524D5554ull, (uint64_t)i);
        int64_t j = (int64_t)(((unsigned __int128)r * (uint64_t)(i + 1)) >> 64);
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    return 0;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static void sort_row(int32_t *p, int64_t len) {
    if (len < 2) return;
    if (len <= 32) {
        for (int64_t i = 1; i < len; i++) {
            int32_t v = p[i]; int64_t j = i - 1;
            while (j >= 0 && p[j] > v) { p[j + 1] = p[j]; j--; }
            p[j + 1] = v;
        }
        return;
    }
    qsort(p, (size_t)len, sizeof(int32_t), cmp_i32);
}

/*
 * Build an R-MAT CSR graph.
 *   scale      : n = 2^scale vertices
 *   n_samples  : number of R-MAT edge samples (n*deg for directed, n*deg/2 for symmetric)
 *   a,b,c      : quadrant probabilities (d = 1-a-b-c), as doubles converted once to
 *                32-bit thresholds
 *   symmetric  : emit both directions of every sample
 *   row_ptr    : out, int64[n+1] (caller-allocated)
 *   col        : out, int32[cap] (caller-allocated; cap >= n_samples * (symmetric ? 2 : 1))
 * Returns the realized number of directed edges m (after dropping self-loops and duplicates),
 * or -1 on allocation failure.
 */
int64_t synth_rmat_csr(int scale, int64_t n_samples, double a, double b, double c,
                       int symmetric, uint64_t seed, int64_t *row_ptr, int32_t *col) {
    const int64_t n = (int64_t)1 << scale;
    const uint64_t ta = (uint64_t)(a * 4294967296.0);
    const uint64_t tb = (uint64_t)((a + b) * 4294967296.0);
    const uint64_t tc = (uint64_t)((a + b + c) * 4294967296.0);
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *su = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_samples);
    int32_t *sv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_samples);
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!perm || !su || !sv || !cnt) { free(perm); free(su); free(sv); free(cnt); return -1; }
    synth_permutation(n, seed, perm);

    /* 1. samples */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_samples; i++) {
        uint64_t u = 0, v = 0, r = 0;
        for (int lvl = 0; lvl < scale; lvl++) {
            if ((lvl & 1) == 0) r = hash2(seed, (uint64_t)i * 32u + (uint64_t)(lvl >> 1));
            uint64_t x = (lvl & 1) ? (r >> 32) : (r & 0xFFFFFFFFull);
            /* quadrant (u bit, v bit): [0,ta) -> (0,0), [ta,tb) -> (0,1),
               [tb,tc) -> (1,0), [tc,2^32) -> (1,1); written without branches */
            u = (u << 1) | (uint64_t)(x >= tb);
            v = (v << 1) | ((uint64_t)(x >= ta) ^ (uint64_t)(x >= tb) ^ (uint64_t)(x >= tc));
        }
        int32_t pu = perm[u], pv = perm[v];
        if (pu == pv) { su[i] = -1; sv[i] = -1; }
        else { su[i] = pu; sv[i] = pv; }
    }

    /* 2./3. counting sort by source, in two levels so that the scattered
       writes stay within caches: the directed edges are first partitioned by
       source block (each thread writes its share of every block), then each
       block is counting-sorted by source into its rows.  Rows are sorted and
       deduplicated afterwards, so the order of a row's entries here does not
       matter. */
    const int nthr = omp_get_max_threads();
    const int blk_bits = scale > 10 ? scale - 10 : 0;        /* at most 1024 source blocks */
    const int64_t nblk = ((n - 1) >> blk_bits) + 1;
    const int64_t m_cap = n_samples * (symmetric ? 2 : 1);
    int64_t *bcnt = (int64_t *)calloc((size_t)(nblk * nthr + 1), sizeof(int64_t));
    uint64_t *pairs = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m_cap > 0 ? m_cap : 1));
    if (!bcnt || !pairs) { free(bcnt); free(pairs); free(perm); free(su); free(sv); free(cnt); return -1; }
#pragma omp parallel num_threads(nthr)
    {
        const int t = omp_get_thread_num();
        const int64_t lo = n_samples * t / nthr, hi = n_samples * (t + 1) / nthr;
        int64_t *mine = bcnt + (int64_t)t * nblk;
        for (int64_t i = lo; i < hi; i++) {
            if (su[i] < 0) continue;
            mine[su[i] >> blk_bits]++;
            if (symmetric) mine[sv[i] >> blk_bits]++;
        }
#pragma omp barrier
#pragma omp single
        {   /* block-major, thread-minor offsets */
            int64_t acc = 0;
            for (int64_t b = 0; b < nblk; b++)
                for (int tt = 0; tt < nthr; tt++) {
                    int64_t c = bcnt[(int64_t)tt * nblk + b];
                    bcnt[(int64_t)tt * nblk + b] = acc;
                    acc += c;
                }
            bcnt[(int64_t)nthr * nblk] = acc;
        }
        for (int64_t i = lo; i < hi; i++) {
            if (su[i] < 0) continue;
            const uint64_t u = (uint32_t)su[i], v = (uint32_t)sv[i];
            pairs[mine[u >> blk_bits]++] = (u << 32) | v;
            if (symmetric) pairs[mine[v >> blk_bits]++] = (v << 32) | u;
        }
    }
    const int64_t m_raw = bcnt[(int64_t)nthr * nblk];
    free(su); free(sv); free(perm);
    /* block b's edges are pairs[start_b, end_b): start_b is thread 0's start,
       end_b the next block's (after the second loop each thread's offset has
       advanced to the next thread's start) */
    int64_t *bstart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nblk + 1));
    if (!bstart) { free(bcnt); free(pairs); free(cnt); return -1; }
    bstart[0] = 0;
    for (int64_t b = 1; b < nblk; b++) bstart[b] = bcnt[(int64_t)(nthr - 1) * nblk + (b - 1)];
    bstart[nblk] = m_raw;
    free(bcnt);
    /* row sizes, then row offsets, then each block sorted into its rows */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < nblk; b++)
        for (int64_t e = bstart[b]; e < bstart[b + 1]; e++) cnt[(pairs[e] >> 32) + 1]++;
    for (int64_t v = 0; v < n; v++) cnt[v + 1] += cnt[v];
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!cur) { free(bstart); free(pairs); free(cnt); return -1; }
    memcpy(cur, cnt, sizeof(int64_t) * (size_t)n);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < nblk; b++)
        for (int64_t e = bstart[b]; e < bstart[b + 1]; e++) {
            const uint64_t pr = pairs[e];
            col[cur[pr >> 32]++] = (int32_t)(uint32_t)pr;
        }
    free(cur); free(bstart); free(pairs);

    /* sort rows, drop duplicates (in place, per row) */
    int64_t *newdeg = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!newdeg) { free(cnt); return -1; }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < n; v++) {
        int32_t *p = col + cnt[v];
        int64_t len = cnt[v + 1] - cnt[v];
        sort_row(p, len);
        int64_t k = 0;
        for (int64_t i = 0; i < len; i++)
            if (k == 0 || p[i] != p[k - 1]) p[k++] = p[i];
        newdeg[v] = k;
    }
    /* compact the rows to the left: through a second array, in parallel
       (an in-place move in parallel could overwrite rows not yet moved) */
    row_ptr[0] = 0;
    for (int64_t v = 0; v < n; v++) row_ptr[v + 1] = row_ptr[v] + newdeg[v];
    const int64_t m = row_ptr[n];
    int32_t *packed = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    if (!packed) { free(newdeg); free(cnt); return -1; }
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < n; v++)
        memcpy(packed + row_ptr[v], col + cnt[v], sizeof(int32_t) * (size_t)newdeg[v]);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; e++) col[e] = packed[e];
    free(packed);
    free(newdeg); free(cnt);
    return row_ptr[n];
}

/* Per-edge weights in [lo, hi] and labels in [0, n_labels) keyed by the edge.
 * On symmetric graphs the key is the unordered pair so both directions agree. */
int synth_edge_attrs(int64_t n, const int64_t *row_ptr, const int32_t *col, int symmetric,
                     uint64_t seed, uint32_t w_lo, uint32_t w_hi, uint32_t n_labels,
                     uint32_t *w_out, uint8_t *label_out) {
    const uint64_t span = (uint64_t)w_hi - (uint64_t)w_lo + 1u;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t u = 0; u < n; u++) {
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
            uint64_t v = (uint64_t)(uint32_t)col[e];
            uint64_t x = (uint64_t)u, y = v;
            if (symmetric && x > y) { uint64_t t = x; x = y; y = t; }
            uint64_t key = (x << 32) | y;
            uint64_t h = hash2(seed, key);
            if (w_out) w_out[e] = w_lo + (uint32_t)(((h & 0xFFFFFFFFull) * span) >> 32);
            if (label_out) label_out[e] = (uint8_t)(((h >> 32) * (uint64_t)n_labels) >> 32);
        }
    }
    return 0;
}

/* nq query sources uniform in [0, n). */
int synth_sources(int64_t nq, int64_t n, uint64_t seed, int32_t *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nq; i++) {
        uint64_t h = hash2(seed, (uint64_t)i);
        out[i] = (int32_t)(((h & 0xFFFFFFFFull) * (uint64_t)n) >> 32);
    }
    return 0;
}

/* Generic uniform integers in [0, bound) (schemas, request sizes, algorithm picks). */
int synth_uniform_u32(int64_t count, uint64_t bound, uint64_t seed, uint32_t *out) {
    for (int64_t i = 0; i < count; i++) {
        uint64_t h = hash2(seed, (uint64_t)i);
        out[i] = (uint32_t)(((h & 0xFFFFFFFFull) * bound) >> 32);
    }
    return 0;
}

/* Uniform 53-bit doubles in (0,1) for exponential inter-arrival gaps. */
int synth_uniform_f64(int64_t count, uint64_t seed, double *out) {
    for (int64_t i = 0; i < count; i++) {
        uint64_t h = hash2(seed, (uint64_t)i);
        out[i] = ((double)(h >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    }
    return 0;
}
