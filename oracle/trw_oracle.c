/*
 * ORACLE — test infrastructure, not product code.
 *
 * A plain, single-threaded CPU implementation of the random-walk method of
 * ThunderRW (Sun et al., "ThunderRW: An In-Memory Graph Random Walk Engine",
 * VLDB 2021), written from the paper for checking the HIP path.  Only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg load it.
 * It shares no code, header, table or constant with the HIP library.
 *
 * What is computed (paper section in brackets):
 *   - the execution paradigm: every query repeats "pick a random neighbour of
 *     the current vertex, append it" until it terminates [Introduction,
 *     execution-paradigm algorithm; Step-centric Programming, framework
 *     algorithm: Gather, Move, Update in a do-while loop];
 *   - the sampling methods NAIVE, ITS, ALIAS, REJ and O-REJ [Sampling
 *     Methods];
 *   - the preprocessing of static walks: one sampling table per vertex,
 *     built once [preprocessing algorithm];
 *   - the four applications PPR, DeepWalk, Node2Vec (the second-order
 *     transition equation and the Node2Vec listing), MetaPath [Random Walk
 *     based Algorithms];
 *   - Node2Vec on a weighted graph, whose transition weight is the edge
 *     weight times the second-order factor [Random Walk based Algorithms,
 *     Node2Vec], sampled by rejection against the row's largest weight
 *     [Sampling Methods, rejection sampling]; and Node2Vec sampled by ITS
 *     over weights computed at each step, the default the paper recommends
 *     for dynamic walks [Analysis, recommendation];
 *   - PPR's estimate from the end vertices of a source's queries, and the
 *     k highest-scoring vertices [Random Walk based Algorithms, PPR].
 *
 * The paper uses real-valued uniforms; the oracle fixes one integer random
 * contract so that a second implementation can be compared bit for bit:
 *   block(k, t) = Philox4x32-10(counter = (k, t, qid_lo, qid_hi),
 *                               key = (seed_lo, seed_hi))  -> words r0..r3
 *   uniform index in [0, d)  = floor(r * d / 2^32)       (r a 32-bit word)
 *   ALIAS coin               = r1 < thr                   (thr = floor(H * 2^32))
 *   ITS draw in [0, W)       = floor((r1:r0) * W / 2^64)  (64-bit word)
 *   PPR stop coin            = r2 < stop_q32              (after each move)
 *   O-REJ dart height        = r1 >> 16 against Q16 thresholds
 *   REJ dart (x, y)          = x from r0, hit iff r1 * p*_v < w_x * 2^32
 *                              (y = r1 * p*_v / 2^32 uniform in [0, p*_v))
 *   weighted Node2Vec dart   = x from r0, hit iff r1 * p*_v < w_x * a_x * 2^16
 *                              (a_x the Q16 second-order factor, 65536 for
 *                              the first move; y = r1 * p*_v * 2^16 / 2^32)
 *   dynamic ITS draw in [0, W) = floor(r0 * W / 2^32) while W < 2^32, else
 *                              floor((r1:r0) * W / 2^64)
 * Integer choices that the paper leaves open are listed with the readings in
 * the design notes of the repository.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC 2011).  Ten rounds; each round multiplies counter    */
/* words 0 and 2 by the two round multipliers, recombines the high and low   */
/* halves with words 1 and 3 and the key, and the key is bumped by the two   */
/* Weyl constants between rounds.                                            */
/* ------------------------------------------------------------------------ */
#define ORC_PHILOX_M0 0xD2511F53u
#define ORC_PHILOX_M1 0xCD9E8D57u
#define ORC_PHILOX_W0 0x9E3779B9u
#define ORC_PHILOX_W1 0xBB67AE85u

void trwo_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += ORC_PHILOX_W0; k1 += ORC_PHILOX_W1; }
        uint64_t p0 = (uint64_t)ORC_PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)ORC_PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void block(uint64_t seed, uint64_t qid, uint32_t k, uint32_t t, uint32_t r[4]) {
    uint32_t ctr[4] = { k, t, (uint32_t)qid, (uint32_t)(qid >> 32) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    trwo_philox4x32_10(ctr, key, r);
}

/* floor(r * d / 2^32): a uniform index in [0, d) from one 32-bit word. */
static uint32_t index_of(uint32_t r, uint32_t d) {
    return (uint32_t)(((uint64_t)r * (uint64_t)d) >> 32);
}

/* ------------------------------------------------------------------------ */
/* ALIAS initialization [Sampling Methods, alias sampling; Walker 1977],    */
/* built with Vose's worklist method in exact integer arithmetic.            */
/*                                                                          */
/* For a vertex with degree d and weights w_i, let W = sum w_i and scale     */
/* every weight to s_i = w_i * d, so that the average column holds exactly  */
/* W.  Columns below W go to a "small" stack, the others to a "large" stack */
/* (both last-in first-out, pushed in index order).  While both stacks are  */
/* non-empty: pop a small column l, look at the large column g on top; l's  */
/* bucket is (l with mass s_l, g with the rest); g gives up W - s_l and moves */
/* to the small stack if it falls below W.  Whatever remains on the large   */
/* stack is a full bucket (probability 1, alias = itself).                  */
/*                                                                          */
/* Output per edge slot j of the row: thr[j] = floor(s_j * 2^32 / W), or    */
/* 0xFFFFFFFF for a full bucket, and alias[j] = local index of the second   */
/* element.  A row whose weights sum to zero has no transition: all its     */
/* slots get thr = 0xFFFFFFFF and alias = -1, which the walk reads as a dead */
/* end.                                                                     */
/* ------------------------------------------------------------------------ */
int trwo_alias_build(int64_t n, const int32_t *row_ptr, const uint32_t *w,
                     uint32_t *thr, int32_t *alias) {
    int64_t dmax = 0;
    for (int64_t v = 0; v < n; v++) {
        int64_t d = (int64_t)row_ptr[v + 1] - row_ptr[v];
        if (d > dmax) dmax = d;
    }
    uint64_t *s = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(dmax + 1));
    int64_t *small = (int64_t *)malloc(sizeof(int64_t) * (size_t)(dmax + 1));
    int64_t *large = (int64_t *)malloc(sizeof(int64_t) * (size_t)(dmax + 1));
    if (!s || !small || !large) { free(s); free(small); free(large); return -1; }

    for (int64_t v = 0; v < n; v++) {
        int64_t off = row_ptr[v];
        int64_t d = (int64_t)row_ptr[v + 1] - off;
        if (d == 0) continue;
        uint64_t W = 0;
        for (int64_t i = 0; i < d; i++) W += w[off + i];
        if (W == 0) {
            for (int64_t i = 0; i < d; i++) { thr[off + i] = 0xFFFFFFFFu; alias[off + i] = -1; }
            continue;
        }
        int64_t ns = 0, nl = 0;
        for (int64_t i = 0; i < d; i++) {
            s[i] = (uint64_t)w[off + i] * (uint64_t)d;
            if (s[i] < W) small[ns++] = i; else large[nl++] = i;
        }
        while (ns > 0 && nl > 0) {
            int64_t l = small[--ns];
            int64_t g = large[nl - 1];
            /* bucket l: first = l with mass s[l], second = g */
            thr[off + l] = (uint32_t)(((unsigned __int128)s[l] << 32) / W);
            alias[off + l] = (int32_t)g;
            s[g] -= (W - s[l]);
            if (s[g] < W) { nl--; small[ns++] = g; }
        }
        while (nl > 0) {
            int64_t g = large[--nl];
            thr[off + g] = 0xFFFFFFFFu;
            alias[off + g] = (int32_t)g;
        }
        /* In exact arithmetic the small stack is empty here: the remaining
           columns hold (#remaining) * W in total and each is below W. */
        if (ns != 0) { free(s); free(small); free(large); return -2; }
    }
    free(s); free(small); free(large);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* ITS initialization [Sampling Methods, inverse transformation sampling]:  */
/* per vertex, the inclusive running sum of the weights, in 64-bit integers. */
/* ------------------------------------------------------------------------ */
int trwo_its_build(int64_t n, const int32_t *row_ptr, const uint32_t *w, uint64_t *prefix) {
    for (int64_t v = 0; v < n; v++) {
        uint64_t acc = 0;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            acc += w[e];
            prefix[e] = acc;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* REJ initialization [Sampling Methods, rejection sampling]: per vertex the  */
/* largest weight of its edges, p*_v (0 for a vertex without edges).        */
/* ------------------------------------------------------------------------ */
int trwo_rej_build(int64_t n, const int32_t *row_ptr, const uint32_t *w, uint32_t *pmax) {
    for (int64_t v = 0; v < n; v++) {
        uint32_t mx = 0;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++)
            if (w[e] > mx) mx = w[e];
        pmax[v] = mx;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Walk                                                                      */
/* ------------------------------------------------------------------------ */
enum { ORC_DEEPWALK = 0, ORC_PPR = 1, ORC_NODE2VEC = 2, ORC_METAPATH = 3 };
enum { ORC_NAIVE = 0, ORC_ALIAS = 1, ORC_ITS = 2, ORC_OREJ = 3, ORC_REJ = 4 };
enum { ORC_ST_LENGTH = 1, ORC_ST_STOPPED = 2, ORC_ST_DEAD_END = 3, ORC_ST_BAD_SOURCE = 4 };

/* Upper bound on O-REJ darts per move.  With every threshold >= 1 a dart is
   accepted with probability >= 2^-16, so 2^24 darts are exceeded with
   probability below e^-256; the last dart is then taken. */
#define ORC_OREJ_MAX_TRIALS (1u << 24)

/* The same cap for REJ darts.  A dart at the heaviest edge always hits, so
   the cap is reached with probability (1 - sum w / (d p*))^(2^24): below
   e^-65536 when weights differ by at most a factor 256. */
#define ORC_REJ_MAX_TRIALS (1u << 24)

typedef struct {
    uint32_t algo;
    uint32_t sampler;
    uint32_t max_len;          /* moves per query at most */
    uint32_t stop_q32;         /* PPR: stop after a move iff r2 < stop_q32 */
    uint32_t n2v_thr_q16[3];   /* Node2Vec: x == prev, x adjacent to prev, otherwise */
    uint32_t schema_len;       /* MetaPath */
    uint8_t  schema[16];
    uint64_t seed;
} trwo_params;

typedef struct {
    uint64_t moves;            /* successful moves */
    uint64_t philox_blocks;    /* Philox blocks drawn */
    uint64_t its_probes;       /* prefix entries read by ITS searches */
    uint64_t orej_trials;      /* O-REJ darts */
    uint64_t adjacency_probes; /* entries read by Node2Vec adjacency tests */
    uint64_t label_reads;      /* labels read by MetaPath */
    uint64_t rej_trials;       /* REJ darts */
} trwo_counters;

/* Is x in the sorted row [lo, hi) of col?  Textbook binary search. */
static int in_sorted_row(const int32_t *col, int64_t lo, int64_t hi, int32_t x, uint64_t *probes) {
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        (*probes)++;
        if (col[mid] == x) return 1;
        if (col[mid] < x) lo = mid + 1; else hi = mid;
    }
    return 0;
}

/* Smallest i in [0, d) with t < prefix[off + i]; prefix is non-decreasing. */
static int64_t its_search(const uint64_t *prefix, int64_t off, int64_t d, uint64_t t, uint64_t *probes) {
    int64_t lo = 0, hi = d - 1;        /* answer in [lo, hi]; prefix[off+d-1] = W > t */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        (*probes)++;
        if (t < prefix[off + mid]) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* The second-order factor of Node2Vec's transition equation, Q16: moving
   to x from cur, having come from prev, weighs thr[0] (the 1/p term) when x
   is prev, thr[1] (the 1 term) when x is a neighbour of prev, thr[2] (the
   1/q term) otherwise.  The first move (no prev) weighs 65536 everywhere. */
static uint32_t n2v_factor(const int32_t *row_ptr, const int32_t *col, const trwo_params *p,
                           uint32_t k, int32_t prev, int32_t x, uint64_t *probes) {
    if (k == 0) return 65536u;
    if (x == prev) return p->n2v_thr_q16[0];
    if (in_sorted_row(col, row_ptr[prev], row_ptr[prev + 1], x, probes)) return p->n2v_thr_q16[1];
    return p->n2v_thr_q16[2];
}

/* A uniform draw in [0, W) for dynamic ITS: floor(r0 * W / 2^32) while W fits
   32 bits, else the high 64 bits of the 64-bit word (r1:r0) times W. */
static uint64_t dynamic_its_draw(const uint32_t r[4], uint64_t W) {
    if (W < ((uint64_t)1 << 32)) return ((uint64_t)r[0] * W) >> 32;
    const uint64_t r64 = ((uint64_t)r[1] << 32) | r[0];
    return (uint64_t)(((unsigned __int128)r64 * W) >> 64);
}

/*
 * Run nq queries.  Query i starts at sources[i] and has id qids ? qids[i] : qid_base + i.
 * Its path goes to paths[i * path_stride + 0 .. lengths[i]]; status[i] says why it ended.
 * Tables: thr/alias for ALIAS, prefix for ITS, the weights w and p* for REJ;
 * label for MetaPath.  Node2Vec takes the sampler O-REJ (unweighted), REJ
 * (weighted: w and p*) or ITS (weights computed per step; no table).
 */
int trwo_walk(int64_t n, const int32_t *row_ptr, const int32_t *col,
              const uint32_t *thr, const int32_t *alias, const uint64_t *prefix,
              const uint32_t *w, const uint32_t *pmax,
              const uint8_t *label, const trwo_params *p,
              const int32_t *sources, int64_t nq, uint64_t qid_base, const uint64_t *qids,
              int32_t *paths, int64_t path_stride, uint32_t *lengths, uint8_t *status,
              trwo_counters *cnt) {
    trwo_counters local;
    memset(&local, 0, sizeof(local));
    for (int64_t i = 0; i < nq; i++) {
        const uint64_t qid = qids ? qids[i] : qid_base + (uint64_t)i;
        int32_t *path = paths + i * path_stride;
        const int32_t s = sources[i];
        if (s < 0 || (int64_t)s >= n) { lengths[i] = 0; status[i] = ORC_ST_BAD_SOURCE; continue; }
        int32_t cur = s, prev = -1;
        uint32_t k = 0;
        uint8_t st;
        path[0] = s;
        for (;;) {
            if (k == p->max_len) { st = ORC_ST_LENGTH; break; }
            const int64_t off = row_ptr[cur];
            const uint32_t d = (uint32_t)(row_ptr[cur + 1] - row_ptr[cur]);
            if (d == 0) { st = ORC_ST_DEAD_END; break; }
            uint32_t r[4];
            int32_t nxt = -1;
            if (p->algo == ORC_DEEPWALK || p->algo == ORC_PPR) {
                block(p->seed, qid, k, 0, r);
                local.philox_blocks++;
                if (p->sampler == ORC_NAIVE) {
                    nxt = col[off + index_of(r[0], d)];
                } else if (p->sampler == ORC_ALIAS) {
                    const uint32_t j = index_of(r[0], d);
                    const int32_t a = alias[off + j];
                    if (a < 0) { st = ORC_ST_DEAD_END; break; }
                    nxt = (r[1] < thr[off + j]) ? col[off + j] : col[off + a];
                } else if (p->sampler == ORC_REJ) {
                    /* darts (x, y): x a uniform edge slot, y uniform in
                       [0, p*); the dart hits iff y < w_x.  The block of the
                       hitting dart also gives the PPR stop coin. */
                    const uint32_t ps = pmax[cur];
                    if (ps == 0) { st = ORC_ST_DEAD_END; break; }
                    for (uint32_t t = 0;; t++) {
                        if (t > 0) { block(p->seed, qid, k, t, r); local.philox_blocks++; }
                        local.rej_trials++;
                        const uint32_t x = index_of(r[0], d);
                        const int hit = (uint64_t)r[1] * ps < ((uint64_t)w[off + x] << 32);
                        if (hit || t + 1 == ORC_REJ_MAX_TRIALS) { nxt = col[off + x]; break; }
                    }
                } else { /* ITS */
                    const uint64_t W = prefix[off + d - 1];
                    if (W == 0) { st = ORC_ST_DEAD_END; break; }
                    const uint64_t r64 = ((uint64_t)r[1] << 32) | r[0];
                    const uint64_t t = (uint64_t)(((unsigned __int128)r64 * W) >> 64);
                    nxt = col[off + its_search(prefix, off, d, t, &local.its_probes)];
                }
            } else if (p->algo == ORC_NODE2VEC && p->sampler == ORC_REJ) {
                /* Weighted Node2Vec by rejection: the transition weight of
                   edge x is w_x * a_x, bounded by p*_v * 65536 (p*_v the
                   row's largest weight, a_x <= 65536).  Darts (x, y): x a
                   uniform slot, y uniform in [0, p*_v * 65536); hit iff
                   y < w_x * a_x, i.e. r1 * p*_v < w_x * a_x * 2^16. */
                const uint32_t ps = pmax[cur];
                if (ps == 0) { st = ORC_ST_DEAD_END; break; }
                for (uint32_t t = 0;; t++) {
                    block(p->seed, qid, k, t, r);
                    local.philox_blocks++;
                    local.orej_trials++;
                    const uint32_t j = index_of(r[0], d);
                    const int32_t x = col[off + j];
                    const uint64_t a = n2v_factor(row_ptr, col, p, k, prev, x, &local.adjacency_probes);
                    const int hit = (uint64_t)r[1] * ps < (((uint64_t)w[off + j] * a) << 16);
                    if (hit || t + 1 == ORC_OREJ_MAX_TRIALS) { nxt = x; break; }
                }
            } else if (p->algo == ORC_NODE2VEC && p->sampler == ORC_ITS) {
                /* Node2Vec by ITS over weights computed at this step: each
                   edge of the row weighs its second-order factor a_x; the
                   move takes the first edge whose running sum exceeds a
                   uniform draw in [0, W), W the row's total. */
                uint64_t W = 0;
                for (uint32_t i2 = 0; i2 < d; i2++)
                    W += n2v_factor(row_ptr, col, p, k, prev, col[off + i2], &local.adjacency_probes);
                if (W == 0) { st = ORC_ST_DEAD_END; break; }
                block(p->seed, qid, k, 0, r);
                local.philox_blocks++;
                const uint64_t t = dynamic_its_draw(r, W);
                uint64_t acc = 0;
                for (uint32_t i2 = 0; i2 < d; i2++) {
                    acc += n2v_factor(row_ptr, col, p, k, prev, col[off + i2], &local.adjacency_probes);
                    local.its_probes++;
                    if (t < acc) { nxt = col[off + i2]; break; }
                }
            } else if (p->algo == ORC_NODE2VEC) {
                /* O-REJ: darts (x, y) until y falls under p(x) / p*; the
                   Q16 thresholds are p(e) / p* scaled by 2^16. */
                for (uint32_t t = 0;; t++) {
                    block(p->seed, qid, k, t, r);
                    local.philox_blocks++;
                    local.orej_trials++;
                    const int32_t x = col[off + index_of(r[0], d)];
                    if (k == 0 || t + 1 == ORC_OREJ_MAX_TRIALS) { nxt = x; break; }
                    uint32_t th;
                    if (x == prev) th = p->n2v_thr_q16[0];
                    else if (in_sorted_row(col, row_ptr[prev], row_ptr[prev + 1], x, &local.adjacency_probes))
                        th = p->n2v_thr_q16[1];
                    else th = p->n2v_thr_q16[2];
                    if ((r[1] >> 16) < th) { nxt = x; break; }
                }
            } else { /* METAPATH: only edges whose label is the schema's label for this move */
                const uint8_t want = p->schema[k % p->schema_len];
                uint32_t m = 0;
                for (uint32_t i2 = 0; i2 < d; i2++) m += (label[off + i2] == want);
                local.label_reads += d;
                if (m == 0) { st = ORC_ST_DEAD_END; break; }
                block(p->seed, qid, k, 0, r);
                local.philox_blocks++;
                const uint32_t j = index_of(r[0], m);
                uint32_t seen = 0;
                for (uint32_t i2 = 0; i2 < d; i2++) {
                    if (label[off + i2] == want) {
                        if (seen == j) { nxt = col[off + i2]; break; }
                        seen++;
                    }
                }
            }
            path[k + 1] = nxt;
            prev = cur;
            cur = nxt;
            k++;
            local.moves++;
            if (p->algo == ORC_PPR && r[2] < p->stop_q32) { st = ORC_ST_STOPPED; break; }
        }
        lengths[i] = k;
        status[i] = st;
    }
    if (cnt) {
        cnt->moves += local.moves;
        cnt->philox_blocks += local.philox_blocks;
        cnt->its_probes += local.its_probes;
        cnt->orej_trials += local.orej_trials;
        cnt->adjacency_probes += local.adjacency_probes;
        cnt->label_reads += local.label_reads;
        cnt->rej_trials += local.rej_trials;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* PPR estimate [Random Walk based Algorithms, PPR]: the score of v' for a   */
/* source is the share of that source's queries whose walk ends at v'.       */
/* Query i belongs to group i / group (every query to group 0 when group is  */
/* 0); counts[g * n + v] is increased once for each query of group g whose   */
/* path ends at v, i.e. paths[i * stride + lengths[i]] == v.  Queries with a */
/* bad source, and paths whose end lies outside the row or outside [0, n),   */
/* are skipped; their number is returned.                                    */
/* ------------------------------------------------------------------------ */
int64_t trwo_end_counts(int64_t n, const int32_t *paths, int64_t stride, const uint32_t *lengths,
                        const uint8_t *status, int64_t nq, int64_t group, uint32_t *counts) {
    int64_t skipped = 0;
    for (int64_t i = 0; i < nq; i++) {
        if (status[i] == ORC_ST_BAD_SOURCE || (int64_t)lengths[i] >= stride) { skipped++; continue; }
        const int32_t v = paths[i * stride + lengths[i]];
        if (v < 0 || (int64_t)v >= n) { skipped++; continue; }
        const int64_t g = group > 0 ? i / group : 0;
        counts[g * n + v]++;
    }
    return skipped;
}

/* The k highest counts, larger count first and the smaller vertex id first   */
/* among equal counts: sort all (count, id) pairs in that order and take k.   */
typedef struct { uint32_t count; int32_t id; } orc_scored;

static int by_score(const void *a, const void *b) {
    const orc_scored *x = (const orc_scored *)a, *y = (const orc_scored *)b;
    if (x->count != y->count) return x->count > y->count ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

int trwo_topk(int64_t n, const uint32_t *counts, int64_t k, int32_t *ids, uint32_t *vals) {
    if (k < 0 || k > n) return -1;
    orc_scored *all = (orc_scored *)malloc(sizeof(orc_scored) * (size_t)(n > 0 ? n : 1));
    if (!all) return -2;
    for (int64_t v = 0; v < n; v++) { all[v].count = counts[v]; all[v].id = (int32_t)v; }
    qsort(all, (size_t)n, sizeof(orc_scored), by_score);
    for (int64_t i = 0; i < k; i++) { ids[i] = all[i].id; vals[i] = all[i].count; }
    free(all);
    return 0;
}
