/*
 * trw.h — C ABI of the MI355X random-walk engine (libtrw.so).
 *
 * The engine runs the step of ThunderRW's method (Sun et al., "ThunderRW: An
 * In-Memory Graph Random Walk Engine", VLDB 2021) over many independent
 * random-walk queries on one GPU: each step gathers the current vertex's
 * neighbours and transition weights, samples the next vertex and updates the
 * walker (Step-centric Programming: the Gather-Move-Update framework).  The
 * calls follow the paper's problem statement: input a graph and a set of
 * queries, output each query's walk sequence (Introduction, execution
 * paradigm; Other Implementation Details: graph storage, walker management,
 * input and output).
 *
 * Conventions
 *  - Every call returns trw_status (TRW_OK = 0).  Nothing throws across the
 *    ABI.  A failing call leaves its outputs untouched and records a message
 *    that trw_last_error() returns (per thread).
 *  - Device pointers ("d_" prefix) are HIP device memory owned by the caller.
 *    The library allocates no device memory on these paths: it reports the
 *    sizes it needs (trw_table_bytes, trw_walk_workspace_bytes) and the
 *    caller passes buffers.  Handles borrow the caller's buffers; keep them
 *    alive until the handle is destroyed.
 *  - Device work is asynchronous on the caller's stream (a hipStream_t passed
 *    as trw_stream_t; NULL = the null stream) unless a call says it
 *    synchronises.  Host pointers are read before the call returns.
 *  - Handles are not thread-safe.
 *
 * Random contract (the paper samples with real uniforms; this engine fixes an
 * integer contract so that any run is reproducible bit for bit):
 *   block(k, t) = Philox4x32-10(counter = (k, t, qid_lo, qid_hi),
 *                               key = (seed_lo, seed_hi)) -> words r0..r3
 * where k is the move number (0-based), t the dart number (O-REJ) and qid the
 * query id.  A query's walk depends only on (graph, params, seed, qid,
 * source), never on batch composition, launch shape or tuning.
 */
#ifndef TRW_H
#define TRW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TRW_ABI_VERSION 1u

typedef void *trw_stream_t;          /* hipStream_t */

typedef enum {
    TRW_OK = 0,
    TRW_E_INVALID = 1,       /* bad argument, size or missing input */
    TRW_E_UNSUPPORTED = 2,   /* (algorithm, sampler) pair not provided */
    TRW_E_DEVICE = 3,        /* a HIP runtime call failed */
    TRW_E_NOMEM_BUDGET = 4,  /* serving: request can never fit the memory budget */
    TRW_E_BUSY = 5,          /* serving: no slot free right now (retry) */
    TRW_E_TIMEOUT = 6,       /* serving: poll timed out with nothing complete */
    TRW_E_CANCELLED = 7      /* serving: request was cancelled */
} trw_status;

/* Message of the last failing call on this thread ("" if none).  Owned by the library. */
const char *trw_last_error(void);
/* TRW_ABI_VERSION of the loaded library. */
uint32_t trw_abi_version(void);

/* ------------------------------------------------------------------------ */
/* Graph (Preliminary: directed G = (V, E), an undirected edge as two        */
/* directed edges; Other Implementation Details, graph storage: CSR with     */
/* per-edge weight and label arrays).                                        */
/* ------------------------------------------------------------------------ */
typedef struct trw_graph_s *trw_graph;

enum { TRW_G_SYMMETRIC = 1 };

/*
 * Memory.  Every array and buffer passed to the library is addressed by the
 * device.  Graph arrays and table / index buffers may be device memory or
 * pinned host memory mapped for the device (hipHostMalloc): a graph and
 * tables larger than HBM stay in host memory and every move reads them over
 * the host link (slower, identical results).  The edge index is the
 * exception: its build uses device atomics and must be in device memory.
 * Walk outputs, counts and workspaces are device memory.
 */

/*
 * Wrap a CSR graph the device can read (device memory, or pinned host memory).
 *   n          vertices, 1 <= n < 2^31
 *   m          directed edges, 0 <= m < 2^31
 *   d_row_ptr  int32[n+1]: row v is col[row_ptr[v] .. row_ptr[v+1])
 *   d_col      int32[m]: destinations, each row sorted ascending without
 *              duplicates (Node2Vec's adjacency test is a binary search)
 *   d_weight   uint32[m] or NULL: static transition weights (ALIAS, ITS)
 *   d_label    uint8[m] or NULL: edge labels (MetaPath)
 *   flags      TRW_G_SYMMETRIC if every edge has its reverse; Node2Vec then tests
 *              adjacency in the shorter of the two rows.  Must be true when
 *              set (trw_graph_validate checks it)
 * Borrows the arrays; does not read them (see trw_graph_validate).
 * Errors: TRW_E_INVALID for sizes out of range or NULL row_ptr/col.
 */
trw_status trw_graph_create(int64_t n, int64_t m, const int32_t *d_row_ptr, const int32_t *d_col,
                            const uint32_t *d_weight, const uint8_t *d_label, uint32_t flags,
                            trw_graph *out);

/*
 * O(n + m) check on the device: row_ptr[0] == 0, row_ptr non-decreasing,
 * row_ptr[n] == m, every col in [0, n), rows strictly ascending; and, for a
 * graph created with TRW_G_SYMMETRIC, O(m log d) check that every edge has
 * its reverse.
 * d_ws: device scratch of at least 64 bytes, 8-byte aligned.  Synchronises the stream and
 * writes the number of violations to *n_bad.  Returns TRW_E_INVALID if
 * *n_bad > 0.
 */
trw_status trw_graph_validate(trw_graph g, void *d_ws, size_t ws_bytes, trw_stream_t stream,
                              uint64_t *n_bad);

trw_status trw_graph_destroy(trw_graph g);

/*
 * Count the query sources outside [0, n).  A query starts at a vertex of the
 * graph (Preliminary: a walk is a sequence of vertices of G; Other
 * Implementation Details, input: the caller names each query's source).
 * trw_walk does not fail for such sources: each gets status BAD_SOURCE and
 * length 0, asynchronously.  A caller who wants a hard error runs this first.
 *   d_sources  int32[nq], device memory or pinned host memory
 *   d_ws       device scratch of at least 8 bytes, 8-byte aligned (cleared by
 *              the call's own kernel)
 * Synchronises the stream, writes the count to *n_bad and returns
 * TRW_E_INVALID if it is not 0.  Errors: TRW_E_INVALID for a NULL graph or
 * n_bad, NULL sources with nq > 0, nq >= 2^32, or a short or misaligned
 * workspace (*n_bad untouched); TRW_E_DEVICE if a HIP call fails.
 */
trw_status trw_validate_sources(trw_graph g, const int32_t *d_sources, uint64_t nq, void *d_ws, size_t ws_bytes,
                                trw_stream_t stream, uint64_t *n_bad);

/* ------------------------------------------------------------------------ */
/* Sampling tables (Sampling Methods; preprocessing algorithm for static      */
/* walks: one table C_v per vertex, built once before the queries run).      */
/* ------------------------------------------------------------------------ */
typedef enum {
    TRW_S_NAIVE = 0,   /* uniform index; no table */
    TRW_S_ALIAS = 1,   /* Walker alias table, integer Vose construction */
    TRW_S_ITS = 2,     /* inverse transform: inclusive uint64 prefix + binary search */
    TRW_S_OREJ = 3,    /* rejection with a user bound p*; no table (Node2Vec) */
    TRW_S_REJ = 4      /* rejection with p*_v = the row's largest weight (per-vertex table) */
} trw_sampler;

typedef struct trw_table_s *trw_table;

/* Bytes of device memory the table for `sampler` needs: ALIAS 32*m; ITS 8*m and
 * 32*m, each rounded up to 256, plus 8*n; REJ 32*m rounded up to 256, plus 4*n. */
trw_status trw_table_bytes(trw_graph g, uint32_t sampler, size_t *bytes);

/*
 * Build the per-vertex table for `sampler` from the graph's weights into
 * d_buf (caller-owned, >= trw_table_bytes, 32-byte aligned; 256-byte aligned
 * for ITS, whose search reads whole 64-byte blocks of the prefix), asynchronously.
 * The graph must be valid (trw_graph_validate); rows are read as given.
 * Layout (per directed edge slot e of row v, in CSR order):
 *   ALIAS: 8 x uint32 {thr, dst_first, dst_second, 0,
 *                      row_off(dst_first), deg(dst_first), row_off(dst_second), deg(dst_second)}.
 *          Column j of row v is the bucket (first = col[off+j], second =
 *          col[off+alias_j]); it picks the first iff r1 < thr.  thr =
 *          floor(s_j * 2^32 / W) from Vose's worklist method in exact
 *          integers (W = sum of the row's weights, s_j = w_j * d after the
 *          transfers), 0xFFFFFFFF for a full bucket.  The row ranges of both
 *          candidates ride along so that a move needs one 32-byte read.
 *          A row whose weights sum to 0 holds {0xFFFFFFFF, -1, -1, 0, 0, 0,
 *          0, 0}: a walk that reaches it ends as a dead end.
 *   ITS:   uint64 prefix[e] = sum of w over row v up to and including e; then,
 *          at byte 8*m rounded up to 256, 8 x uint32 per edge slot {col[e],
 *          row_off(col[e]), deg(col[e]), 0, W lo, W hi, 0, 0} with W the
 *          weight sum of col[e]'s row; then, at 32*m further (rounded up to
 *          256), uint64 W[n].  A move searches the prefix and reads the
 *          chosen slot's record, which carries the next row and its total.
 *   REJ:   (Sampling Methods, rejection sampling: initialization finds
 *          p*_v = max weight of v's row; generation throws darts (x, y) with x
 *          uniform in [0, d_v), y uniform in [0, p*_v) until y < w_x.)
 *          8 x uint32 per edge slot {w[e], col[e], row_off(col[e]), deg(col[e]),
 *          p*(col[e]), 0, 0, 0}, then, at byte 32*m rounded up to 256,
 *          uint32 p*[n] (0 for a vertex without edges, or whose weights are
 *          all 0: a walk that reaches it ends as a dead end).  A dart is one
 *          32-byte read that also carries everything the next move needs.
 * Errors: TRW_E_INVALID if the graph has no weights, bytes is too small or the
 * buffer is misaligned; TRW_E_UNSUPPORTED for NAIVE / OREJ (no table).
 */
trw_status trw_table_build(trw_graph g, uint32_t sampler, void *d_buf, size_t bytes,
                           trw_stream_t stream, trw_table *out);

trw_status trw_table_destroy(trw_table t);

/*
 * Adjacency index (optional, for NAIVE and OREJ walks).  Every edge slot e
 * holds uint32x4 {col[e], row_off(col[e]), deg(col[e]), 0}, so a move that
 * picks a slot learns the next vertex's row range with the same read, and
 * Node2Vec darts learn the candidate's degree.  Results are identical with
 * and without it.  16*m bytes, 16-byte aligned.
 */
trw_status trw_adjacency_index_bytes(trw_graph g, size_t *bytes);
trw_status trw_adjacency_index_build(trw_graph g, void *d_buf, size_t bytes, trw_stream_t stream,
                                     trw_table *out);

/*
 * Edge index (optional, for NAIVE and OREJ walks and the server): the
 * adjacency index above, then a hash set of every edge (u, v).  Node2Vec's
 * acceptance test asks whether a dart's vertex x is a neighbour of the
 * previous vertex (the Node2Vec transition equation); the paper answers it by
 * binary search in the sorted row, O(log d) dependent reads.  With the edge
 * index it is one probe sequence of the hash set, usually one cache line.
 * Membership is exact, so results are identical with and without it.
 * d_buf must be device memory (the set is filled with device atomics):
 * TRW_E_UNSUPPORTED for pinned host memory.
 * Layout in d_buf (256-byte aligned): uint32x4 records[m] padded to 256 bytes,
 * then uint64 keys[S], S = the smallest power of two >= max(64, 2m), key
 * u << 32 | v, empty slots all ones, linear probing from SplitMix64's
 * finalizer of the key.  Bytes: 16m rounded up to 256, plus 8S.
 */
trw_status trw_edge_index_bytes(trw_graph g, size_t *bytes);
trw_status trw_edge_index_build(trw_graph g, void *d_buf, size_t bytes, trw_stream_t stream, trw_table *out);

/*
 * MetaPath label index (optional).  A MetaPath move only considers the edges
 * of the current vertex whose label equals the schema's label for that move
 * (Random Walk based Algorithms, MetaPath); without an index every move
 * counts the matching labels of the row (the dynamic Gather).  The index
 * stores every row stably sorted by label and, per vertex, where each label's
 * run starts, so a move reads two offsets and one destination.  It selects
 * the same edge as the scan (the j-th match in CSR order is the j-th entry of
 * the label's run), so results are identical with and without it.
 *   n_labels  L in 1..64; edges with labels >= L are left out of the index
 *             and schemas used with it must have every label < L
 * Layout in d_buf (256-byte aligned): int32 loff[n][L+1] (absolute offsets
 * into lcol; loff[v][L] = end of v's indexed edges), padded to 256 bytes,
 * then int32 lcol[m] (-1 in the slots of edges left out).  For L <= 6, then,
 * padded to 256 bytes, 8 x int32 per slot e {lcol[e], loff[lcol[e]][0..L],
 * 0...}: a persistent walk's move reads one such entry, which also holds the
 * next move's label run.  Bytes: 4n(L+1) and 4m, each rounded up to 256,
 * plus 32m when L <= 6.
 */
trw_status trw_label_index_bytes(trw_graph g, uint32_t n_labels, size_t *bytes);
trw_status trw_label_index_build(trw_graph g, uint32_t n_labels, void *d_buf, size_t bytes,
                                 trw_stream_t stream, trw_table *out);

/* ------------------------------------------------------------------------ */
/* Walks                                                                     */
/* ------------------------------------------------------------------------ */
typedef enum {
    TRW_A_DEEPWALK = 0,   /* fixed length (Random Walk based Algorithms: DeepWalk) */
    TRW_A_PPR = 1,        /* stop with a fixed probability after each move (PPR) */
    TRW_A_NODE2VEC = 2,   /* second-order: the Node2Vec transition equation */
    TRW_A_METAPATH = 3    /* only edges whose label matches the schema (MetaPath) */
} trw_algo;

typedef enum {
    TRW_ST_LENGTH = 1,        /* made max_len moves */
    TRW_ST_STOPPED = 2,       /* PPR stop coin after a move */
    TRW_ST_DEAD_END = 3,      /* no eligible edge at the current vertex */
    TRW_ST_BAD_SOURCE = 4     /* source outside [0, n) */
} trw_walk_status;

typedef struct {
    uint32_t algo;             /* trw_algo */
    uint32_t sampler;          /* DEEPWALK/PPR: NAIVE, ALIAS, ITS or REJ; NODE2VEC: OREJ;
                                  METAPATH: ITS.  REJ darts of move k are Philox blocks
                                  (k, t = 0, 1, ...): x = high half of r0 * d, hit iff
                                  r1 * p*_v < w_x * 2^32; PPR's stop coin is r2 of the
                                  block of the hitting dart */
    uint32_t max_len;          /* moves per query, 1..65535; a path holds max_len+1 vertices */
    uint32_t stop_q32;         /* PPR: stop after a move iff r2 < stop_q32 (0.2 -> 858993459) */
    uint32_t n2v_thr_q16[3];   /* NODE2VEC: accept a dart iff (r1 >> 16) < thr[c], c = 0 when
                                  the candidate is the previous vertex, 1 when it is adjacent to
                                  it, 2 otherwise; thr = round(2^16 p(e) / p*), in [1, 65536] */
    uint32_t schema_len;       /* METAPATH: 1..16; move k uses label schema[k % schema_len] */
    uint8_t schema[16];
    uint64_t seed;             /* Philox key */
} trw_walk_params;

typedef enum {
    TRW_M_PER_STEP = 0,        /* one launch per move over the live walkers (bulk-synchronous) */
    TRW_M_PERSISTENT = 1       /* one launch; lanes refill from a device queue as walks end */
} trw_mode;

/* Launch and scheduling knobs.  Any field 0 = library default.  Results never depend on them. */
typedef struct {
    uint32_t walkers_per_lane;  /* persistent: 1, 2 or 4 walkers interleaved per lane */
    uint32_t block_threads;     /* 64..1024, multiple of 64 */
    uint32_t blocks_per_cu;     /* persistent grid = CUs * blocks_per_cu */
    uint32_t queue_chunk;       /* persistent: queries claimed per wave per queue access */
    uint32_t coop_degree;       /* MetaPath without an index: rows at least this long are
                                   scanned by the whole wave, shorter ones by their lane */
    uint32_t no_lds_graph;      /* persistent NAIVE DeepWalk / PPR on a graph whose CSR fits one
                                   workgroup's LDS (4(n+1) + 2m bytes, rounded to 16 each, within
                                   the device's per-workgroup limit, n <= 65536): the graph is
                                   copied into LDS and walked there, with its own launch shape
                                   (the fields above do not apply).  Nonzero: never. */
    uint32_t its_gallop_degree; /* ITS DeepWalk / PPR: rows of at least this many slots start
                                   the search at the slot the random fraction points to and
                                   gallop from it; shorter rows bisect the whole row.  Default 1
                                   (every row searches from its guess) */
    uint32_t n2v_search_degree; /* Node2Vec with an edge index: when the previous vertex has at
                                   most this many edges, the adjacency test searches its sorted
                                   row instead of probing the hash set.  Default: never */
} trw_tuning;

/* Workspace bytes trw_walk needs for nq queries in `mode`. */
trw_status trw_walk_workspace_bytes(trw_graph g, const trw_walk_params *p, uint64_t nq,
                                    uint32_t mode, size_t *bytes);

/* The library's default tuning for this graph, params and mode (what trw_walk
 * uses when given no tuning).  For METAPATH it is the default without a label
 * index; with one, trw_walk runs 2 blocks per CU with 2 walkers per lane. */
trw_status trw_default_tuning(trw_graph g, const trw_walk_params *p, uint32_t mode, trw_tuning *out);

/*
 * Run nq queries, query i starting at d_sources[i] with id qid_base + i.
 *   table       ALIAS/ITS/REJ table built for p->sampler; for NAIVE and OREJ NULL,
 *               an adjacency index or an edge index; for METAPATH NULL (scan
 *               rows) or a label index
 *   d_paths     int32, row i at d_paths + i*path_stride, path_stride >= max_len+1:
 *               paths[i][0] = source, paths[i][1..lengths[i]] = the moves;
 *               entries beyond lengths[i] are left unspecified
 *   d_lengths   uint32[nq]: moves made
 *   d_status    uint8[nq]: trw_walk_status
 *   tuning      NULL = trw_default_tuning
 *   d_ws        workspace of >= trw_walk_workspace_bytes, 256-byte aligned
 * Asynchronous on `stream`.  Sources outside [0, n) get status BAD_SOURCE and
 * length 0 (path row untouched); they are not an error of the call.
 * A persistent NAIVE DeepWalk or PPR walk on a graph whose CSR fits one
 * workgroup's LDS (see trw_tuning.no_lds_graph) copies the graph into LDS and
 * walks there; the results are the same bits either way.
 * Errors: TRW_E_UNSUPPORTED for an (algo, sampler) pair outside the list
 * above; TRW_E_INVALID for max_len outside 1..65535, thresholds > 65536 or
 * 0, schema_len outside 1..16, a missing or mismatched table, missing labels
 * for METAPATH, path_stride < max_len+1, a short or misaligned workspace, or
 * nq >= 2^32.
 */
trw_status trw_walk(trw_graph g, trw_table table, const trw_walk_params *p,
                    const int32_t *d_sources, uint64_t nq, uint64_t qid_base,
                    int32_t *d_paths, uint64_t path_stride, uint32_t *d_lengths, uint8_t *d_status,
                    uint32_t mode, const trw_tuning *tuning, void *d_ws, size_t ws_bytes,
                    trw_stream_t stream);

/*
 * trw_walk without a workspace argument, for callers that cannot allocate
 * device memory (code under graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The workspace trw_walk would take lives in a
 * device array inside the library, TRW_NOALLOC_SCRATCH_BYTES per GPU, held
 * until the process ends; the call itself allocates nothing.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (on different
 * streams, or from several threads) race and must not be issued.  The array
 * is cleared by the call's own kernels wherever a walk needs zeros.
 * Limit: trw_walk_workspace_bytes(g, p, nq, mode) <= TRW_NOALLOC_SCRATCH_BYTES
 * (persistent: any nq; per step: 32 bytes per query plus 4 * (max_len + 2),
 * each rounded up to 256), else TRW_E_INVALID before any device work.  Other
 * arguments, outputs and errors as trw_walk.
 */
#define TRW_NOALLOC_SCRATCH_BYTES (8u << 20)
trw_status trw_walk_noalloc(trw_graph g, trw_table table, const trw_walk_params *p,
                            const int32_t *d_sources, uint64_t nq, uint64_t qid_base,
                            int32_t *d_paths, uint64_t path_stride, uint32_t *d_lengths,
                            uint8_t *d_status, uint32_t mode, const trw_tuning *tuning,
                            trw_stream_t stream);

/*
 * Pick a tuning by pre-executing short walks (the paper tunes its ring sizes
 * the same way: Ring Size Tuning).  Runs up to `budget` (0 = all) candidate
 * launches of `nq` queries (a sample, length-capped at p->max_len) from
 * d_sources in `mode`, timing each with HIP events, and writes the fastest to
 * *out.  Candidates: the default tuning first, then walkers per lane x blocks
 * per CU x queue chunk (persistent) or blocks per CU x block size (per step),
 * and for METAPATH without a label index the wave-scan degree; then, with the
 * best of those, the walk's degree threshold if it has one (ITS DeepWalk /
 * PPR: its_gallop_degree 8, 64, 512; Node2Vec with an edge index:
 * n2v_search_degree 4, 16, 64).  The default is
 * kept unless a candidate is at least 3% faster, first in the scan and again
 * in five alternating timings of the two (medians).  Pass the whole batch when
 * a launch of it is short; a sample otherwise.  d_paths, d_lengths,
 * d_status and d_ws are scratch of the sizes trw_walk needs for nq queries.
 * Synchronises the stream.  Errors as trw_walk.
 */
trw_status trw_autotune(trw_graph g, trw_table table, const trw_walk_params *p,
                        const int32_t *d_sources, uint64_t nq, int32_t *d_paths,
                        uint64_t path_stride, uint32_t *d_lengths, uint8_t *d_status,
                        uint32_t mode, uint32_t budget, void *d_ws, size_t ws_bytes,
                        trw_stream_t stream, trw_tuning *out, float *best_ms);

/* ------------------------------------------------------------------------ */
/* Streamed output (Implementation details, input and output: the engine     */
/* fills one buffer while the other is written out).  The batch runs in      */
/* chunks; each chunk's paths are packed on the device, copied by DMA into   */
/* one of two pinned host buffers and handed to the caller while the next    */
/* chunk walks, so output never needs nq * (max_len + 1) entries of memory.  */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t qid_base;         /* id of the chunk's first query */
    uint32_t nq;               /* queries in the chunk */
    uint32_t reserved;
    const uint32_t *lengths;   /* [nq] moves made */
    const uint8_t *status;     /* [nq] trw_walk_status */
    const uint64_t *offsets;   /* [nq + 1]: query i's path is entries[offsets[i] .. offsets[i+1]) */
    const int32_t *entries;    /* packed paths (source first); a bad source has an empty path */
} trw_chunk;

/* Called on the calling thread once per chunk, in order; the chunk's arrays
 * are valid until it returns.  Nonzero return: stop the stream. */
typedef int (*trw_chunk_fn)(void *user, const trw_chunk *chunk);

/* A trw_chunk_fn that appends each chunk to a file (the paper's dump of the
 * output to disk while the engine fills the other buffer: Other
 * Implementation Details, input and output).  user: pointer to an open file
 * descriptor (int).  Record per chunk, native byte order: {qid_base u64,
 * nq u32, 0 u32}, lengths u32[nq], status u8[nq] zero-padded to a multiple of
 * 8 bytes, offsets u64[nq + 1], entries i32[offsets[nq]].  Returns nonzero
 * (stopping the stream) when a write fails. */
int trw_chunk_to_fd(void *user, const trw_chunk *chunk);

/* Device workspace and pinned host bytes trw_walk_stream needs for chunks of
 * chunk_queries queries (two chunk sets each, plus the walk's workspace). */
trw_status trw_walk_stream_bytes(trw_graph g, const trw_walk_params *p, uint32_t chunk_queries,
                                 size_t *device_bytes, size_t *host_bytes);

/*
 * Run nq queries like trw_walk (persistent schedule, query i has id
 * qid_base + i, the same paths), chunk_queries at a time, and call fn for
 * each chunk with its packed output in host memory.  Synchronous: returns
 * when every chunk was delivered, fn stopped the stream (TRW_E_CANCELLED), or
 * a device error occurred; nothing is in flight on the buffers on return.
 *   d_ws        device workspace, >= device_bytes, 256-byte aligned
 *   h_pinned    host memory from hipHostMalloc (pinned), >= host_bytes,
 *               256-byte aligned
 * The walk and packing run on `stream`; the copies run on a stream of the
 * library's own.  Errors as trw_walk, and TRW_E_INVALID for chunk_queries 0,
 * a NULL fn or a short or misaligned buffer.
 */
trw_status trw_walk_stream(trw_graph g, trw_table table, const trw_walk_params *p,
                           const int32_t *d_sources, uint64_t nq, uint64_t qid_base, uint32_t chunk_queries,
                           const trw_tuning *tuning, void *d_ws, size_t d_ws_bytes, void *h_pinned,
                           size_t h_bytes, trw_chunk_fn fn, void *user, trw_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Graphs on disk (Future Extension: a graph too large for memory is hosted   */
/* on disk; Related Work: the I/O-efficient single-machine scheme that splits */
/* the graph into partitions, loads the partition holding the most queries,   */
/* runs each query there until it ends or leaves, and repeats).  Here the     */
/* partitions are vertex ranges of the CSR file, up to `slots` of them        */
/* resident on the device at once (walks cross between resident ones in      */
/* place), each partition's sampling table built on the device at its load,  */
/* and the walks are those trw_walk gives on the whole graph.                 */
/* ------------------------------------------------------------------------ */
/*
 * CSR file, native byte order:
 *   char   magic[8] = "TRWCSR1" (with its NUL)
 *   uint64 n, m, flags          flags bit 0: weights present, bit 1: labels present
 *   int64  row_ptr[n + 1]       row_ptr[0] = 0, non-decreasing, row_ptr[n] = m
 *   int32  col[m]               in [0, n)
 *   uint32 weight[m]            if flags bit 0
 *   uint8  label[m]             if flags bit 1
 * 1 <= n < 2^31.  m may exceed 2^31: only a partition's edges (fewer than 2^31)
 * are ever in device memory.
 */
typedef struct trw_disk_graph_s *trw_disk_graph;

enum { TRW_DISK_WEIGHTS = 1, TRW_DISK_LABELS = 2 };

/* Write a CSR file from host arrays (weight, label: NULL when absent).
 * TRW_E_INVALID for sizes out of range or a failed write. */
trw_status trw_disk_graph_write(const char *path, int64_t n, int64_t m, const int64_t *row_ptr,
                                const int32_t *col, const uint32_t *weight, const uint8_t *label);

/*
 * Open a CSR file and split its vertices into consecutive ranges of at most
 * part_edges edges each (a row longer than that gets a range of its own;
 * part_edges 0: 2^31 - 1).  Reads the header and row_ptr, which stay in host
 * memory (8(n + 1) bytes); the edges are read at each load.  Errors:
 * TRW_E_INVALID for a file that cannot be read, a bad magic, flags or size, a
 * row_ptr that breaks the rules above, a row of 2^31 edges or more, or
 * part_edges >= 2^31.
 */
trw_status trw_disk_graph_open(const char *path, uint64_t part_edges, trw_disk_graph *out);
trw_status trw_disk_graph_info(trw_disk_graph g, uint64_t *n, uint64_t *m, uint32_t *flags, uint32_t *parts);
/* Partition i: vertices [v_begin, v_end) and their edges [e_begin, e_end). */
trw_status trw_disk_graph_partition(trw_disk_graph g, uint32_t i, int64_t *v_begin, int64_t *v_end,
                                    int64_t *e_begin, int64_t *e_end);
trw_status trw_disk_graph_close(trw_disk_graph g);

typedef struct {
    uint64_t runs;             /* rounds: each walks every query waiting in a resident partition */
    uint64_t loads;            /* partitions read and copied to the device */
    uint64_t bytes_read;       /* file bytes read */
    uint64_t read_ns;          /* host time spent reading the file */
    uint64_t total_ns;         /* host time of the whole call */
} trw_disk_walk_stats;

/* Device workspace and pinned host bytes trw_disk_walk needs for nq queries
 * with `slots` partitions resident at once (1 .. the partition count; 0 counts
 * as 1, more than the partitions as all of them; Node2Vec takes at least 2).  Per slot: 4(n + 1) bytes of
 * row offsets plus the largest partition's edges (4 B each, 4 more for
 * weights, 1 for labels) and table (ALIAS 32 B per edge; ITS 40 B per edge +
 * 8n; REJ 32 B per edge + 4n). */
trw_status trw_disk_walk_bytes(trw_disk_graph g, const trw_walk_params *p, uint64_t nq, uint32_t slots,
                               size_t *device_bytes, size_t *host_bytes);

/*
 * Run nq queries over the file's graph: the same paths, lengths and status as
 * trw_walk over the whole graph (query i has id qid_base + i).  DeepWalk and
 * PPR with NAIVE, ALIAS, ITS or REJ, MetaPath, and Node2Vec with O-REJ.  A
 * query waits under its partition; a Node2Vec query, whose acceptance test
 * searches the previous vertex's row, under the pair of its current and
 * previous vertices' partitions (so at most 1024 partitions, and rows sorted
 * as trw_graph_validate wants them).  Until every query ends: the queries
 * waiting under resident partitions move until they end or need a partition
 * that is not resident; when none waits there, the partitions of the key
 * holding the most queries (the lowest index among equals) are loaded (edges
 * read through h_pinned, copied to the device, table built there) into free
 * slots or those whose partitions ran longest ago.
 *   d_sources, d_paths, path_stride, d_lengths, d_status   as trw_walk
 *   slots       partitions resident at once, as trw_disk_walk_bytes
 *   d_ws        device workspace, >= device_bytes, 256-byte aligned
 *   h_pinned    host memory from hipHostMalloc, >= host_bytes, 256-byte aligned
 *   stats       filled on return (NULL: not wanted)
 * Synchronous: returns when every query has ended; runs on `stream`.  Errors
 * as trw_walk (TRW_E_INVALID for a file whose weights or labels the walk needs
 * are absent), TRW_E_INVALID for a destination outside [0, n) in a loaded
 * partition, an unsorted row (Node2Vec) or a failed read, TRW_E_UNSUPPORTED for
 * Node2Vec over more than 1024 partitions, TRW_E_DEVICE for a device error.
 * Unlike other calls, an error found at a load (a bad destination, an unsorted
 * row, a failed read) comes after some queries have run: their outputs are
 * written, the others' are not; nothing of the call is in flight on return.
 */
trw_status trw_disk_walk(trw_disk_graph g, const trw_walk_params *p, const int32_t *d_sources, uint64_t nq,
                         uint64_t qid_base, int32_t *d_paths, uint64_t path_stride, uint32_t *d_lengths,
                         uint8_t *d_status, uint32_t slots, void *d_ws, size_t ws_bytes, void *h_pinned,
                         size_t h_bytes, trw_disk_walk_stats *stats, trw_stream_t stream);

/* ------------------------------------------------------------------------ */
/* PPR estimate (Random Walk based Algorithms, PPR): the score of vertex v   */
/* for a source is the share of the source's queries whose walk ends at v;   */
/* the highest-scoring vertices are the answer.                              */
/* ------------------------------------------------------------------------ */
/*
 * Add the end vertices of a batch's walks to per-group counts.  Query i
 * belongs to group i / group (group 0: every query to group 0) and adds one
 * to d_counts[(i / group) * n + paths[i][lengths[i]]].  A walk that ended at
 * a dead end counts its last vertex (a dangling source counts itself).
 * Skipped, and added to *d_skipped (a device uint64, nullable): queries with
 * status BAD_SOURCE, lengths[i] >= path_stride, or an end outside [0, n).
 *   d_paths, path_stride, d_lengths, d_status   as trw_walk wrote them
 *   d_counts    uint32, counts_len >= groups * n entries, groups = ceil(nq /
 *               group) (1 when group is 0); added to, not cleared
 * Asynchronous on `stream` (device atomics; the counts do not depend on
 * their order).  Errors: TRW_E_INVALID for a NULL pointer with nq > 0,
 * counts_len too small, path_stride 0 or nq >= 2^32.
 */
trw_status trw_ppr_end_counts(trw_graph g, const int32_t *d_paths, uint64_t path_stride,
                              const uint32_t *d_lengths, const uint8_t *d_status, uint64_t nq,
                              uint64_t group, uint32_t *d_counts, uint64_t counts_len,
                              unsigned long long *d_skipped, trw_stream_t stream);

/*
 * PPR walks that count end vertices instead of writing paths: the same walk
 * as trw_walk (PPR, persistent schedule, same random contract and tuning),
 * but query i, when it ends, adds one to d_counts[(i / group) * n + its last
 * vertex] (group 0: one row), the counts trw_ppr_end_counts would give for
 * trw_walk's outputs.  No path is stored, so the walk writes no path rows.
 *   table, p, d_sources, nq, qid_base, tuning   as trw_walk (p->algo = PPR)
 *   d_counts    uint32, counts_len >= groups * n entries; added to, not cleared
 *   d_lengths, d_status   as trw_walk (bad sources: BAD_SOURCE, not counted); both
 *               may be NULL, and then nothing is stored per query, only the counts
 *   d_ws        trw_walk_workspace_bytes for TRW_M_PERSISTENT, 256-byte aligned
 * Errors as trw_walk; TRW_E_UNSUPPORTED unless p->algo is PPR; TRW_E_INVALID
 * for a NULL d_counts or counts_len too small.
 */
trw_status trw_ppr_walk_counts(trw_graph g, trw_table table, const trw_walk_params *p,
                               const int32_t *d_sources, uint64_t nq, uint64_t qid_base, uint64_t group,
                               uint32_t *d_counts, uint64_t counts_len, uint32_t *d_lengths,
                               uint8_t *d_status, const trw_tuning *tuning, void *d_ws, size_t ws_bytes,
                               trw_stream_t stream);

/* Workspace bytes of trw_topk: 1280 + 8*k.  k <= min(n, 4096). */
trw_status trw_topk_workspace_bytes(uint64_t n, uint32_t k, size_t *bytes);

/*
 * The k largest of d_counts[0..n) (n < 2^31), largest first; equal counts
 * are ordered by the smaller index.  Writes d_ids[0..k) (int32) and
 * d_vals[0..k) (the counts).  The result is unique, so it equals a sort of
 * all n (count, index) pairs cut at k.  d_ws: >= trw_topk_workspace_bytes,
 * 256-byte aligned.  Asynchronous on `stream`, no host synchronisation.
 * Errors: TRW_E_INVALID for k > n, k > 4096, n >= 2^31, NULL pointers with
 * k > 0, or a short or misaligned workspace.
 */
trw_status trw_topk(const uint32_t *d_counts, uint64_t n, uint32_t k, int32_t *d_ids, uint32_t *d_vals,
                    void *d_ws, size_t ws_bytes, trw_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Walk programs (Step-centric Programming: the user picks the sampling      */
/* method and writes Weight and Update).  A program is HIP C++ source that   */
/* defines `struct TrwProgram` against paper_2107_11983_amd/csrc/            */
/* program_rt.hpp (it documents the interface):                              */
/*   static constexpr uint32_t kind;   trw_prog::STATIC_NAIVE, STATIC_ALIAS,  */
/*                                     STATIC_ITS, STATIC_REJ, DYNAMIC_REJ,   */
/*                                     DYNAMIC_ITS                            */
/*   __device__ uint32_t weight(walker, graph, params, slot) const;          */
/*       DYNAMIC_REJ: Weight / MaxWeight as Q16 in [0, 65536] (O-REJ);        */
/*       DYNAMIC_ITS: an integer weight (row sums below 2^32)                 */
/*   __device__ bool update(walker, graph, params, r2) const;                */
/*       after a move; true ends the walk (STOPPED); for the rejection kinds */
/*       r2 comes from the accepted dart's block, as in trw_walk's REJ       */
/* The framework runs the batch with the random contract of trw_walk, so    */
/* DeepWalk, PPR, Node2Vec and MetaPath written as programs reproduce the    */
/* built-in walks bit for bit.  Compilation needs the csrc/ directory next   */
/* to libtrw.so (the header is included at run time).                        */
/* ------------------------------------------------------------------------ */
typedef struct trw_program_s *trw_program;

typedef struct {
    uint32_t max_len;          /* moves, 1..65535 */
    uint32_t reserved;
    uint64_t seed;             /* Philox key */
    uint32_t user[16];         /* the program's parameters (params.user in device code) */
} trw_program_params;

/* Compile a program for `arch` (e.g. "gfx950") without loading it: TRW_OK, or
 * TRW_E_INVALID with the compiler's log in trw_last_error().  Needs no GPU. */
trw_status trw_program_check(const char *source, const char *arch);

/* Compile and load a program for the current device.  Errors as
 * trw_program_check, TRW_E_DEVICE if the module cannot be loaded. */
trw_status trw_program_create(const char *source, trw_program *out);

/* The program's sampling method (TrwProgram::kind). */
trw_status trw_program_kind(trw_program p, uint32_t *kind);

/*
 * Run nq queries of program p: query i starts at d_sources[i] with id
 * qid_base + i; outputs as trw_walk (paths rows of path_stride >= max_len+1,
 * lengths, status; sources outside [0, n) get BAD_SOURCE).  table: the ALIAS
 * or ITS table for STATIC_ALIAS / STATIC_ITS programs; otherwise NULL or an
 * edge index (then graph.is_neighbor probes its hash set).  d_ws: 8 bytes of
 * device scratch, 8-byte aligned.  Asynchronous on `stream`.
 */
trw_status trw_program_walk(trw_program p, trw_graph g, trw_table table, const trw_program_params *params,
                            const int32_t *d_sources, uint64_t nq, uint64_t qid_base, int32_t *d_paths,
                            uint64_t path_stride, uint32_t *d_lengths, uint8_t *d_status, void *d_ws,
                            size_t ws_bytes, trw_stream_t stream);

trw_status trw_program_destroy(trw_program p);

/* ------------------------------------------------------------------------ */
/* Serving (all calls thread-safe).  A server keeps the graph, its tables and */
/* a pool of walker slots resident on the GPU and runs a host thread that     */
/* admits requests as memory and request slots free up (continuous batching: */
/* requests that arrive while others run share the device from the next tick)*/
/* The paper's engine runs one batch of queries at a time (Step-centric      */
/* Programming: parallelization); serving is this engine's addition.         */
/* ------------------------------------------------------------------------ */
typedef struct trw_server_s *trw_server;

typedef struct {
    uint32_t max_slots;        /* walker slots, a multiple of 256; 0 = 2048 per CU */
    uint32_t max_requests;     /* requests admitted at once, <= 65536; 0 = 1024 */
    uint32_t steps_per_tick;   /* moves per slot per tick; 0 = 16 */
    uint32_t use_hipgraph;     /* 1: replay the tick as a captured HIP graph */
    uint32_t serial_ticks;     /* 0 (default): the next tick is queued before the host reads the
                                  last one, whose finished requests complete (host outputs copied
                                  on a second stream) while the next tick runs.  1: each tick is
                                  read as it ends and its requests completed before the next one
                                  is queued */
    uint32_t ring_chunks;      /* entries of the device queue of 64-query chunks, 16..2^24;
                                  0 = 2^20.  A request holds at most 32 * ring_chunks - 1 queries;
                                  admission waits while the chunks the device may still read and
                                  the new request's would not fit the ring together */
    uint32_t reserved[2];
} trw_server_cfg;

enum { TRW_REQ_HOST = 1 };     /* sources / paths / lengths / status are host memory */

typedef struct {
    trw_walk_params params;    /* DeepWalk / PPR with NAIVE or ALIAS, Node2Vec with OREJ */
    const int32_t *sources;    /* nq sources: host memory is copied at admission; device
                                  memory is read in place until the request completes */
    uint32_t nq;               /* >= 1 */
    uint32_t flags;            /* TRW_REQ_HOST or 0 (device buffers) */
    uint64_t qid_base;         /* query i has id qid_base + i (same walks as trw_walk) */
    int32_t *paths;            /* nq rows of path_stride entries; device buffers are written in
                                  place as the walks run, host ones at completion */
    uint64_t path_stride;      /* >= max_len + 1 */
    uint32_t *lengths;         /* nq */
    uint8_t *status;           /* nq, trw_walk_status */
    void *user;                /* returned in the completion */
} trw_request;

typedef struct {
    uint64_t request_id;
    int32_t status;            /* TRW_OK or TRW_E_CANCELLED */
    uint32_t nq;
    void *user;
    uint64_t t_submit_ns;      /* host steady clock: submit, admission, outputs complete */
    uint64_t t_admit_ns;
    uint64_t t_done_ns;
} trw_completion;

typedef struct {
    uint64_t submitted, completed, cancelled, rejected, ticks, moves;
    uint32_t active, waiting;
    uint64_t pool_bytes, pool_bytes_used;
    uint64_t tick_device_ns;   /* device time of the tick kernels (HIP events around each launch) */
} trw_server_stats;

/* Device bytes of a server arena for `cfg` with a request pool of pool_bytes. */
trw_status trw_server_arena_bytes(const trw_server_cfg *cfg, size_t pool_bytes, size_t *bytes);

/*
 * Create a server on the current device.  alias: the graph's ALIAS table (or
 * NULL: then ALIAS requests are refused); adjacency: an adjacency or edge
 * index (or NULL).  d_arena: caller-owned device memory (256-byte aligned) holding the
 * fixed server state and, after it, the request pool; keep it alive until
 * trw_server_destroy.  Starts the server thread.
 */
trw_status trw_server_create(trw_graph g, trw_table alias, trw_table adjacency, const trw_server_cfg *cfg,
                             void *d_arena, size_t arena_bytes, trw_server *out);

/* Pool bytes a request occupies while admitted: for host buffers its sources
 * and outputs, staged on the device; 0 for device buffers (used in place). */
trw_status trw_server_request_bytes(trw_server s, const trw_request *r, size_t *bytes);

/*
 * Queue a request.  Returns at once with its id; the request is admitted when
 * a request slot and pool space are free, in submission order.  Errors:
 * TRW_E_NOMEM_BUDGET if it can never fit the pool, TRW_E_UNSUPPORTED /
 * TRW_E_INVALID as trw_walk.  The caller keeps the sources and the output
 * buffers valid until the completion is polled, and reads the outputs only
 * then.  Device outputs are written in place by the walks (no copy at the
 * end; after a cancellation their contents are unspecified); host outputs
 * are staged in the pool and copied out when the request completes.
 */
trw_status trw_server_submit(trw_server s, const trw_request *r, uint64_t *request_id);

/* Cancel a request: it completes with TRW_E_CANCELLED; others are unaffected. */
trw_status trw_server_cancel(trw_server s, uint64_t request_id);

/*
 * Take up to `max` completions, waiting up to timeout_ms for the first one
 * (0 = do not wait).  Returns TRW_E_TIMEOUT if it waited and none arrived.
 */
trw_status trw_server_poll(trw_server s, trw_completion *out, uint32_t max, uint32_t *n_out,
                           uint32_t timeout_ms);

trw_status trw_server_stats_get(trw_server s, trw_server_stats *out);

/* Cancel what is queued or running, stop the thread and release host state. */
trw_status trw_server_destroy(trw_server s);

#ifdef __cplusplus
}
#endif

#endif /* TRW_H */
