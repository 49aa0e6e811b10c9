// The Gather-Move-Update walk step on CDNA4 (gfx950).
//
// One walker per lane.  Each step of a walker (Step-centric Programming, the
// framework algorithm) reads the current vertex's row range (Gather; for
// static walks the per-vertex table built beforehand replaces the gather),
// draws one Philox block keyed by (seed, query, move), samples the next vertex
// (Move) and appends it, then applies the termination rule (Update).
//
// Two schedules:
//  * persistent: one launch.  Each wave claims chunks of query ids from a
//    device queue; a lane whose walk ends takes the next id from its wave's
//    chunk (ballot + mbcnt rank), so lanes stay busy however uneven the walk
//    lengths are.  GPU occupancy plays the part of the paper's step
//    interleaving: many independent walkers per CU keep many random reads in
//    flight.  Optionally each lane interleaves 2 or 4 walkers.
//  * per step (bulk-synchronous): one launch per move over a compacted list
//    of live walker records; finished walkers drop out of the next list.
//
// Memory traffic per move is what bounds the step (random reads fetch whole
// cache lines).  ALIAS entries carry the row range of both candidate
// destinations, so an ALIAS move is a single random 32-byte read; path
// entries are buffered in registers and written 16 bytes at a time on 16-byte
// boundaries of the path row.
//
// Sampling is integer throughout: uniform index = high half of r * d; ALIAS
// coin r1 < thr; ITS draw = high half of (r1:r0) * W and a binary search over
// the uint64 prefix; O-REJ darts compare r1 >> 16 with Q16 thresholds; REJ
// darts compare r1 * p* with w * 2^32; MetaPath counts the matching labels of
// the row and takes the j-th.
#include <algorithm>

#include "trw_device.hpp"
#include "trw_internal.hpp"
#include "walk_common.hpp"

namespace trw {
namespace {


// ---------------------------------------------------------------------------
// MetaPath Gather (the dynamic walk: only edges whose label is the schema's
// label for this move are eligible).  Degree-bucketed:
//  * a row below `coop` labels is scanned by its own lane, 16 bytes per load
//    with kScanLoads loads in flight: one pass counts the matches m, a second
//    stops at the block that holds the j-th one (j = mulhi32(r0, m));
//  * a longer row is scanned by the whole wave, 1 KiB per coalesced load
//    round (16 bytes a lane), the wave's rows one after another.  The row's
//    1 KiB chunks fall into 64 segments whose match counts stay in the lanes'
//    registers (lane s holds segment s), so the second pass rereads one
//    segment instead of the row.
// Labels are compared 16 at a time (SWAR on four 32-bit words).  With a label
// index (rows sorted by label, per-vertex label offsets) the Gather is two
// reads instead.
// ---------------------------------------------------------------------------
constexpr uint32_t kScanLoads = 4;

__device__ __forceinline__ uint32_t match_bits(uint32_t word, uint32_t want4) {
    const uint32_t x = word ^ want4;
    return ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x | 0x7F7F7F7Fu);   // 0x80 where a byte equals want
}

// 0x80 flags of the bytes of the word at wa that lie in [lo, hi).
__device__ __forceinline__ uint32_t byte_window(uintptr_t wa, uintptr_t lo, uintptr_t hi) {
    if (wa >= hi || wa + 4 <= lo) return 0u;
    uint32_t m = 0x80808080u;
    if (lo > wa) m &= 0xFFFFFFFFu << (8u * (uint32_t)(lo - wa));
    if (hi < wa + 4) m &= (1u << (8u * (uint32_t)(hi - wa))) - 1u;
    return m;
}

// The 16-byte-aligned block at ba of the label array [arr_lo, arr_hi); bytes
// outside the array are not read (they read as 0 and lie outside every row,
// so the row window masks them).
__device__ __forceinline__ uint4 load_block(uintptr_t ba, uintptr_t arr_lo, uintptr_t arr_hi) {
    if (ba >= arr_lo && ba + 16 <= arr_hi) return *reinterpret_cast<const uint4 *>(ba);
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    for (uint32_t b = 0; b < 16; ++b)
        if (ba + b >= arr_lo && ba + b < arr_hi)
            w[b >> 2] |= (uint32_t)(*reinterpret_cast<const uint8_t *>(ba + b)) << (8u * (b & 3u));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// Match flags (0x80 per matching byte) of the four words of the block at ba,
// restricted to the row [lo, hi).
struct BlockBits {
    uint32_t w[4];
};

__device__ __forceinline__ BlockBits block_bits(const uint4 &v, uintptr_t ba, uintptr_t lo, uintptr_t hi,
                                                uint32_t want4) {
    BlockBits b;
    b.w[0] = match_bits(v.x, want4) & byte_window(ba, lo, hi);
    b.w[1] = match_bits(v.y, want4) & byte_window(ba + 4, lo, hi);
    b.w[2] = match_bits(v.z, want4) & byte_window(ba + 8, lo, hi);
    b.w[3] = match_bits(v.w, want4) & byte_window(ba + 12, lo, hi);
    return b;
}

__device__ __forceinline__ uint32_t bits_count(const BlockBits &b) {
    return __popc(b.w[0]) + __popc(b.w[1]) + __popc(b.w[2]) + __popc(b.w[3]);
}

// Offset from ba of the j-th (0-based) flagged byte of the block; j < bits_count(b).
__device__ __forceinline__ uint32_t bits_select(BlockBits b, uint32_t j) {
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
        const uint32_t c = __popc(b.w[q]);
        if (j < c) {
            uint32_t bits = b.w[q];
            for (; j > 0; --j) bits &= bits - 1u;
            return 4u * q + (uint32_t)(__builtin_ctz(bits) >> 3);
        }
        j -= c;
    }
    return 16u;
}

// One lane, a whole row [l, l + d): the offset from l of the j-th matching
// label, j = mulhi32(r0, m) with m the row's number of matches; -1 when m = 0.
__device__ __forceinline__ int64_t lane_pick(uintptr_t l, uint32_t d, uint32_t want4, uint32_t r0, uintptr_t arr_lo,
                                             uintptr_t arr_hi) {
    const uintptr_t h = l + d;
    const uintptr_t b0 = l & ~(uintptr_t)15;
    uint32_t m = 0;
    for (uintptr_t ba = b0; ba < h; ba += 16 * kScanLoads) {
        uint4 v[kScanLoads];
#pragma unroll
        for (uint32_t u = 0; u < kScanLoads; ++u)
            v[u] = ba + 16 * u < h ? load_block(ba + 16 * u, arr_lo, arr_hi) : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (uint32_t u = 0; u < kScanLoads; ++u) m += bits_count(block_bits(v[u], ba + 16 * u, l, h, want4));
    }
    if (m == 0) return -1;
    uint32_t j = scale32(r0, m);                 // < m: the second pass stops inside the row
    for (uintptr_t ba = b0; ba < h; ba += 16 * kScanLoads) {
        uint4 v[kScanLoads];
#pragma unroll
        for (uint32_t u = 0; u < kScanLoads; ++u)
            v[u] = ba + 16 * u < h ? load_block(ba + 16 * u, arr_lo, arr_hi) : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (uint32_t u = 0; u < kScanLoads; ++u) {
            const BlockBits b = block_bits(v[u], ba + 16 * u, l, h, want4);
            const uint32_t c = bits_count(b);
            if (j < c) return (int64_t)(ba + 16 * u + bits_select(b, j)) - (int64_t)l;
            j -= c;
        }
    }
    return -1;
}

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o);
        if (lane >= (uint32_t)o) v += t;
    }
    return v;
}

// Whole wave, uniform arguments: the offset from l of the j-th matching label
// with j = mulhi32(r0, m), m the number of matches; -1 when m == 0.  Chunk c
// is the 1 KiB at b0 + 1024 c (lane i reads its 16 bytes at + 16 i); chunks
// [s cps, (s + 1) cps) form segment s, whose match count lane s keeps.
__device__ int64_t wave_pick(uintptr_t l, uint32_t d, uint32_t want4, uint32_t r0, uintptr_t arr_lo,
                             uintptr_t arr_hi) {
    const uint32_t lane = lane_id();
    const uintptr_t h = l + d;
    const uintptr_t b0 = l & ~(uintptr_t)15;
    const uint32_t nchunk = (uint32_t)((h - b0 + 1023) >> 10);
    const uint32_t cps = (nchunk + 63) >> 6;
    uint32_t seg = 0, run = 0;
    for (uint32_t c0 = 0; c0 < nchunk; c0 += kScanLoads) {
        uint4 v[kScanLoads];
#pragma unroll
        for (uint32_t u = 0; u < kScanLoads; ++u) {
            const uintptr_t ba = b0 + 1024 * (uintptr_t)(c0 + u) + 16 * lane;
            v[u] = c0 + u < nchunk && ba < h ? load_block(ba, arr_lo, arr_hi) : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (uint32_t u = 0; u < kScanLoads; ++u) {
            const uint32_t c = c0 + u;
            if (c >= nchunk) break;
            run += bits_count(block_bits(v[u], b0 + 1024 * (uintptr_t)c + 16 * lane, l, h, want4));
            if ((c + 1) % cps == 0 || c + 1 == nchunk) {       // end of segment c / cps
                const uint32_t tot = wave_total(run);
                if (lane == c / cps) seg = tot;
                run = 0;
            }
        }
    }
    const uint32_t incl = wave_inclusive_scan(seg);
    const uint32_t m = __shfl(incl, 63);
    if (m == 0) return -1;
    const uint32_t j = scale32(r0, m);
    const int s = (int)__builtin_ctzll(__ballot(j < incl));      // the segment holding match j
    uint32_t jj = j - (uint32_t)__shfl(incl - seg, s);
    const uint32_t c_end = min(nchunk, (uint32_t)(s + 1) * cps);
    for (uint32_t c0 = (uint32_t)s * cps; c0 < c_end; c0 += kScanLoads) {
        uint4 v[kScanLoads];
#pragma unroll
        for (uint32_t u = 0; u < kScanLoads; ++u) {
            const uintptr_t ba = b0 + 1024 * (uintptr_t)(c0 + u) + 16 * lane;
            v[u] = c0 + u < c_end && ba < h ? load_block(ba, arr_lo, arr_hi) : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (uint32_t u = 0; u < kScanLoads; ++u) {
            const uint32_t c = c0 + u;
            if (c >= c_end) break;
            const uintptr_t ba = b0 + 1024 * (uintptr_t)c + 16 * lane;
            const BlockBits b = block_bits(v[u], ba, l, h, want4);
            const uint32_t cnt = bits_count(b);
            const uint32_t ci = wave_inclusive_scan(cnt);
            const uint32_t total = __shfl(ci, 63);
            if (jj < total) {
                const bool mine = cnt != 0 && ci - cnt <= jj && jj < ci;
                int64_t pos = -1;
                if (mine) pos = (int64_t)(ba + bits_select(b, jj - (ci - cnt))) - (int64_t)l;
                return __shfl(pos, (int)__builtin_ctzll(__ballot(mine)));
            }
            jj -= total;
        }
    }
    return -1;
}

// The label the schema gives move k.
__device__ __forceinline__ uint32_t schema_label(const WalkDev &a, uint32_t k) {
    const uint32_t si = k % a.schema_len;
    const uint64_t word = si < 8 ? a.schema_lo : a.schema_hi;
    return (uint32_t)(uint8_t)(word >> ((si & 7u) * 8u));
}

// Label offset i (0..kMaxFusedLabels) of a fused entry {dst, offsets...}.
__device__ __forceinline__ int32_t fused_offset(const uint4 &f0, const uint4 &f1, uint32_t i) {
    const uint32_t v = i == 0 ? f0.y : i == 1 ? f0.z : i == 2 ? f0.w : i == 3 ? f1.x : i == 4 ? f1.y : i == 5 ? f1.z
                                                                                                               : f1.w;
    return (int32_t)v;
}

// One MetaPath move for every lane of the wave (call with uniform control
// flow; `active` says whether this lane has a walker).  Returns the next
// vertex or -1 (no eligible edge).
template <uint32_t SMP>
__device__ __forceinline__ int32_t metapath_move(const GraphDev &g, const TableDev &t, const WalkDev &a, bool active,
                                                 uint32_t k, int32_t cur, int32_t off, uint32_t d, uint32_t r0,
                                                 uint32_t coop) {
    const uint32_t si = k % a.schema_len;
    const uint64_t word = si < 8 ? a.schema_lo : a.schema_hi;
    const uint32_t want = (uint32_t)(uint8_t)(word >> ((si & 7u) * 8u));
    if (SMP == SMP_LABEL_INDEX) {
        if (!active) return -1;
        const int32_t *rec = t.loff + (uint64_t)cur * (t.nlab + 1);
        const int32_t lo = rec[want], hi = rec[want + 1];
        if (hi == lo) return -1;
        return t.lcol[lo + scale32(r0, (uint32_t)(hi - lo))];
    }
    const uint32_t want4 = want * 0x01010101u;
    const uintptr_t base = reinterpret_cast<uintptr_t>(g.label);
    const uintptr_t arr_end = base + (uintptr_t)g.m;
    int32_t nxt = -1;
    const bool big = active && d >= coop;
    if (active && !big && d > 0) {
        const int64_t pos = lane_pick(base + (uintptr_t)off, d, want4, r0, base, arr_end);
        if (pos >= 0) nxt = g.col[off + pos];
    }
    uint64_t todo = __ballot(big);
    while (todo) {
        const int src = (int)__builtin_ctzll(todo);
        todo &= todo - 1;
        const int32_t off_s = __shfl(off, src);
        const uint32_t d_s = __shfl(d, src);
        const uint32_t want4_s = __shfl(want4, src);
        const uint32_t r0_s = __shfl(r0, src);
        const int64_t pos = wave_pick(base + (uintptr_t)off_s, d_s, want4_s, r0_s, base, arr_end);
        if (lane_id() == (uint32_t)src && pos >= 0) nxt = g.col[off_s + pos];
    }
    return nxt;
}

// ---------------------------------------------------------------------------
// Persistent schedule
// ---------------------------------------------------------------------------
// Lengths and status of a wave's queries are gathered in LDS, one slot per id
// range the wave claims, and written with coalesced stores when the range's
// last query has ended; stored one by one as walks end they would land on
// scattered, partly written lines.  A range that finds no free slot, or any
// range when the launch has no slots, is written directly.  A query carries
// its place as code = slot * kStageQueries + index in the range.
constexpr uint32_t kStageQueries = 256;        // ids per staged range (queue_chunk <= this)
constexpr uint32_t kStageDirect = 0xFFFFFFFFu;
constexpr uint32_t kMaxStageSlots = 8;
struct StageSlot {
    uint32_t base, size, left, pad;            // size 0: free
    uint16_t len[kStageQueries];               // moves (max_len <= 65535)
    uint8_t st[kStageQueries];
};

struct Walker {
    uint32_t qi;     // index in the batch, kIdle when the slot is free
    uint32_t code;   // where its length and status go (kStageDirect: straight to memory)
    int32_t cur;
    int32_t prev;
    uint32_t k;
    int32_t off;     // row of cur (valid when !need_row)
    int32_t deg;
    int32_t poff;    // row of prev (Node2Vec)
    int32_t pdeg;
    uint32_t dart;   // REJ: darts thrown for the current move
    uint32_t pm;     // REJ: p* of cur
    uint64_t W;      // ITS: weight sum of cur's row
    bool need_row;
    PathBuf path;
};

constexpr int32_t kMissed = -2;   // REJ: this iteration's dart missed; no move

// COUNTS: instead of writing paths, a walk that ends adds one to
// a.end_counts[group of its query][its last vertex] (PPR's estimate).
template <uint32_t ALGO, uint32_t SMP, int WPL, bool COUNTS = false>
__global__ void __launch_bounds__(256)
k_walk_persistent(GraphDev g, TableDev t, WalkDev a, unsigned long long *__restrict__ queue_head,
                  uint32_t chunk, uint32_t coop, uint32_t n_slots) {
    constexpr bool kStatic = (ALGO == ALG_DEEPWALK || ALGO == ALG_PPR);
    constexpr bool kAlias = kStatic && SMP == SMP_ALIAS;
    constexpr bool kOneRead = kAlias || (kStatic && SMP == SMP_NAIVE_ADJ);   // entry carries the next row
    constexpr bool kNoRows = (SMP == SMP_LABEL_INDEX);   // the label index replaces the row lookup
    constexpr bool kRej = kStatic && SMP == SMP_REJ;
    constexpr bool kIts = kStatic && SMP == SMP_ITS;    // search, then the chosen slot's next record
    // MetaPath through fused label-index entries: off / deg hold the run of the
    // label the walker's next move wants; the entry a move reads carries the
    // destination's label offsets, so the next run needs no further read.
    constexpr bool kLabelFused = ALGO == ALG_METAPATH && SMP == SMP_LABEL_FUSED;
    Walker w[WPL];
#pragma unroll
    for (int i = 0; i < WPL; ++i) w[i].qi = kIdle;
    const uint32_t lane = lane_id();
    const unsigned long long n_waves = ((unsigned long long)gridDim.x * blockDim.x + 63) / 64;
    extern __shared__ StageSlot stage_mem[];
    StageSlot *slots = stage_mem + (threadIdx.x >> 6) * n_slots;   // this wave's
    for (uint32_t i = 0; i < n_slots; ++i)
        if (lane == 0) slots[i].size = 0;
    uint32_t done_slots = 0;                // per lane: slots whose last query this lane ended

    // A query ended: record its length and status.
    auto record = [&](uint32_t code, uint32_t qi, uint32_t k, uint8_t st) {
        if (COUNTS && a.lengths == nullptr) return;     // a counting walk that keeps only the counts
        if (code == kStageDirect) {
            a.lengths[qi] = k;
            a.status[qi] = st;
        } else {
            StageSlot &sl = slots[code / kStageQueries];
            sl.len[code % kStageQueries] = (uint16_t)k;
            sl.st[code % kStageQueries] = st;
            if (atomicSub(&sl.left, 1u) == 1u) done_slots |= 1u << (code / kStageQueries);
        }
    };

    // Query starts are prepared ahead of need, one stage per iteration, so a
    // walker's first move never waits for its source and row range: the
    // loads of both stages are in flight together with the moves' reads.
    //   S: a claimed query index and its source (load issued);
    //   R: a query ready to start: source and row range (loads issued).
    // The loaded values are first used right after the moves' reads have
    // arrived (s_bad, r_deg), never at the top of the next iteration: there a
    // wait for them would also wait for this iteration's stores.
    uint32_t s_qi = kIdle, r_qi = kIdle, s_code = kStageDirect, r_code = kStageDirect;
    int32_t s_src = 0, r_src = 0, r_lo = 0, r_hi = 0, r_deg = 0;
    uint32_t r_pm = 0;                      // REJ: p* of the ready query's source
    uint64_t r_W = 0;                       // ITS: weight sum of the ready query's source
    bool s_bad = false;

    // Id ranges come from the queue head one claim ahead: the next range is
    // requested when the current one is taken into use, so its atomic's
    // latency is hidden too.  Guided sizes: a share of what was left at the
    // previous claim, between 64 ids and `chunk`, so that early claims are
    // large (few atomics) and late ones small (waves finish together).
    auto guided = [&](unsigned long long seen) -> uint32_t {
        const unsigned long long left = seen < a.nq ? a.nq - seen : 0;
        const uint32_t take = (uint32_t)min(left / (2ull * n_waves), (unsigned long long)chunk);
        return max(take, min(64u, chunk));
    };
    uint32_t pool_next = 0, pool_end = 0;   // the wave's current id range (wave-uniform)
    uint32_t pool_base = 0, pool_slot = kStageDirect;   // its first id and staging slot
    uint32_t ahead_take = guided(0);
    unsigned long long ahead_base = 0;      // lane 0: result of the claim issued ahead
    if (lane == 0) ahead_base = atomicAdd(queue_head, (unsigned long long)ahead_take);
    unsigned long long ahead_seen = __shfl(ahead_base, 0);   // the same, wave-wide, once it has arrived
    bool ahead_pending = false;             // claim issued this iteration, ahead_seen not updated yet
    bool exhausted = false;

    // The exit test sits at the bottom of the loop: a break in the middle
    // gives the compiler a loop edge on which the prepared loads look
    // outstanding, and it then waits for them (and for every store before
    // them) at the top of each iteration.
    bool more = true;
    do {
        // Start: an idle walker takes the ready query (its loads were issued
        // in an earlier iteration).
#pragma unroll
        for (int i = 0; i < WPL; ++i) {
            if (w[i].qi == kIdle && r_qi != kIdle) {
                w[i].qi = r_qi; w[i].code = r_code; w[i].cur = r_src; w[i].prev = -1; w[i].k = 0;
                w[i].poff = 0; w[i].pdeg = 0; w[i].need_row = false;
                w[i].dart = 0; w[i].pm = r_pm; w[i].W = r_W;
                w[i].off = r_lo; w[i].deg = kNoRows ? 1 : r_deg;
                if (!COUNTS) {
                    w[i].path.start(a.paths + (uint64_t)r_qi * a.stride);
                    w[i].path.push(r_src);
                }
                r_qi = kIdle;
            }
        }
        // S -> R: the source is known; reject it or request its row range.
        if (r_qi == kIdle && s_qi != kIdle) {
            if (s_bad) {
                record(s_code, s_qi, 0, ST_BAD_SOURCE);
            } else {
                r_qi = s_qi; r_code = s_code; r_src = s_src;
                if (kLabelFused) {
                    const int32_t *lrec = t.loff + (uint64_t)s_src * (t.nlab + 1);
                    const uint32_t l0 = schema_label(a, 0);
                    r_lo = lrec[l0];
                    r_hi = lrec[l0 + 1];
                } else if (!kNoRows) {
                    r_lo = g.row_ptr[s_src];
                    r_hi = g.row_ptr[s_src + 1];
                }
                if (kRej) r_pm = t.pmax[s_src];
                if (kIts) r_W = t.its_w[s_src];
            }
            s_qi = kIdle;
        }
        // Claim: lanes with an empty S take the next ids of the wave's range.
        uint64_t need = __ballot(s_qi == kIdle);
        while (need != 0 && !exhausted) {
            uint32_t avail = pool_end - pool_next;
            if (avail == 0) {
                if (ahead_pending) { ahead_seen = __shfl(ahead_base, 0); ahead_pending = false; }   // rare
                const unsigned long long base = ahead_seen;
                if (base >= a.nq) { exhausted = true; break; }
                pool_next = (uint32_t)base;
                pool_end = (uint32_t)min(base + ahead_take, (unsigned long long)a.nq);
                avail = pool_end - pool_next;
                pool_base = pool_next;
                pool_slot = kStageDirect;
                for (uint32_t i = 0; i < n_slots; ++i) {
                    if (slots[i].size == 0) {
                        if (lane == 0) { slots[i].base = pool_base; slots[i].size = avail; slots[i].left = avail; }
                        pool_slot = i;
                        break;
                    }
                }
                ahead_take = guided(base + ahead_take);
                if (lane == 0) ahead_base = atomicAdd(queue_head, (unsigned long long)ahead_take);
                ahead_pending = true;
            }
            const uint32_t rk = rank_below(need);
            if (((need >> lane) & 1ull) && rk < avail) {
                s_qi = pool_next + rk;
                s_code = pool_slot == kStageDirect ? kStageDirect : pool_slot * kStageQueries + (s_qi - pool_base);
                s_src = a.sources[s_qi];
            }
            pool_next += min((uint32_t)__popcll(need), avail);
            need = __ballot(s_qi == kIdle);
        }
        // Gather: row ranges the walkers do not carry yet (independent loads).
#pragma unroll
        for (int i = 0; i < WPL; ++i) {
            if (w[i].qi != kIdle && w[i].need_row) {
                const int32_t lo = g.row_ptr[w[i].cur];
                w[i].deg = g.row_ptr[w[i].cur + 1] - lo;
                w[i].off = lo;
                w[i].need_row = false;
            }
        }
        Rand4 r[WPL];
#pragma unroll
        for (int i = 0; i < WPL; ++i) r[i] = philox(w[i].k, kRej ? w[i].dart : 0u, a.qid_base + w[i].qi, a.seed);

        // Move.
        int32_t nxt[WPL];
        if (kOneRead) {
            uint4 e0[WPL], e1[WPL];
#pragma unroll
            for (int i = 0; i < WPL; ++i) {
                if (w[i].qi != kIdle && w[i].deg != 0) {
                    const uint32_t e = (uint32_t)w[i].off + scale32(r[i].r0, (uint32_t)w[i].deg);
                    if (kAlias) {
                        e0[i] = t.alias[2 * (uint64_t)e];
                        e1[i] = t.alias[2 * (uint64_t)e + 1];
                    } else {
                        e0[i] = t.adj[e];
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < WPL; ++i) {
                nxt[i] = -1;
                if (w[i].qi != kIdle && w[i].deg != 0) {
                    w[i].poff = w[i].off; w[i].pdeg = w[i].deg;
                    if (kAlias) {
                        nxt[i] = alias_pick(e0[i], e1[i], r[i].r1, w[i].off, w[i].deg);
                    } else {
                        nxt[i] = (int32_t)e0[i].x; w[i].off = (int32_t)e0[i].y; w[i].deg = (int32_t)e0[i].z;
                    }
                }
            }
        } else if (kLabelFused) {
            uint4 f0[WPL], f1[WPL];
#pragma unroll
            for (int i = 0; i < WPL; ++i) {
                if (w[i].qi != kIdle && w[i].deg != 0) {
                    const uint64_t e = (uint64_t)(uint32_t)w[i].off + scale32(r[i].r0, (uint32_t)w[i].deg);
                    f0[i] = t.lfused[2 * e];
                    f1[i] = t.lfused[2 * e + 1];
                }
            }
#pragma unroll
            for (int i = 0; i < WPL; ++i) {
                nxt[i] = -1;
                if (w[i].qi != kIdle && w[i].deg != 0) {
                    nxt[i] = (int32_t)f0[i].x;
                    const uint32_t nl = schema_label(a, w[i].k + 1);
                    const int32_t lo = fused_offset(f0[i], f1[i], nl);
                    w[i].off = lo;
                    w[i].deg = fused_offset(f0[i], f1[i], nl + 1) - lo;
                }
            }
        } else if (ALGO == ALG_METAPATH) {
#pragma unroll
            for (int i = 0; i < WPL; ++i) {
                const bool act = w[i].qi != kIdle;
                nxt[i] = metapath_move<SMP>(g, t, a, act, w[i].k, w[i].cur, w[i].off, (uint32_t)w[i].deg,
                                            r[i].r0, coop);
                if (act) w[i].need_row = !kNoRows;
            }
        } else if (ALGO == ALG_NODE2VEC) {
            constexpr bool kAdj = SMP == SMP_OREJ_ADJ;
#pragma unroll
            for (int i = 0; i < WPL; ++i) {
                nxt[i] = -1;
                if (w[i].qi != kIdle && w[i].deg != 0) {
                    int32_t no = 0, nd = 0;
                    nxt[i] = n2v_move<kAdj>(g, t, a, a.qid_base + w[i].qi, w[i].k, w[i].off, (uint32_t)w[i].deg,
                                            r[i], w[i].prev, w[i].poff, w[i].pdeg, no, nd);
                    w[i].poff = w[i].off; w[i].pdeg = w[i].deg;
                    if (kAdj) { w[i].off = no; w[i].deg = nd; }
                    w[i].need_row = !kAdj;
                }
            }
        } else if (kIts) {
            // x uniform in [0, W) from 64 bits; the smallest i with x < prefix[i]
            // (its_search_block; bisection for rows below a tuned degree); the slot's record then gives the next vertex,
            // its row and its W.
#pragma unroll
            for (int i = 0; i < WPL; ++i) {
                nxt[i] = -1;
                if (w[i].qi != kIdle && w[i].deg != 0 && w[i].W != 0) {
                    const uint64_t *__restrict__ pr = t.prefix + (uint32_t)w[i].off;
                    const uint64_t x = scale64(r[i].r0, r[i].r1, w[i].W);
                    const uint32_t dg = (uint32_t)w[i].deg;
                    const uint32_t lo = dg >= a.its_gallop
                                            ? its_search_block(pr, dg, x, ((uint64_t)r[i].r1 << 32) | r[i].r0)
                                            : its_bisect(pr, dg, x);
                    const uint64_t e = (uint64_t)(uint32_t)w[i].off + lo;
                    const uint4 n0 = t.its_next[2 * e];
                    const uint4 n1 = t.its_next[2 * e + 1];
                    nxt[i] = (int32_t)n0.x;
                    w[i].off = (int32_t)n0.y; w[i].deg = (int32_t)n0.z;
                    w[i].W = (uint64_t)n1.x | ((uint64_t)n1.y << 32);
                }
            }
        } else if (kRej) {
            // One dart per walker per iteration: a walker whose dart misses
            // keeps its state and throws its next dart in the next iteration,
            // so the lanes of a wave never wait for each other's misses.
            uint4 e0[WPL];
            uint32_t e_pm[WPL];
#pragma unroll
            for (int i = 0; i < WPL; ++i) {
                if (w[i].qi != kIdle && w[i].deg != 0 && w[i].pm != 0) {
                    const uint64_t e = (uint64_t)(uint32_t)w[i].off + scale32(r[i].r0, (uint32_t)w[i].deg);
                    e0[i] = t.rej[2 * e];
                    e_pm[i] = t.rej[2 * e + 1].x;
                }
            }
#pragma unroll
            for (int i = 0; i < WPL; ++i) {
                nxt[i] = -1;
                if (w[i].qi != kIdle && w[i].deg != 0 && w[i].pm != 0) {
                    if (rej_hit(r[i].r1, w[i].pm, e0[i].x) || w[i].dart + 1 == kMaxDarts) {
                        nxt[i] = (int32_t)e0[i].y;
                        w[i].off = (int32_t)e0[i].z; w[i].deg = (int32_t)e0[i].w;
                        w[i].pm = e_pm[i]; w[i].dart = 0;
                    } else {
                        nxt[i] = kMissed;
                        w[i].dart += 1;
                    }
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < WPL; ++i) {
                nxt[i] = -1;
                if (w[i].qi != kIdle && w[i].deg != 0) {
                    nxt[i] = static_next<SMP>(g, t, w[i].off, (uint32_t)w[i].deg, r[i], a.its_gallop);
                    w[i].poff = w[i].off; w[i].pdeg = w[i].deg;
                    w[i].need_row = true;
                }
            }
        }

        // The prepared starts' loads were issued before the moves' reads and
        // have arrived with them.  The empty asm reads the loaded registers
        // here, on every path through the loop, so that the compiler knows
        // they are complete at the top of the next iteration.
        asm volatile("" ::"v"(s_src), "v"(r_lo), "v"(r_hi), "v"(ahead_base));
        if (kRej) asm volatile("" ::"v"(r_pm));
        if (kIts) asm volatile("" ::"v"(r_W));
        s_bad = (uint32_t)s_src >= (uint32_t)g.n;
        r_deg = r_hi - r_lo;
        ahead_seen = __shfl(ahead_base, 0);
        ahead_pending = false;

        // Update.
#pragma unroll
        for (int i = 0; i < WPL; ++i) {
            if (w[i].qi == kIdle) continue;
            if (kRej && nxt[i] == kMissed) continue;
            uint8_t st = 0;
            if (nxt[i] < 0) {
                st = ST_DEAD_END;
            } else {
                if (!COUNTS) w[i].path.push(nxt[i]);
                w[i].prev = w[i].cur;
                w[i].cur = nxt[i];
                w[i].k += 1;
                if (ALGO == ALG_PPR && r[i].r2 < a.stop_q32) st = ST_STOPPED;
                else if (w[i].k == a.max_len) st = ST_LENGTH;
            }
            if (st) {
                if (COUNTS) {
                    const uint64_t row = a.end_group ? (uint64_t)w[i].qi / a.end_group : 0;
                    atomicAdd(&a.end_counts[row * (uint64_t)g.n + (uint32_t)w[i].cur], 1u);
                } else {
                    w[i].path.finish(a.paths + ((uint64_t)w[i].qi + 1) * a.stride);
                }
                record(w[i].code, w[i].qi, w[i].k, st);
                w[i].qi = kIdle;
            }
        }

        // Ranges whose last query ended in this iteration: coalesced writes.
        if (__ballot(done_slots != 0) != 0) {
            uint32_t wave_done = done_slots;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) wave_done |= __shfl_xor(wave_done, o);
            done_slots = 0;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            while (wave_done != 0) {
                const uint32_t sl_i = __builtin_ctz(wave_done);
                wave_done &= wave_done - 1;
                StageSlot &sl = slots[sl_i];
                const uint32_t base = sl.base, size = sl.size;
                for (uint32_t j = lane; j < size; j += 64) {
                    a.lengths[base + j] = sl.len[j];
                    a.status[base + j] = sl.st[j];
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                if (lane == 0) sl.size = 0;
            }
        }

        // Done when the queue is drained and nothing is running or prepared.
        bool any = r_qi != kIdle || s_qi != kIdle;
#pragma unroll
        for (int i = 0; i < WPL; ++i) any |= (w[i].qi != kIdle);
        more = !exhausted || __ballot(any) != 0;
    } while (more);
}

// ---------------------------------------------------------------------------
// Per-step (bulk-synchronous) schedule
// ---------------------------------------------------------------------------
// A live walker between launches: query index, current vertex and two words
// that are the row range of cur for ALIAS walks, and (prev, unused) otherwise.
// REJ walks keep p* of cur in place of cur (the vertex itself is not needed
// again) and its row range in the two words.
struct alignas(16) Rec {
    uint32_t qi;
    int32_t cur;
    int32_t a;
    int32_t b;
};

__global__ void k_fill_u32(uint32_t *p, uint32_t n, uint32_t v) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// CARRY: 0 records hold (source, -1, 0); 1 the source's row range; 2 for REJ
// also its p*.
template <uint32_t CARRY>
__global__ void __launch_bounds__(256) k_bsp_init(GraphDev g, TableDev t, WalkDev a, Rec *__restrict__ out,
                                                  uint32_t *__restrict__ count) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = 0; base < a.nq; base += stride) {
        const uint64_t i = base + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
        bool keep = false;
        int32_t s = 0;
        if (i < a.nq) {
            s = a.sources[i];
            if (s < 0 || s >= g.n) {
                a.lengths[i] = 0;
                a.status[i] = ST_BAD_SOURCE;
            } else {
                a.paths[i * a.stride] = s;
                keep = true;
            }
        }
        const uint32_t slot = wave_append(count, keep);
        if (keep) {
            if (CARRY != 0) {
                const int32_t lo = g.row_ptr[s];
                const int32_t first = CARRY == 2 ? (int32_t)t.pmax[s] : s;
                out[slot] = Rec{(uint32_t)i, first, lo, g.row_ptr[s + 1] - lo};
            } else {
                out[slot] = Rec{(uint32_t)i, s, -1, 0};
            }
        }
    }
}

template <uint32_t ALGO, uint32_t SMP>
__global__ void __launch_bounds__(256) k_bsp_step(GraphDev g, TableDev t, WalkDev a, uint32_t k,
                                                  const Rec *__restrict__ in, const uint32_t *__restrict__ count_in,
                                                  Rec *__restrict__ out, uint32_t *__restrict__ count_out,
                                                  uint32_t coop) {
    constexpr bool kStatic = (ALGO == ALG_DEEPWALK || ALGO == ALG_PPR);
    constexpr bool kAlias = kStatic && SMP == SMP_ALIAS;
    constexpr bool kRej = kStatic && SMP == SMP_REJ;
    constexpr bool kCarry = kAlias || kRej || (kStatic && SMP == SMP_NAIVE_ADJ);   // records carry cur's row
    const uint32_t n_in = *count_in;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = 0; base < n_in; base += stride) {
        const uint32_t idx = base + blockIdx.x * blockDim.x + threadIdx.x;
        const bool act = idx < n_in;
        Rec rc{0u, 0, -1, 0};
        Rand4 r{0u, 0u, 0u, 0u};
        int32_t off = 0;
        uint32_t d = 0;
        if (act) {
            rc = in[idx];
            r = philox(k, 0, a.qid_base + rc.qi, a.seed);
            if (!kCarry && SMP != SMP_LABEL_INDEX) {
                off = g.row_ptr[rc.cur];
                d = (uint32_t)(g.row_ptr[rc.cur + 1] - off);
            }
        }
        int32_t nxt = -1, noff = 0, ndeg = 0;
        uint32_t npm = 0;
        if (ALGO == ALG_METAPATH) {
            nxt = metapath_move<SMP>(g, t, a, act, k, rc.cur, off, d, r.r0, coop);
        } else if (act) {
            if (kCarry) {
                if (rc.b != 0 && kRej) {
                    nxt = rej_move(t, a, a.qid_base + rc.qi, k, rc.a, (uint32_t)rc.b, (uint32_t)rc.cur, r, noff, ndeg,
                                   npm);
                } else if (rc.b != 0) {
                    const uint32_t e = (uint32_t)rc.a + scale32(r.r0, (uint32_t)rc.b);
                    if (kAlias) {
                        // the whole 32-byte entry in one read, then the pick (picking from
                        // the loads lets the compiler read the threshold, then the half)
                        const uint4 e0 = t.alias[2 * (uint64_t)e], e1 = t.alias[2 * (uint64_t)e + 1];
                        asm volatile("" ::"v"(e0.x), "v"(e0.y), "v"(e0.z), "v"(e1.x), "v"(e1.y), "v"(e1.z),
                                     "v"(e1.w));
                        nxt = alias_pick(e0, e1, r.r1, noff, ndeg);
                    } else {
                        const uint4 rec = t.adj[e];
                        nxt = (int32_t)rec.x; noff = (int32_t)rec.y; ndeg = (int32_t)rec.z;
                    }
                }
            } else if (ALGO == ALG_NODE2VEC) {
                int32_t poff = 0, pd = 0, no = 0, nd = 0;
                if (rc.a >= 0) {
                    poff = g.row_ptr[rc.a];
                    pd = g.row_ptr[rc.a + 1] - poff;
                }
                if (d != 0)
                    nxt = n2v_move<SMP == SMP_OREJ_ADJ>(g, t, a, a.qid_base + rc.qi, k, off, d, r, rc.a, poff, pd, no, nd);
            } else {
                if (d != 0) nxt = static_next<SMP>(g, t, off, d, r, a.its_gallop);
            }
        }
        bool keep = false;
        Rec nr{};
        if (act) {
            uint8_t st = 0;
            uint32_t len = k;
            if (nxt < 0) {
                st = ST_DEAD_END;
            } else {
                a.paths[(uint64_t)rc.qi * a.stride + k + 1] = nxt;
                len = k + 1;
                if (ALGO == ALG_PPR && r.r2 < a.stop_q32) st = ST_STOPPED;
                else if (len == a.max_len) st = ST_LENGTH;
            }
            if (st) {
                a.lengths[rc.qi] = len;
                a.status[rc.qi] = st;
            } else {
                keep = true;
                nr = kRej ? Rec{rc.qi, (int32_t)npm, noff, ndeg}
                          : kCarry ? Rec{rc.qi, nxt, noff, ndeg} : Rec{rc.qi, nxt, rc.cur, 0};
            }
        }
        const uint32_t slot = wave_append(count_out, keep);
        if (keep) out[slot] = nr;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
constexpr size_t kAlign = 256;
inline size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

template <uint32_t ALGO, uint32_t SMP, bool COUNTS = false>
hipError_t run_persistent(const GraphDev &g, const TableDev &t, const WalkDev &w, const Tuning &tu,
                          const DeviceInfo &di, void *ws, hipStream_t s) {
    auto *head = reinterpret_cast<unsigned long long *>(ws);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t *>(ws), 2u, 0u);
    const uint32_t threads = tu.block_threads;
    const uint64_t waves_needed = ((uint64_t)w.nq + 63) / 64;
    uint64_t blocks = (uint64_t)di.num_cus * tu.blocks_per_cu;
    const uint64_t max_useful = (waves_needed * 64 + threads - 1) / threads;
    if (blocks > max_useful) blocks = max_useful;
    if (blocks == 0) blocks = 1;
    // Staging slots per wave: as many as the CU's LDS holds for blocks_per_cu
    // resident blocks (so staging never lowers occupancy), at most
    // kMaxStageSlots and 64 KiB per block; none when ranges can exceed a slot.
    const uint32_t waves = threads / 64;
    uint32_t n_slots = 0;
    if (tu.queue_chunk <= kStageQueries && !(COUNTS && w.lengths == nullptr)) {
        const uint64_t per_wave = (uint64_t)di.lds_per_cu / ((uint64_t)tu.blocks_per_cu * waves);
        n_slots = (uint32_t)std::min<uint64_t>(per_wave / sizeof(StageSlot), kMaxStageSlots);
        while (n_slots > 0 && (uint64_t)n_slots * waves * sizeof(StageSlot) > 64 * 1024) --n_slots;
        if (n_slots < 2) n_slots = 0;
    }
    const size_t lds = (size_t)n_slots * waves * sizeof(StageSlot);
    switch (tu.walkers_per_lane) {
        case 2:
            hipLaunchKernelGGL((k_walk_persistent<ALGO, SMP, 2, COUNTS>), dim3(blocks), dim3(threads), lds, s, g, t, w, head,
                               tu.queue_chunk, tu.coop_degree, n_slots);
            break;
        case 4:
            hipLaunchKernelGGL((k_walk_persistent<ALGO, SMP, 4, COUNTS>), dim3(blocks), dim3(threads), lds, s, g, t, w, head,
                               tu.queue_chunk, tu.coop_degree, n_slots);
            break;
        default:
            hipLaunchKernelGGL((k_walk_persistent<ALGO, SMP, 1, COUNTS>), dim3(blocks), dim3(threads), lds, s, g, t, w, head,
                               tu.queue_chunk, tu.coop_degree, n_slots);
    }
    return hipGetLastError();
}

template <uint32_t ALGO, uint32_t SMP>
hipError_t run_bsp(const GraphDev &g, const TableDev &t, const WalkDev &w, const Tuning &tu,
                   const DeviceInfo &di, void *ws, hipStream_t s) {
    constexpr bool kStatic = ALGO == ALG_DEEPWALK || ALGO == ALG_PPR;
    constexpr uint32_t kCarry = !kStatic ? 0u : SMP == SMP_REJ ? 2u : (SMP == SMP_ALIAS || SMP == SMP_NAIVE_ADJ) ? 1u : 0u;
    char *base = reinterpret_cast<char *>(ws);
    uint32_t *counts = reinterpret_cast<uint32_t *>(base);
    const size_t counts_bytes = round_up(sizeof(uint32_t) * (w.max_len + 2));
    Rec *lists[2] = {reinterpret_cast<Rec *>(base + counts_bytes),
                     reinterpret_cast<Rec *>(base + counts_bytes + round_up(sizeof(Rec) * (size_t)w.nq))};
    const uint32_t nfill = w.max_len + 2;
    hipLaunchKernelGGL(k_fill_u32, dim3((nfill + 255) / 256), dim3(256), 0, s, counts, nfill, 0u);
    const uint32_t threads = tu.block_threads;
    uint64_t blocks = (uint64_t)di.num_cus * tu.blocks_per_cu;
    const uint64_t need = ((uint64_t)w.nq + threads - 1) / threads;
    if (blocks > need) blocks = need;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_bsp_init<kCarry>, dim3(blocks), dim3(threads), 0, s, g, t, w, lists[0], counts);
    for (uint32_t k = 0; k < w.max_len; ++k) {
        hipLaunchKernelGGL((k_bsp_step<ALGO, SMP>), dim3(blocks), dim3(threads), 0, s, g, t, w, k,
                           lists[k & 1], counts + k, lists[(k + 1) & 1], counts + k + 1, tu.coop_degree);
    }
    return hipGetLastError();
}

template <uint32_t ALGO, uint32_t SMP>
hipError_t run(const GraphDev &g, const TableDev &t, const WalkDev &w, uint32_t mode, const Tuning &tu,
               const DeviceInfo &di, void *ws, hipStream_t s) {
    return mode == TRW_M_PERSISTENT ? run_persistent<ALGO, SMP>(g, t, w, tu, di, ws, s)
                                    : run_bsp<ALGO, SMP>(g, t, w, tu, di, ws, s);
}

}  // namespace

hipError_t launch_ppr_counts(const GraphDev &g, const TableDev &t, uint32_t sampler, const WalkDev &w,
                             const Tuning &tu, const DeviceInfo &di, void *ws, hipStream_t s) {
    if (w.nq == 0) return hipSuccess;
    switch (sampler) {
        case SMP_NAIVE:
            if (t.adj) return run_persistent<ALG_PPR, SMP_NAIVE_ADJ, true>(g, t, w, tu, di, ws, s);
            return run_persistent<ALG_PPR, SMP_NAIVE, true>(g, t, w, tu, di, ws, s);
        case SMP_ALIAS: return run_persistent<ALG_PPR, SMP_ALIAS, true>(g, t, w, tu, di, ws, s);
        case SMP_REJ: return run_persistent<ALG_PPR, SMP_REJ, true>(g, t, w, tu, di, ws, s);
        default: return run_persistent<ALG_PPR, SMP_ITS, true>(g, t, w, tu, di, ws, s);
    }
}

size_t walk_workspace_bytes(uint32_t mode, uint64_t nq, uint32_t max_len) {
    if (mode == TRW_M_PERSISTENT) return kAlign;
    return round_up(sizeof(uint32_t) * (max_len + 2)) + 2 * round_up(sizeof(Rec) * (size_t)nq);
}

hipError_t launch_walk(const GraphDev &g, const TableDev &t, uint32_t algo, uint32_t sampler,
                       const WalkDev &w, uint32_t mode, const Tuning &tu, const DeviceInfo &di,
                       void *ws, size_t, hipStream_t s) {
    if (w.nq == 0) return hipSuccess;
    if ((algo == ALG_DEEPWALK || algo == ALG_PPR) && sampler == SMP_NAIVE && mode == TRW_M_PERSISTENT &&
        tu.lds_graph && small_graph_fits(g, di))
        return launch_walk_small(g, w, algo, di, ws, s);
    switch (algo) {
        case ALG_DEEPWALK:
            if (sampler == SMP_NAIVE && t.adj) return run<ALG_DEEPWALK, SMP_NAIVE_ADJ>(g, t, w, mode, tu, di, ws, s);
            if (sampler == SMP_NAIVE) return run<ALG_DEEPWALK, SMP_NAIVE>(g, t, w, mode, tu, di, ws, s);
            if (sampler == SMP_ALIAS) return run<ALG_DEEPWALK, SMP_ALIAS>(g, t, w, mode, tu, di, ws, s);
            if (sampler == SMP_REJ) return run<ALG_DEEPWALK, SMP_REJ>(g, t, w, mode, tu, di, ws, s);
            return run<ALG_DEEPWALK, SMP_ITS>(g, t, w, mode, tu, di, ws, s);
        case ALG_PPR:
            if (sampler == SMP_NAIVE && t.adj) return run<ALG_PPR, SMP_NAIVE_ADJ>(g, t, w, mode, tu, di, ws, s);
            if (sampler == SMP_NAIVE) return run<ALG_PPR, SMP_NAIVE>(g, t, w, mode, tu, di, ws, s);
            if (sampler == SMP_ALIAS) return run<ALG_PPR, SMP_ALIAS>(g, t, w, mode, tu, di, ws, s);
            if (sampler == SMP_REJ) return run<ALG_PPR, SMP_REJ>(g, t, w, mode, tu, di, ws, s);
            return run<ALG_PPR, SMP_ITS>(g, t, w, mode, tu, di, ws, s);
        case ALG_NODE2VEC:
            if (t.adj) return run<ALG_NODE2VEC, SMP_OREJ_ADJ>(g, t, w, mode, tu, di, ws, s);
            return run<ALG_NODE2VEC, SMP_OREJ>(g, t, w, mode, tu, di, ws, s);
        default:
            if (t.loff && t.lfused && mode == TRW_M_PERSISTENT)
                return run_persistent<ALG_METAPATH, SMP_LABEL_FUSED>(g, t, w, tu, di, ws, s);
            if (t.loff) return run<ALG_METAPATH, SMP_LABEL_INDEX>(g, t, w, mode, tu, di, ws, s);
            return run<ALG_METAPATH, SMP_ITS>(g, t, w, mode, tu, di, ws, s);
    }
}

}  // namespace trw
