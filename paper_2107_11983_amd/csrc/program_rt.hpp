// Walk programs: the step-centric programming model (Step-centric
// Programming) as a device template.  A program says how a walk moves and
// when it stops; the framework runs it over a batch of queries with the same
// schedule, random contract and outputs as the built-in walks:
//
//   struct TrwProgram {
//       static constexpr uint32_t kind = trw_prog::DYNAMIC_REJ;   // the sampling method
//       // Weight (the paper's Weight): the transition weight of edge slot
//       // `slot` of the current row (to g.col[slot]; g.weight[slot],
//       // g.label[slot] when the graph has them) for the walker as it
//       // stands.  Used by DYNAMIC_REJ and DYNAMIC_ITS; a row's weights must
//       // sum below 2^64.
//       __device__ uint64_t weight(const trw_prog::Walker &w, const trw_prog::Graph &g,
//                                  const trw_prog::Params &p, uint32_t slot) const;
//       // MaxWeight (DYNAMIC_REJ only): a bound on weight() over the current
//       // row; 0 means the row has no transition (the walk ends, DEAD_END).
//       __device__ uint64_t max_weight(const trw_prog::Walker &w, const trw_prog::Graph &g,
//                                      const trw_prog::Params &p) const;
//       // Update after a move (w already at the new vertex, w.k moves made):
//       // true ends the walk (status STOPPED).  r2 is the step's third random word
//       // (for the rejection kinds: that of the dart that was accepted).
//       __device__ bool update(const trw_prog::Walker &w, const trw_prog::Graph &g,
//                              const trw_prog::Params &p, uint32_t r2) const;
//   };
//
// Sampling methods (Sampling Methods; a move draws Philox4x32-10 with counter
// (k, t, qid) and key seed, words r0..r3):
//   STATIC_NAIVE  uniform slot mulhi32(r0, d)                      (no table)
//   STATIC_ALIAS  the ALIAS table's bucket mulhi32(r0, d), coin r1  (ALIAS table)
//   STATIC_ITS    x = high half of (r1:r0) * W, first prefix > x    (ITS table)
//   STATIC_REJ    darts t = 0, 1, ...: slot mulhi32(r0, d), accept iff
//                 r1 * p*_v < w * 2^32, p*_v the row's largest weight (REJ table)
//   DYNAMIC_REJ   darts t = 0, 1, ...: slot mulhi32(r0, d), accept iff
//                 r1 * MaxWeight < Weight(slot) * 2^32, compared exactly (the
//                 dart height y = r1 * MaxWeight / 2^32 is uniform in
//                 [0, MaxWeight); the move is taken iff y < Weight)
//   DYNAMIC_ITS   weights of the row computed on the fly, W their sum; the
//                 draw j = mulhi32(r0, W) while W < 2^32, else the high half
//                 of (r1:r0) * W; the slot whose running-sum range holds j
// A walk ends after max_len moves (LENGTH), when update says so (STOPPED,
// checked first), or when the row has no transition (DEAD_END).  DeepWalk,
// PPR, Node2Vec and MetaPath written as programs give the built-in walks'
// paths bit for bit.
#pragma once

#include "trw_device.hpp"

namespace trw_prog {

using trw::alias_pick;
using trw::eset_has;
using trw::its_search;
using trw::lane_id;
using trw::PathBuf;
using trw::philox;
using trw::Rand4;
using trw::rank_below;
using trw::scale32;
using trw::scale64;

enum : uint32_t { STATIC_NAIVE = 0, STATIC_ALIAS = 1, STATIC_ITS = 2, DYNAMIC_REJ = 3, DYNAMIC_ITS = 4,
                  STATIC_REJ = 5 };
enum : uint8_t { ST_LENGTH = 1, ST_STOPPED = 2, ST_DEAD_END = 3, ST_BAD_SOURCE = 4 };
constexpr uint32_t kIdle = 0xFFFFFFFFu;
constexpr uint32_t kMaxDarts = 1u << 24;   // the last dart of a move is accepted (as the built-ins)

struct Graph {
    const int32_t *row_ptr;
    const int32_t *col;
    const uint32_t *weight;             // NULL when the graph has none
    const uint8_t *label;               // NULL when the graph has none
    int32_t n, m;
    uint32_t symmetric;
    uint32_t pad;
    const unsigned long long *eset;     // edge index hash set, or NULL
    unsigned long long eset_mask;
    const uint32_t *pmax;               // with a REJ table: p* per vertex (its row's largest weight), else NULL

    __device__ int32_t row_off(int32_t v) const { return row_ptr[v]; }
    __device__ uint32_t degree(int32_t v) const { return (uint32_t)(row_ptr[v + 1] - row_ptr[v]); }
    // Is v a neighbour of u (edge u -> v)?  The edge index when there is one,
    // else binary search in u's sorted row.
    __device__ bool is_neighbor(int32_t u, int32_t v) const {
        if (eset) return eset_has(eset, eset_mask, u, v);
        int32_t lo = row_ptr[u], hi = row_ptr[u + 1];
        while (lo < hi) {
            const int32_t mid = lo + ((hi - lo) >> 1);
            const int32_t c = col[mid];
            if (c == v) return true;
            if (c < v) lo = mid + 1; else hi = mid;
        }
        return false;
    }
};

struct Walker {
    uint64_t qid;
    uint32_t k;            // moves made
    int32_t src, cur, prev;   // prev = -1 before the first move
    int32_t off;           // cur's row
    uint32_t deg;
    uint32_t pm;           // with a REJ table (g.pmax): p* of cur (its row's largest weight), else 0
};

struct Params {
    uint32_t max_len;      // moves, 1..65535
    uint32_t pad;
    uint64_t seed;
    uint32_t user[16];     // the program's own parameters
};

struct Args {
    Graph g;
    const uint4 *alias;            // STATIC_ALIAS: 32-byte entries per slot
    const uint64_t *prefix;        // STATIC_ITS: inclusive prefix per row
    const uint4 *rej;              // STATIC_REJ: 32-byte slot records {w, dst, row(dst)}, {p*(dst), ...}
    const int32_t *sources;
    uint32_t nq, chunk;
    uint64_t qid_base;
    int32_t *paths;
    uint64_t stride;
    uint32_t *lengths;
    uint8_t *status;
    unsigned long long *head;      // queue head, zero at launch
    Params p;
};

// DYNAMIC_ITS's draw in [0, W): mulhi32(r0, W) while W fits 32 bits (so a
// 0/1 weighting picks the j-th match exactly as the built-in MetaPath does),
// else the high half of the 64-bit word (r1:r0) times W.
__device__ __forceinline__ uint64_t dynamic_its_draw(uint32_t r0, uint32_t r1, uint64_t W) {
    return W < (1ull << 32) ? (uint64_t)scale32(r0, (uint32_t)W) : scale64(r0, r1, W);
}

// One move of walker w under program P; returns the next vertex or -1.  For
// the rejection kinds r ends as the accepted dart's block.
template <class P>
__device__ __forceinline__ int32_t program_move(const P &prog, const Args &a, const Walker &w, Rand4 &r,
                                                int32_t &noff, uint32_t &ndeg, uint32_t &npm) {
    const Graph &g = a.g;
    if (w.deg == 0) return -1;
    int32_t nxt = -1;
    if constexpr (P::kind == STATIC_NAIVE) {
        nxt = g.col[w.off + scale32(r.r0, w.deg)];
    } else if constexpr (P::kind == STATIC_ALIAS) {
        const uint64_t e = (uint64_t)(w.off + scale32(r.r0, w.deg));
        int32_t o, d;
        // the whole 32-byte entry in one read, then the pick (picking from the
        // loads lets the compiler read the threshold first, then the half)
        const uint4 e0 = a.alias[2 * e], e1 = a.alias[2 * e + 1];
        asm volatile("" ::"v"(e0.x), "v"(e0.y), "v"(e0.z), "v"(e1.x), "v"(e1.y), "v"(e1.z), "v"(e1.w));
        nxt = alias_pick(e0, e1, r.r1, o, d);
        if (nxt >= 0) { noff = o; ndeg = (uint32_t)d; }
        return nxt;
    } else if constexpr (P::kind == STATIC_ITS) {
        const uint64_t *pr = a.prefix + w.off;
        const uint64_t W = pr[w.deg - 1];
        if (W == 0) return -1;
        const uint64_t x = scale64(r.r0, r.r1, W);
        nxt = g.col[w.off + its_search(pr, w.deg, x, ((uint64_t)r.r1 << 32) | r.r0)];
    } else if constexpr (P::kind == STATIC_REJ) {
        if (w.pm == 0) return -1;
        for (uint32_t t = 0;; ++t) {
            if (t > 0) r = philox(w.k, t, w.qid, a.p.seed);
            const uint64_t e = (uint64_t)(uint32_t)w.off + scale32(r.r0, w.deg);
            const uint4 rec = a.rej[2 * e];
            if (t + 1 == kMaxDarts || (uint64_t)r.r1 * w.pm < ((uint64_t)rec.x << 32)) {
                noff = (int32_t)rec.z;
                ndeg = rec.w;
                npm = a.rej[2 * e + 1].x;
                return (int32_t)rec.y;
            }
        }
    } else if constexpr (P::kind == DYNAMIC_REJ) {
        const uint64_t bound = prog.max_weight(w, g, a.p);
        if (bound == 0) return -1;
        for (uint32_t t = 0;; ++t) {
            if (t > 0) r = philox(w.k, t, w.qid, a.p.seed);
            const uint32_t slot = (uint32_t)w.off + scale32(r.r0, w.deg);
            if (t + 1 == kMaxDarts ||
                (unsigned __int128)r.r1 * bound < ((unsigned __int128)prog.weight(w, g, a.p, slot) << 32)) {
                nxt = g.col[slot];
                break;
            }
        }
    } else {   // DYNAMIC_ITS, rows below kCoopSlots (longer rows: wave_its_moves)
        uint64_t W = 0;
        for (uint32_t i = 0; i < w.deg; ++i) W += prog.weight(w, g, a.p, (uint32_t)w.off + i);
        if (W == 0) return -1;
        const uint64_t j = dynamic_its_draw(r.r0, r.r1, W);
        uint64_t acc = 0;
        for (uint32_t i = 0; i < w.deg; ++i) {
            const uint32_t slot = (uint32_t)w.off + i;
            acc += prog.weight(w, g, a.p, slot);
            if (j < acc) { nxt = g.col[slot]; break; }
        }
    }
    if (nxt >= 0) {
        noff = g.row_ptr[nxt];
        ndeg = (uint32_t)(g.row_ptr[nxt + 1] - noff);
        if (g.pmax) npm = g.pmax[nxt];
    }
    return nxt;
}

// DYNAMIC_ITS on rows of at least kCoopSlots slots: the whole wave takes
// such walkers one at a time; per round each lane weighs 4 consecutive slots
// (256 per round).  A wave-wide sum gives W; a second pass with a running
// scan finds the slot holding j = mulhi32(r0, W): the same choice as the
// lane scan.
constexpr uint32_t kCoopSlots = 128;

template <typename T>
__device__ __forceinline__ T wave_scan(T v) {             // inclusive, over the 64 lanes
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T t = __shfl_up(v, o);
        if (lane_id() >= (uint32_t)o) v += t;
    }
    return v;
}

template <class P>
__device__ __forceinline__ void wave_its_moves(const P &prog, const Args &a, const Walker &w, const Rand4 &r,
                                               bool mine, int32_t &nxt) {
    const Graph &g = a.g;
    const uint32_t lane = lane_id();
    uint64_t owners = __ballot(mine);
    while (owners != 0) {
        const int o = __builtin_ctzll(owners);
        owners &= owners - 1;
        Walker v;                                    // the owner's walker, in every lane
        v.qid = __shfl(w.qid, o); v.k = __shfl(w.k, o); v.src = __shfl(w.src, o);
        v.cur = __shfl(w.cur, o); v.prev = __shfl(w.prev, o); v.off = __shfl(w.off, o);
        v.deg = __shfl(w.deg, o); v.pm = __shfl(w.pm, o);
        const uint32_t r0 = __shfl(r.r0, o), r1 = __shfl(r.r1, o);
        uint64_t W = 0;
        for (uint32_t base = 0; base < v.deg; base += 256) {
            uint64_t part = 0;
#pragma unroll
            for (uint32_t q = 0; q < 4; ++q) {
                const uint32_t i = base + 4 * lane + q;
                if (i < v.deg) part += prog.weight(v, g, a.p, (uint32_t)v.off + i);
            }
            W += __shfl(wave_scan(part), 63);
        }
        int32_t pick = -1;
        if (W != 0) {
            const uint64_t j = dynamic_its_draw(r0, r1, W);
            uint64_t acc = 0;
            for (uint32_t base = 0; base < v.deg; base += 256) {
                uint32_t wq[4];
                uint64_t part = 0;
#pragma unroll
                for (uint32_t q = 0; q < 4; ++q) {
                    const uint32_t i = base + 4 * lane + q;
                    wq[q] = i < v.deg ? prog.weight(v, g, a.p, (uint32_t)v.off + i) : 0u;
                    part += wq[q];
                }
                const uint64_t incl = acc + wave_scan(part);          // running sum through this lane's 4
                const uint64_t hit = __ballot(j < incl);
                if (hit != 0) {
                    const int hl = __builtin_ctzll(hit);
                    // in the first lane whose slots reach past j: which of its 4
                    uint64_t run = incl - part;
                    int32_t choice = -1;
#pragma unroll
                    for (uint32_t q = 0; q < 4; ++q) {
                        const uint32_t i = base + 4 * lane + q;
                        run += wq[q];
                        if (choice < 0 && i < v.deg && j < run) choice = g.col[v.off + i];
                    }
                    pick = __shfl(choice, hl);
                    break;
                }
                acc = __shfl(incl, 63);
            }
        }
        if (lane == (uint32_t)o) nxt = pick;
    }
}

// The batch: one walker per lane; each wave claims `chunk` query ids at a
// time from the queue head and refills lanes whose walk ended.
template <class P>
__device__ void run(const Args &a) {
    const P prog{};
    const Graph &g = a.g;
    const uint32_t lane = lane_id();
    Walker w{};
    uint32_t qi = kIdle;
    PathBuf path;
    uint32_t pool_next = 0, pool_end = 0;
    bool exhausted = false;
    for (;;) {
        uint64_t idle = __ballot(qi == kIdle);
        while (idle != 0 && !exhausted) {
            uint32_t avail = pool_end - pool_next;
            if (avail == 0) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(a.head, (unsigned long long)a.chunk);
                base = __shfl(base, 0);
                if (base >= a.nq) { exhausted = true; break; }
                pool_next = (uint32_t)base;
                pool_end = (uint32_t)min(base + a.chunk, (unsigned long long)a.nq);
                avail = pool_end - pool_next;
            }
            const uint32_t rk = rank_below(idle);
            if (((idle >> lane) & 1ull) && rk < avail) {
                const uint32_t q = pool_next + rk;
                const int32_t s = a.sources[q];
                if (s < 0 || s >= g.n) {
                    a.lengths[q] = 0;
                    a.status[q] = ST_BAD_SOURCE;
                } else {
                    qi = q;
                    w.qid = a.qid_base + q; w.k = 0; w.src = s; w.cur = s; w.prev = -1;
                    w.off = g.row_ptr[s]; w.deg = (uint32_t)(g.row_ptr[s + 1] - w.off);
                    if (g.pmax) w.pm = g.pmax[s];
                    path.start(a.paths + (uint64_t)q * a.stride);
                    path.push(s);
                }
            }
            pool_next += min((uint32_t)__popcll(idle), avail);
            idle = __ballot(qi == kIdle);
        }
        if (__ballot(qi != kIdle) == 0) break;
        Rand4 r = philox(w.k, 0, w.qid, a.p.seed);
        const bool coop = P::kind == DYNAMIC_ITS && qi != kIdle && w.deg >= kCoopSlots;
        int32_t nxt = -1;
        if (P::kind == DYNAMIC_ITS) wave_its_moves(prog, a, w, r, coop, nxt);   // whole wave, uniform
        if (qi != kIdle) {
            int32_t noff = 0;
            uint32_t ndeg = 0, npm = 0;
            if (!coop) {
                nxt = program_move(prog, a, w, r, noff, ndeg, npm);
            } else if (nxt >= 0) {
                noff = g.row_ptr[nxt]; ndeg = (uint32_t)(g.row_ptr[nxt + 1] - noff);
                if (g.pmax) npm = g.pmax[nxt];
            }
            uint8_t st = 0;
            if (nxt < 0) {
                st = ST_DEAD_END;
            } else {
                path.push(nxt);
                w.prev = w.cur; w.cur = nxt; w.off = noff; w.deg = ndeg; w.pm = npm; w.k += 1;
                if (prog.update(w, g, a.p, r.r2)) st = ST_STOPPED;
                else if (w.k == a.p.max_len) st = ST_LENGTH;
            }
            if (st) {
                path.flush();
                a.lengths[qi] = w.k;
                a.status[qi] = st;
                qi = kIdle;
            }
        }
    }
}

}  // namespace trw_prog
