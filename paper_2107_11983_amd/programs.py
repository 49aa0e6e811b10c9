"""Walk programs for the step-centric programming model (Step-centric
Programming: the user picks the walker type and sampling method and writes
Weight, MaxWeight and Update).  Each source defines `struct TrwProgram`
against csrc/program_rt.hpp and is compiled at run time by `Program(source)`.

The four applications of the paper (Random Walk based Algorithms) are given
as programs; they reproduce the built-in walks bit for bit.  Three programs
cover walks the built-ins do not have: Node2Vec on a weighted graph (the
transition weight is the edge weight times the second-order factor), Node2Vec
by dynamic ITS instead of rejection, and a weighted walk by rejection (REJ).
Each of these equals the oracle's walk of the same name bit for bit.

User parameters (params.user) per program:
  deepwalk            none
  ppr                 user[0] = stop threshold (stop after a move iff r2 < it)
  node2vec            user[0..2] = the factors of the transition equation for
                      distance 0, 1, 2 from the previous vertex (1/p, 1, 1/q
                      over their maximum, Q16: trw_walk_params.n2v_thr_q16)
  metapath            user[0] = schema length L (<= 15), user[1..L] = labels
  weighted_node2vec   user[0..2] as node2vec; the bound on the edge weights is
                      p* of the current vertex when a REJ table is passed,
                      else user[3] (at least every edge weight)
  node2vec_its        user[0..2] as node2vec (any non-negative integers)
  weighted_rej        user[0] = a bound on the edge weights (at least every one)
"""

_STATIC = """
struct TrwProgram {{
    static constexpr uint32_t kind = trw_prog::{kind};
    __device__ uint64_t weight(const trw_prog::Walker &, const trw_prog::Graph &, const trw_prog::Params &,
                               uint32_t) const {{ return 0; }}
    __device__ bool update(const trw_prog::Walker &, const trw_prog::Graph &, const trw_prog::Params &p,
                           uint32_t r2) const {{ return {stop}; }}
}};
"""

_KINDS = {"naive": "STATIC_NAIVE", "alias": "STATIC_ALIAS", "its": "STATIC_ITS", "rej": "STATIC_REJ"}


def deepwalk(sampler: str = "alias") -> str:
    """DeepWalk: a static walk of fixed length (max_len moves); sampler naive, alias, its or rej."""
    return _STATIC.format(kind=_KINDS[sampler], stop="false")


def ppr(sampler: str = "alias") -> str:
    """PPR: a static walk that stops after each move with a fixed probability."""
    return _STATIC.format(kind=_KINDS[sampler], stop="r2 < p.user[0]")


# Node2Vec's second-order transition equation: from v, reached from prev, the
# move to x weighs alpha = 1/p, 1 or 1/q as the distance between prev and x is
# 0 (x is prev), 1 (x neighbours prev) or 2.  The first move has no prev.
_N2V_DISTANCE = """
__device__ inline uint32_t n2v_distance(const trw_prog::Walker &w, const trw_prog::Graph &g, int32_t x) {
    if (x == w.prev) return 0u;
    return g.is_neighbor(w.prev, x) ? 1u : 2u;
}
"""

NODE2VEC = _N2V_DISTANCE + """
// Node2Vec with O-REJ: the weight of x is the factor of its distance class,
// user[n2v_distance] (Q16 over the largest factor), bounded by 65536; the
// first move weighs 65536 everywhere (uniform).
struct TrwProgram {
    static constexpr uint32_t kind = trw_prog::DYNAMIC_REJ;
    __device__ uint64_t weight(const trw_prog::Walker &w, const trw_prog::Graph &g, const trw_prog::Params &p,
                               uint32_t slot) const {
        return w.k == 0 ? 65536u : p.user[n2v_distance(w, g, g.col[slot])];
    }
    __device__ uint64_t max_weight(const trw_prog::Walker &, const trw_prog::Graph &,
                                   const trw_prog::Params &) const { return 65536u; }
    __device__ bool update(const trw_prog::Walker &, const trw_prog::Graph &, const trw_prog::Params &,
                           uint32_t) const { return false; }
};
"""

METAPATH = """
// MetaPath: move k may only take an edge whose label is the schema's label
// schema[k mod L]; uniform among those (weights 0 / 1, dynamic ITS).
struct TrwProgram {
    static constexpr uint32_t kind = trw_prog::DYNAMIC_ITS;
    __device__ uint64_t weight(const trw_prog::Walker &w, const trw_prog::Graph &g, const trw_prog::Params &p,
                               uint32_t slot) const {
        return (uint32_t)g.label[slot] == p.user[1 + w.k % p.user[0]] ? 1u : 0u;
    }
    __device__ bool update(const trw_prog::Walker &, const trw_prog::Graph &, const trw_prog::Params &,
                           uint32_t) const { return false; }
};
"""

WEIGHTED_NODE2VEC = _N2V_DISTANCE + """
// Node2Vec on a weighted graph: the weight of edge x is w(x) times the factor
// of its distance class (65536 on the first move), bounded by p* * 65536 with
// p* the row's largest weight (from a REJ table) or user[3].
struct TrwProgram {
    static constexpr uint32_t kind = trw_prog::DYNAMIC_REJ;
    __device__ uint64_t weight(const trw_prog::Walker &w, const trw_prog::Graph &g, const trw_prog::Params &p,
                               uint32_t slot) const {
        const uint64_t f = w.k == 0 ? 65536u : p.user[n2v_distance(w, g, g.col[slot])];
        return f * g.weight[slot];
    }
    __device__ uint64_t max_weight(const trw_prog::Walker &w, const trw_prog::Graph &g,
                                   const trw_prog::Params &p) const {
        return (uint64_t)(g.pmax ? w.pm : p.user[3]) << 16;
    }
    __device__ bool update(const trw_prog::Walker &, const trw_prog::Graph &, const trw_prog::Params &,
                           uint32_t) const { return false; }
};
"""

NODE2VEC_ITS = _N2V_DISTANCE + """
// Node2Vec by dynamic ITS instead of rejection (the paper's default sampler
// for dynamic walks): every move weighs the whole row with the factors of the
// distance classes, user[0..2] (65536 everywhere on the first move), and
// draws one slot in proportion.
struct TrwProgram {
    static constexpr uint32_t kind = trw_prog::DYNAMIC_ITS;
    __device__ uint64_t weight(const trw_prog::Walker &w, const trw_prog::Graph &g, const trw_prog::Params &p,
                               uint32_t slot) const {
        return w.k == 0 ? 65536u : p.user[n2v_distance(w, g, g.col[slot])];
    }
    __device__ bool update(const trw_prog::Walker &, const trw_prog::Graph &, const trw_prog::Params &,
                           uint32_t) const { return false; }
};
"""

WEIGHTED_REJ = """
// A weighted static walk by rejection (REJ; Sampling Methods): darts at
// uniform slots, accepted with probability w(e) / bound, so a move follows e
// with probability proportional to w(e) without building a table.  The bound
// is p* of the current vertex when a REJ table is passed, else user[0].
struct TrwProgram {
    static constexpr uint32_t kind = trw_prog::DYNAMIC_REJ;
    __device__ uint64_t weight(const trw_prog::Walker &, const trw_prog::Graph &g, const trw_prog::Params &,
                               uint32_t slot) const {
        return g.weight[slot];
    }
    __device__ uint64_t max_weight(const trw_prog::Walker &w, const trw_prog::Graph &g,
                                   const trw_prog::Params &p) const {
        return g.pmax ? w.pm : p.user[0];
    }
    __device__ bool update(const trw_prog::Walker &, const trw_prog::Graph &, const trw_prog::Params &,
                           uint32_t) const { return false; }
};
"""
