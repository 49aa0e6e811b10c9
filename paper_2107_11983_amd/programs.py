"""Walk programs for the step-centric programming model (Step-centric
Programming: the user picks the walker type and sampling method and writes
Weight and Update).  Each source defines `struct TrwProgram` against
csrc/program_rt.hpp and is compiled at run time by `Program(source)`.

The four applications of the paper (Random Walk based Algorithms) are given
as programs; they reproduce the built-in walks bit for bit.  Three programs
cover walks the built-ins do not have: Node2Vec on a weighted graph (the
transition weight is the edge weight times the second-order factor), Node2Vec
by dynamic ITS instead of rejection, and a weighted walk by rejection (REJ).

User parameters (params.user) per program:
  deepwalk            none
  ppr                 user[0] = stop threshold (stop after a move iff r2 < it)
  node2vec            user[0..2] = Q16 acceptance for x == prev, x adjacent to
                      prev, otherwise (as trw_walk_params.n2v_thr_q16)
  metapath            user[0] = schema length L (<= 15), user[1..L] = labels
  weighted_node2vec   user[0..2] as node2vec, user[3] = the largest edge weight
  node2vec_its        user[0..2] as node2vec (weights, any positive integers)
  weighted_rej        user[0] = a bound on the edge weights
"""

_STATIC = """
struct TrwProgram {{
    static constexpr uint32_t kind = trw_prog::{kind};
    __device__ uint32_t weight(const trw_prog::Walker &, const trw_prog::Graph &, const trw_prog::Params &,
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


NODE2VEC = """
// Node2Vec (the second-order transition equation) with O-REJ: the first move
// is uniform; then x == prev, x adjacent to prev, other x accept with the
// thresholds in user[0..2] (the factors 1/p, 1, 1/q over their maximum, Q16).
struct TrwProgram {
    static constexpr uint32_t kind = trw_prog::DYNAMIC_REJ;
    __device__ uint32_t weight(const trw_prog::Walker &w, const trw_prog::Graph &g, const trw_prog::Params &p,
                               uint32_t slot) const {
        if (w.k == 0) return 65536u;
        const int32_t x = g.col[slot];
        if (x == w.prev) return p.user[0];
        return g.is_neighbor(w.prev, x) ? p.user[1] : p.user[2];
    }
    __device__ bool update(const trw_prog::Walker &, const trw_prog::Graph &, const trw_prog::Params &,
                           uint32_t) const { return false; }
};
"""

METAPATH = """
// MetaPath: move k may only take an edge whose label is the schema's label
// schema[k mod L]; uniform among those (weights 0 / 1, dynamic ITS).
struct TrwProgram {
    static constexpr uint32_t kind = trw_prog::DYNAMIC_ITS;
    __device__ uint32_t weight(const trw_prog::Walker &w, const trw_prog::Graph &g, const trw_prog::Params &p,
                               uint32_t slot) const {
        return (uint32_t)g.label[slot] == p.user[1 + w.k % p.user[0]] ? 1u : 0u;
    }
    __device__ bool update(const trw_prog::Walker &, const trw_prog::Graph &, const trw_prog::Params &,
                           uint32_t) const { return false; }
};
"""

WEIGHTED_NODE2VEC = """
// Node2Vec on a weighted graph: the transition weight is w(e) times the
// second-order factor; with O-REJ the acceptance is that over its maximum,
// factor_q16 * w(e) / w_max (w_max = user[3], the largest edge weight).
struct TrwProgram {
    static constexpr uint32_t kind = trw_prog::DYNAMIC_REJ;
    __device__ uint32_t weight(const trw_prog::Walker &w, const trw_prog::Graph &g, const trw_prog::Params &p,
                               uint32_t slot) const {
        uint32_t f = 65536u;
        const int32_t x = g.col[slot];
        if (w.k != 0) f = (x == w.prev) ? p.user[0] : (g.is_neighbor(w.prev, x) ? p.user[1] : p.user[2]);
        return (uint32_t)(((uint64_t)f * g.weight[slot]) / p.user[3]);
    }
    __device__ bool update(const trw_prog::Walker &, const trw_prog::Graph &, const trw_prog::Params &,
                           uint32_t) const { return false; }
};
"""

NODE2VEC_ITS = """
// Node2Vec with dynamic ITS instead of rejection (the paper's default sampler
// for dynamic walks): every step weighs the whole row with the second-order
// factors of user[0..2] (Q16) and draws one slot in proportion.
struct TrwProgram {
    static constexpr uint32_t kind = trw_prog::DYNAMIC_ITS;
    __device__ uint32_t weight(const trw_prog::Walker &w, const trw_prog::Graph &g, const trw_prog::Params &p,
                               uint32_t slot) const {
        if (w.k == 0) return 1u;
        const int32_t x = g.col[slot];
        if (x == w.prev) return p.user[0];
        return g.is_neighbor(w.prev, x) ? p.user[1] : p.user[2];
    }
    __device__ bool update(const trw_prog::Walker &, const trw_prog::Graph &, const trw_prog::Params &,
                           uint32_t) const { return false; }
};
"""

WEIGHTED_REJ = """
// A weighted static walk by rejection (REJ; Sampling Methods): darts at
// uniform slots, accepted with probability w(e) / w_max (w_max = user[0], a
// bound on every edge weight), so a move follows e with probability
// proportional to w(e) without any table.
struct TrwProgram {
    static constexpr uint32_t kind = trw_prog::DYNAMIC_REJ;
    __device__ uint32_t weight(const trw_prog::Walker &, const trw_prog::Graph &g, const trw_prog::Params &p,
                               uint32_t slot) const {
        return (uint32_t)(((uint64_t)g.weight[slot] << 16) / p.user[0]);
    }
    __device__ bool update(const trw_prog::Walker &, const trw_prog::Graph &, const trw_prog::Params &,
                           uint32_t) const { return false; }
};
"""
