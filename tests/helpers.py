"""Small graphs and checks shared by the tests (test code only)."""
import numpy as np

import synth


def golden_path(name):
    import os
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)


def star(d, weights=None, labels=None):
    """Vertex 0 -> 1..d (directed), each leaf -> 0."""
    edges = [(0, i) for i in range(1, d + 1)] + [(i, 0) for i in range(1, d + 1)]
    w = None if weights is None else list(weights) + [1] * d
    lab = None if labels is None else list(labels) + [0] * d
    return synth.from_edges(d + 1, edges, w, lab)


def undirected(n, pairs, weights=None, labels=None):
    """Both directions of every pair; attributes shared by the two directions."""
    edges, w, lab = [], [], []
    for i, (u, v) in enumerate(pairs):
        edges += [(u, v), (v, u)]
        if weights is not None:
            w += [weights[i]] * 2
        if labels is not None:
            lab += [labels[i]] * 2
    g = synth.from_edges(n, edges, w if weights is not None else None,
                         lab if labels is not None else None)
    g.symmetric = True
    return g


def zoo():
    """Tiny graphs with hand-checkable structure."""
    return {
        # triangle 0-1-2 with a tail 2-3-4 and a chord 1-3 (Node2Vec needs triangles)
        "tri_tail": undirected(5, [(0, 1), (1, 2), (0, 2), (2, 3), (3, 4), (1, 3)],
                               weights=[3, 1, 4, 1, 5, 9], labels=[0, 1, 2, 0, 1, 2]),
        # weighted K4
        "k4": undirected(4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)],
                         weights=[1, 2, 3, 4, 5, 6], labels=[0, 1, 0, 1, 0, 1]),
        # star with 6 leaves, heavy skew in weights
        "star6": undirected(7, [(0, i) for i in range(1, 7)], weights=[1, 1, 2, 3, 5, 200],
                            labels=[0, 1, 2, 0, 1, 2]),
        # path 0-1-2-3-4-5
        "path6": undirected(6, [(i, i + 1) for i in range(5)], weights=[7, 1, 3, 2, 9],
                            labels=[0, 0, 1, 1, 0]),
    }


def edge_index(g, u, v):
    """Position of edge (u, v) in the CSR arrays, or -1."""
    lo, hi = int(g.row_ptr[u]), int(g.row_ptr[u + 1])
    row = g.col[lo:hi]
    i = int(np.searchsorted(row, v))
    return lo + i if i < len(row) and row[i] == v else -1


def transition_matrix(g, use_weights):
    """Row-stochastic first-order transition matrix (float64); dangling rows are zero."""
    P = np.zeros((g.n, g.n))
    for u in range(g.n):
        lo, hi = int(g.row_ptr[u]), int(g.row_ptr[u + 1])
        if hi == lo:
            continue
        w = g.weight[lo:hi].astype(np.float64) if use_weights else np.ones(hi - lo)
        for e, x in zip(range(lo, hi), w):
            P[u, g.col[e]] += x / w.sum()
    return P
