"""Pins for the oracle's per-vertex sampling tables (preprocessing of static walks).

ALIAS [Sampling Methods, alias sampling]: hand-worked Vose tables, and for
random rows the exact mass identity of a Walker table -- every element j gets
exactly w_j / W of the probability, summed over its own column and the
columns that alias to it -- up to the 2^-32 quantisation of each coin.
ITS [Sampling Methods, inverse transformation]: per-row prefix = numpy.cumsum.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import golden_path


def _rows_graph(weight_rows):
    rp = np.zeros(len(weight_rows) + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in weight_rows])
    w = np.concatenate([np.asarray(r, dtype=np.uint32) for r in weight_rows]) if weight_rows else np.zeros(0, np.uint32)
    return rp, w


def _golden_alias():
    cases, cur = [], {}
    for line in open(golden_path("alias_worked_examples.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, val = line.split("=")
        cur[key] = [int(x) for x in val.split()]
        if key == "alias":
            cases.append(cur)
            cur = {}
    return cases


def test_alias_worked_examples(oracle_lib):
    cases = _golden_alias()
    assert len(cases) == 5
    rp, w = _rows_graph([c["weights"] for c in cases])
    thr, alias = oracle.alias_build(rp, w)
    for i, c in enumerate(cases):
        lo, hi = rp[i], rp[i + 1]
        assert list(thr[lo:hi]) == c["thr"], c
        assert list(alias[lo:hi]) == c["alias"], c


def _mass_identity(w, thr, alias):
    """Check sum over columns of the mass each gives element j against w_j*d/W (exact ints)."""
    d = len(w)
    W = int(sum(int(x) for x in w))
    two32 = 1 << 32
    mass = [0] * d                      # in units of 2^-32 of one column
    naliased = [0] * d
    for x in range(d):
        a = int(alias[x])
        assert 0 <= a < d
        if a == x:                       # full bucket: all of the column is x
            assert int(thr[x]) == 0xFFFFFFFF
            mass[x] += two32
        else:
            mass[x] += int(thr[x])
            mass[a] += two32 - int(thr[x])
            naliased[a] += 1
    for j in range(d):
        target_num = int(w[j]) * d * two32     # mass_j should be target_num / W
        err = abs(mass[j] * W - target_num)
        # each quantised coin is off by < 1 unit; j's own column and every column aliasing to j
        assert err <= (1 + naliased[j]) * W, (j, mass[j], target_num / W)


@pytest.mark.parametrize("wmax", [1, 3, 255, 2**32 - 1])
def test_alias_mass_identity_random_rows(oracle_lib, wmax):
    rng = np.random.default_rng(wmax)
    rows = []
    for _ in range(300):
        d = int(rng.integers(1, 200))
        rows.append(rng.integers(1, wmax + 1, size=d, dtype=np.uint64).astype(np.uint32))
    rows.append(np.array([1], np.uint32))
    rows.append(np.array([2**32 - 1] * 5 + [1], np.uint32))
    rp, w = _rows_graph(rows)
    thr, alias = oracle.alias_build(rp, w)
    for i, r in enumerate(rows):
        lo, hi = rp[i], rp[i + 1]
        _mass_identity(r, thr[lo:hi], alias[lo:hi])


def test_alias_uniform_weights_are_full_buckets(oracle_lib):
    rows = [[7] * d for d in (1, 2, 5, 64, 1000)]
    rp, w = _rows_graph(rows)
    thr, alias = oracle.alias_build(rp, w)
    assert (thr == 0xFFFFFFFF).all()
    for i in range(len(rows)):
        lo, hi = rp[i], rp[i + 1]
        assert (alias[lo:hi] == np.arange(hi - lo)).all()


def test_alias_zero_weights(oracle_lib):
    # zero-weight edges are never chosen; an all-zero row is marked as having no transition
    rows = [[0, 0, 0], [0, 5, 0, 5], [0]]
    rp, w = _rows_graph(rows)
    thr, alias = oracle.alias_build(rp, w)
    assert (alias[0:3] == -1).all() and (alias[7:8] == -1).all()
    _mass_identity(np.array(rows[1]), thr[3:7], alias[3:7])


def test_alias_scale_invariant(oracle_lib):
    rng = np.random.default_rng(7)
    rows = [rng.integers(1, 256, size=int(rng.integers(1, 60))).astype(np.uint32) for _ in range(100)]
    rp, w = _rows_graph(rows)
    t1, a1 = oracle.alias_build(rp, w)
    t2, a2 = oracle.alias_build(rp, w * np.uint32(12345))
    assert np.array_equal(t1, t2) and np.array_equal(a1, a2)


def test_its_prefix_is_cumsum(oracle_lib):
    g = synth.rmat(10, 8, False, 99)
    synth.attach_attrs(g, 3, weights=True, w_range=(1, 2**32 - 1))
    prefix = oracle.its_build(g.row_ptr, g.weight)
    for v in range(g.n):
        lo, hi = g.row_ptr[v], g.row_ptr[v + 1]
        assert np.array_equal(prefix[lo:hi], np.cumsum(g.weight[lo:hi].astype(np.uint64)))
