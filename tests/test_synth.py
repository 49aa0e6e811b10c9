"""The seeded input generator: R-MAT CSR well-formedness and determinism."""
import numpy as np

import synth


def test_rmat_csr_wellformed(synth_lib):
    for sym in (True, False):
        g = synth.rmat(11, 10, sym, 1234)
        assert g.row_ptr[0] == 0 and (np.diff(g.row_ptr) >= 0).all()
        assert g.col.min() >= 0 and g.col.max() < g.n
        src = np.repeat(np.arange(g.n), g.degrees())
        assert (src != g.col).all()                                  # no self-loops
        key = src.astype(np.int64) * g.n + g.col
        assert (np.diff(key) > 0).all()                              # sorted rows, no duplicates
        if sym:
            rev = np.sort(g.col.astype(np.int64) * g.n + src)
            assert np.array_equal(rev, key)
        assert g.m <= g.n * 10


def test_rmat_is_skewed_and_permuted(synth_lib):
    g = synth.rmat(14, 16, True, 77)
    deg = g.degrees()
    assert deg.max() > 20 * deg.mean()                   # power-law-like hubs
    top = np.argsort(deg)[-16:]
    assert top.min() > 64                                # hubs are not clustered at low ids


def test_attrs_symmetric_and_in_range(synth_lib):
    g = synth.rmat(10, 12, True, 5)
    synth.attach_attrs(g, 9, weights=True, labels=5)
    assert g.weight.min() >= 1 and g.weight.max() <= 255
    assert set(np.unique(g.label)) == {0, 1, 2, 3, 4}
    src = np.repeat(np.arange(g.n), g.degrees())
    fwd = dict(zip(zip(src.tolist(), g.col.tolist()), zip(g.weight.tolist(), g.label.tolist())))
    for (u, v), a in list(fwd.items())[:5000]:
        assert fwd[(v, u)] == a


def test_deterministic(synth_lib):
    a = synth.rmat(12, 8, False, 42)
    b = synth.rmat(12, 8, False, 42)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
    assert np.array_equal(synth.sources(1000, 4096, 3), synth.sources(1000, 4096, 3))
    s = synth.sources(100000, 1000, 8)
    assert s.min() >= 0 and s.max() < 1000
