"""The seeded input generator: deterministic, well-formed, shaped as stated."""
import numpy as np

from paper_2507_20441_amd import workloads as W


def _well_formed(g):
    assert g.src.dtype == np.int32 and g.dst.dtype == np.int32 and g.t.dtype == np.int64
    assert (g.src != g.dst).all()
    assert g.src.min() >= 0 and g.src.max() < g.n and g.dst.min() >= 0 and g.dst.max() < g.n
    key = np.lexsort((g.t, g.dst, g.src))
    s, d, t = g.src[key], g.dst[key], g.t[key]
    assert not ((s[1:] == s[:-1]) & (d[1:] == d[:-1]) & (t[1:] == t[:-1])).any()


def test_tiny_is_deterministic_and_well_formed():
    a, b = W.tiny_graph(), W.tiny_graph()
    assert a.m == 20_000 and a.n == 1000
    assert (a.src == b.src).all() and (a.t == b.t).all()
    _well_formed(a)
    assert a.t.min() >= 0 and a.t.max() <= 100_000
    # power-law: the top vertex carries far more than the average degree
    assert np.bincount(a.src, minlength=a.n).max() > 20 * (a.m / a.n)


def test_bursty_small_graph():
    g = W.small_graph(50_000, 3, span=1_000_000)
    _well_formed(g)
    assert g.t.min() >= 0 and g.t.max() < 1_000_000
    # bursty: gaps between a busy source's consecutive edges are heavy-tailed
    busiest = np.bincount(g.src).argmax()
    gaps = np.diff(np.sort(g.t[g.src == busiest]))
    assert gaps.max() > 20 * max(1.0, np.median(gaps))


def test_reciprocal_edges():
    g = W.chung_lu_graph(500, 5000, 2.0, seed=4, times="bursty", span=100_000, reciprocal=500)
    _well_formed(g)
    assert g.m == 5000


def test_batched_jobs_spec():
    jobs = W.batched_jobs()
    assert len(jobs) == 64
    for j in jobs:
        assert 1e4 * 0.99 <= j["m"] <= 5e6 * 1.01
        assert 600 <= j["delta"] <= 86400
        assert 1e5 * 0.99 <= j["k"] <= 1e7 * 1.01
        assert j["motif"] in W.MOTIFS
