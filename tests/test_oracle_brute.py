"""Pins for the brute-force exact counter C (Def. "temporal match").

Hand-worked fixtures, closed forms, an independent pure-Python enumeration on
tiny inputs, and invariances (relabelling, time shift, monotonicity in delta).
"""
import itertools

import numpy as np
import pytest

import oracle as O
from golden_io import load
from paper_2507_20441_amd import workloads as W


@pytest.mark.parametrize("name", ["cycle3_hand.txt", "star2_hand.txt"])
def test_hand_worked_counts(name):
    fx = load(name)
    g = O.Graph(fx["src"], fx["dst"], fx["t"], fx["n"])
    mo = O.make_motif(fx["motif"], fx["delta"])
    assert g.brute_count(mo) == fx["expect_count"]


def python_count(src, dst, t, motif, delta):
    """Def. "temporal match" by exhaustive enumeration of ordered edge tuples."""
    m = len(src)
    k = 1 + max(max(e) for e in motif)
    cnt = 0
    for tup in itertools.permutations(range(m), len(motif)):
        ts = [t[i] for i in tup]
        if any(not ts[a] < ts[a + 1] for a in range(len(ts) - 1)):
            continue
        if ts[-1] - ts[0] > delta:
            continue
        img = [None] * k
        ok = True
        for (x, y), i in zip(motif, tup):
            for z, gv in ((x, src[i]), (y, dst[i])):
                if img[z] is None:
                    img[z] = gv
                elif img[z] != gv:
                    ok = False
        if ok and len(set(img)) == k:
            cnt += 1
    return cnt


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("motif", [W.MOTIFS["3cycle"], ((0, 1), (1, 2), (0, 2)),
                                   ((0, 1), (1, 0), (0, 1)), ((0, 1), (2, 1))])
def test_matches_python_enumeration(seed, motif):
    g = W.small_graph(22, seed, n=5, span=40)
    delta = 12
    G = O.Graph(g.src, g.dst, g.t, g.n)
    want = python_count(g.src.tolist(), g.dst.tolist(), g.t.tolist(), motif, delta)
    assert G.brute_count(O.make_motif(motif, delta)) == want


def test_single_edge_motif_counts_every_edge():
    g = W.small_graph(500, 3)
    G = O.Graph(g.src, g.dst, g.t, g.n)
    assert G.brute_count(O.make_motif([(0, 1)], 5)) == g.m


@pytest.mark.parametrize("seed", range(4))
def test_two_path_closed_form(seed):
    """a->b then b->c: for each first edge (x, y, t1), the out-edges of y with
    time in (t1, t1 + delta] whose head is not x."""
    g = W.small_graph(400, seed, n=30, span=600)
    delta = 40
    C = 0
    for x, y, t1 in zip(g.src, g.dst, g.t):
        sel = (g.src == y) & (g.t > t1) & (g.t <= t1 + delta) & (g.dst != x)
        C += int(sel.sum())
    G = O.Graph(g.src, g.dst, g.t, g.n)
    assert G.brute_count(O.make_motif([(0, 1), (1, 2)], delta)) == C


def test_relabel_and_shift_invariance():
    g = W.small_graph(300, 8, n=25, span=500)
    mo = O.make_motif(W.MOTIFS["3cycle"], 60)
    base = O.Graph(g.src, g.dst, g.t, g.n).brute_count(mo)
    perm = np.random.default_rng(1).permutation(g.n).astype(np.int32)
    shifted = O.Graph(perm[g.src], perm[g.dst], g.t + 123456789, g.n)
    assert shifted.brute_count(mo) == base
    rev = np.arange(g.m)[::-1]
    assert O.Graph(g.src[rev], g.dst[rev], g.t[rev], g.n).brute_count(mo) == base


def test_monotone_in_delta():
    g = W.small_graph(300, 9, n=20, span=500)
    G = O.Graph(g.src, g.dst, g.t, g.n)
    counts = [G.brute_count(O.make_motif(W.MOTIFS["3cycle"], d)) for d in (5, 20, 60, 200, 1000)]
    assert counts == sorted(counts)
    assert counts[-1] > 0
