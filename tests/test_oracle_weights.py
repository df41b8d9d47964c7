"""Pins for the oracle's s-weights and W (Def. "s-weight", Claims
"overall-num-matches" and "num-matches-entire-tree", Alg. 1 / Alg. 2).

W must equal the number of delta-partial matches of the tree counted once per
interval that holds them, enumerated by brute force; every single weight must
equal the brute-force count of partial matches of the subtree below it.
"""
import numpy as np
import pytest

import oracle as O
from golden_io import load
from oracle_helpers import all_tree_choices
from paper_2507_20441_amd import workloads as W

CASES = [
    ("3cycle", W.MOTIFS["3cycle"], 50, 100, 10, 300),
    ("4cycle", W.MOTIFS["4cycle"], 60, 100, 10, 300),
    ("4star", W.MOTIFS["4star"], 40, 90, 8, 250),
    ("scatter_gather", W.MOTIFS["scatter_gather"], 60, 70, 6, 150),
    ("6chain", W.MOTIFS["6chain"], 60, 70, 8, 200),
    ("5edge", ((0, 1), (1, 2), (2, 3), (3, 0), (0, 2)), 80, 90, 8, 250),
    ("parallel", ((0, 1), (1, 0), (0, 1)), 40, 100, 8, 300),
]


@pytest.mark.parametrize("name,edges,delta,m,n,span", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("seed", [1, 2])
def test_total_weight_equals_brute_partial_matches(name, edges, delta, m, n, span, seed):
    g = W.small_graph(m, seed, n=n, span=span)
    G = O.Graph(g.src, g.dst, g.t, g.n)
    mo = O.make_motif(edges, delta)
    checked = 0
    for tr in all_tree_choices(edges):
        P = O.Prep(G, mo, tr)
        Wb = G.brute_tree_weight(mo, tr)
        assert P.W == Wb, (list(tr.edge)[: tr.n_edges], tr.center)
        assert sum(P.interval_weights()) == P.W
        checked += 1
        if checked >= 12:
            break


@pytest.mark.parametrize("name,edges,delta,m,n,span", CASES[:5], ids=[c[0] for c in CASES[:5]])
def test_every_weight_equals_brute_subtree_count(name, edges, delta, m, n, span):
    g = W.small_graph(m, 4, n=n, span=span)
    G = O.Graph(g.src, g.dst, g.t, g.n)
    _, _, tt = G.edges()
    mo = O.make_motif(edges, delta)
    for tr in list(all_tree_choices(edges))[:4]:
        P = O.Prep(G, mo, tr)
        for s in list(tr.edge)[: tr.n_edges]:
            for slot in (0, 1):
                w = O.u128_array_to_int(P.weights(s, slot))
                for eid in range(0, g.m, 3):
                    i = int(tt[eid]) // delta - slot
                    if i < 0 or i >= P.q:
                        assert w[eid] == 0
                        continue
                    assert w[eid] == G.brute_edge_weight(mo, tr, i, s, eid), (s, slot, eid)


def test_prose_example_weight():
    fx = load("prose_weight.txt")
    G = O.Graph(fx["src"], fx["dst"], fx["t"], fx["n"])
    mo = O.make_motif(fx["motif"], fx["delta"])
    tr = O.make_tree(fx["tree"], fx["center"])
    P = O.Prep(G, mo, tr)
    s, d, t = G.edges()
    u, v, tw = fx["weight_of"]
    eid = int(np.nonzero((s == u) & (d == v) & (t == tw - G.shift))[0][0])
    w0 = O.u128_array_to_int(P.weights(fx["center"], 0))[eid]
    w1 = O.u128_array_to_int(P.weights(fx["center"], 1))[eid]
    assert (w0, w1) == (fx["expect_weight_slot0"], fx["expect_weight_slot1"])


def test_default_trees_follow_looseness_rule():
    want = {"3cycle": ((0, 1), 0), "4cycle": ((0, 1, 2), 1), "4star": ((0, 1, 2, 3), 0),
            "scatter_gather": ((0, 1, 4, 5), 1), "6chain": ((0, 1, 2, 3, 4), 2)}
    for name, (edges, center) in want.items():
        tr = O.default_tree(O.make_motif(W.MOTIFS[name], 10))
        assert tuple(tr.edge[: tr.n_edges]) == edges and tr.center == center, name


def test_empty_graph_has_zero_weight():
    G = O.Graph(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64), 3)
    P = O.Prep(G, O.make_motif(W.MOTIFS["3cycle"], 10))
    assert P.W == 0 and P.q == 0
    res, recs = P.sample(1, 10, records=True)
    assert res.flags & 1 and res.estimate == 0.0
    assert (recs["status"] == 4).all()


@pytest.mark.parametrize("name,edges,delta,m,n,span", CASES[:6], ids=[c[0] for c in CASES[:6]])
def test_single_edge_weight_equals_tables(name, edges, delta, m, n, span):
    """The table-free single-edge weight (recursion over candidate lists) gives
    every table entry of every tree edge, both slots, for every tree choice;
    and a tight work limit is reported instead of a wrong value."""
    g = W.small_graph(m, 7, n=n, span=span)
    og = O.Graph(g.src, g.dst, g.t, g.n)
    for tr in all_tree_choices(edges):
        mo = O.make_motif(edges, delta)
        P = O.Prep(og, mo, tr)
        L = O.Prep(og, mo, tr, light=True)
        t = og.edges()[2]
        for s in tr.edge[:tr.n_edges]:
            for slot in (0, 1):
                ref = O.u128_array_to_int(P.weights(s, slot))
                for e in range(og.m):
                    i = int(t[e]) // delta - slot
                    if i < 0 or i >= P.q:
                        continue
                    assert L.edge_weight(i, s, e) == ref[e], (s, slot, e)
    # a limit smaller than the first candidate list: refused, not truncated
    mo = O.make_motif(edges, delta)
    L = O.Prep(og, mo, light=True)
    c = L.tr.center
    t = og.edges()[2]
    seen = False
    for e in range(og.m):
        i = int(t[e]) // delta
        if i >= L.q:
            continue
        full = L.edge_weight(i, c, e)
        if full and full > 1:
            assert L.edge_weight(i, c, e, work_limit=0) is None
            seen = True
            break
    assert seen
