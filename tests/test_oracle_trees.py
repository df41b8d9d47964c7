"""Choosing the spanning tree (Sec. "Choosing the Spanning Tree"): the
candidates of Alg. 8 and the choice of Alg. 7, pinned against hand-worked
looseness values, brute-force enumeration of spanning trees, and the
brute-force count of partial matches (which W equals)."""
import os

import pytest

import oracle as O
from oracle_helpers import spanning_trees
from paper_2507_20441_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "looseness_hand.txt")

EXTRA = {
    "diamond": ((0, 1), (0, 2), (1, 3), (2, 3)),
    "triangle_tail": ((0, 1), (1, 2), (2, 0), (2, 3)),
}


def motifs():
    out = dict(W.MOTIFS)
    out.update(EXTRA)
    return out


def hand_values():
    rows = []
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        _, name, *rest = line.split()
        eq = rest.index("=")
        rows.append((name, tuple(int(x) for x in rest[:eq]), int(rest[eq + 1])))
    return rows


def test_hand_worked_looseness():
    for name, edges, want in hand_values():
        mo = O.make_motif(W.MOTIFS[name], 100)
        got = {tuple(t.edge[:t.n_edges]): loose for t, loose in O.tree_candidates(mo)}
        assert got[edges] == want, (name, edges)


@pytest.mark.parametrize("name", sorted(motifs()))
def test_candidates_are_every_tree_and_center(name):
    edges = motifs()[name]
    k = 1 + max(max(e) for e in edges)
    mo = O.make_motif(edges, 100)
    cands = O.tree_candidates(mo)
    got = sorted((tuple(t.edge[:t.n_edges]), t.center) for t, _ in cands)
    want = sorted((tuple(tr), c) for tr in spanning_trees(edges, k) for c in tr)
    assert got == want
    # ordered by looseness; the first is the default tree
    loose = [x for _, x in cands]
    assert loose == sorted(loose)
    d = O.default_tree(mo)
    first = cands[0][0]
    assert tuple(first.edge[:first.n_edges]) == tuple(d.edge[:d.n_edges]) and first.center == d.center


@pytest.mark.parametrize("name", ["3cycle", "4cycle", "scatter_gather", "diamond"])
def test_choice_minimises_brute_force_weight(name):
    edges = motifs()[name]
    g = W.small_graph(600, 21, n=40, span=4000)
    og = O.Graph(g.src, g.dst, g.t, g.n)
    mo = O.make_motif(edges, 300)
    cands = O.tree_candidates(mo)
    n_c = min(6, len(cands))
    best, Ws = O.choose_tree(og, mo, n_c)
    assert len(Ws) == n_c
    brute = [og.brute_tree_weight(mo, t) for t, _ in cands[:n_c]]
    assert Ws == brute
    arg = min(range(n_c), key=lambda x: (brute[x], x))
    bt = cands[arg][0]
    assert tuple(best.edge[:best.n_edges]) == tuple(bt.edge[:bt.n_edges]) and best.center == bt.center
