"""Tree choice on the GPU (tm_tree_candidates, tm_choose_tree) equals the
oracle's: the same candidates in the same order with the same looseness, the
same W for every evaluated candidate and the same choice."""
import pytest

import oracle as O
from paper_2507_20441_amd import workloads as W

pytestmark = pytest.mark.gpu

EXTRA = {
    "diamond": ((0, 1), (0, 2), (1, 3), (2, 3)),
    "fan5": ((0, 1), (0, 2), (1, 2), (2, 3), (3, 1)),
}


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available()
    from paper_2507_20441_amd import timest
    timest.lib()
    return timest


def key(t):
    return tuple(t.edge[:t.n_edges]), t.center


@pytest.mark.parametrize("name", sorted(list(W.MOTIFS) + list(EXTRA)))
def test_tree_choice_matches_oracle(T, name):
    edges = W.MOTIFS.get(name) or EXTRA[name]
    g = W.small_graph(5000, 31, n=150, span=40000)
    og = O.Graph(g.src, g.dst, g.t, g.n)
    tg = T.Graph(g.src, g.dst, g.t, g.n)
    mo_o, mo_t = O.make_motif(edges, 2000), T.make_motif(edges, 2000)
    co, ct = O.tree_candidates(mo_o), T.tree_candidates(mo_t)
    assert [(key(t), x) for t, x in co] == [(key(t), x) for t, x in ct]
    n_c = min(8, len(co))
    bo, Wo = O.choose_tree(og, mo_o, n_c)
    bt, Wt = T.choose_tree(tg, mo_t, n_c)
    assert Wo == Wt and key(bo) == key(bt)
    tg.close()
