"""Motif families: one stream of tree samples completed for several motifs
that share the spanning tree gives, for each motif, exactly the oracle's own
run of that motif with that tree (same seed, same k): the weights depend on
the tree alone and the draws on (seed, sample id, slot)."""
import pytest

import oracle as O
from paper_2507_20441_amd import workloads as W

pytestmark = pytest.mark.gpu

PATH = ((0, 1), (1, 2), (2, 3))
FAMILY = {
    "path": PATH,
    "cycle": ((0, 1), (1, 2), (2, 3), (3, 0)),
    "back": ((0, 1), (1, 2), (2, 3), (3, 1)),
    "chord_mid": ((0, 1), (1, 2), (2, 0), (2, 3)),
    "lead": ((3, 0), (0, 1), (1, 2), (2, 3)),
    "two_extra": ((0, 1), (1, 2), (2, 3), (3, 0), (1, 3)),
}


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available()
    from paper_2507_20441_amd import timest
    timest.lib()
    return timest


def tree_in(edges):
    idx = [edges.index(e) for e in PATH]
    return idx, idx[1]  # the path's default center is its middle edge


@pytest.mark.parametrize("k", [20000, 70000])
def test_family_equals_separate_oracle_runs(T, k):
    g = W.small_graph(20000, 51, n=300, span=200000)
    og = O.Graph(g.src, g.dst, g.t, g.n)
    tg = T.Graph(g.src, g.dst, g.t, g.n)
    delta = 3000
    pt, pc = tree_in(PATH)
    w = T.Weights(tg, T.make_motif(PATH, delta), T.make_tree(pt, pc))
    names = list(FAMILY)
    got = T.sample_family(w, [T.make_motif(FAMILY[n], delta) for n in names], 7, k)
    for name, r in zip(names, got):
        edges = FAMILY[name]
        ti, c = tree_in(list(edges))
        P = O.Prep(og, O.make_motif(edges, delta), O.make_tree(ti, c))
        o, _ = P.sample(7, k)
        assert r.status == 0 and r.W.value == P.W
        assert r.acc2.value == o.acc2.value and r.acc2_sq.value == o.acc2_sq.value, name
        assert (r.n_valid, r.n_bad_vertex, r.n_bad_delta, r.n_bad_order, r.n_nonzero) == \
               (o.n_valid, o.n_bad_vertex, o.n_bad_delta, o.n_bad_order, o.n_nonzero), name
        assert r.estimate == o.estimate and r.std_error == o.std_error, name
    w.close()


def test_family_rejects_other_trees(T):
    g = W.small_graph(2000, 52, n=80, span=20000)
    tg = T.Graph(g.src, g.dst, g.t, g.n)
    w = T.Weights(tg, T.make_motif(PATH, 1000), T.make_tree([0, 1, 2], 1))
    for edges in (((1, 2), (0, 1), (2, 3)), ((0, 1), (1, 2)), ((0, 1), (1, 2), (2, 3), (0, 1))):
        with pytest.raises(T.TimestError) as e:
            T.sample_family(w, [T.make_motif(edges, 1000)], 1, 100)
        assert e.value.code == T.TM_EINVAL
    with pytest.raises(T.TimestError):
        T.sample_family(w, [T.make_motif(PATH, 999)], 1, 100)
