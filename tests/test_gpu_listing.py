"""Random instance listing on the GPU equals the oracle's: for every valid
sample with 0 < M_phi <= 2^20, the listed instance is the oracle's
completion of that sample's tree image at rank floor(X M_phi / 2^128), X the
sample's draw 15; every other row lists nothing."""
import numpy as np
import pytest

import oracle as O
from paper_2507_20441_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available()
    from paper_2507_20441_amd import timest
    timest.lib()
    return timest


CASES = [
    ("4cycle", W.MOTIFS["4cycle"], 2000),
    ("scatter_gather", W.MOTIFS["scatter_gather"], 3000),
    ("lead_trail", ((0, 1), (1, 2), (2, 3), (3, 0), (0, 2)), 3000),
    ("3cycle", W.MOTIFS["3cycle"], 2000),
    ("4star", W.MOTIFS["4star"], 1500),
]


@pytest.mark.parametrize("name,edges,delta", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("count", [5000, 70000])
def test_listing_matches_oracle(T, name, edges, delta, count):
    g = W.small_graph(20000, 62, n=300, span=200000)
    og = O.Graph(g.src, g.dst, g.t, g.n)
    tg = T.Graph(g.src, g.dst, g.t, g.n)
    P = O.Prep(og, O.make_motif(edges, delta))
    w = T.Weights(tg, T.make_motif(edges, delta))
    j0, seed = 1234, 9
    rows, recs = T.list_instances(w, seed, count, j0=j0)
    _, orecs = P.sample(seed, count, j0=j0, records=True)
    assert (recs == orecs).all()
    l = len(edges)
    listed = 0
    for x in range(count):
        r = recs[x]
        m = int(r["m_lo"]) | (int(r["m_hi"]) << 64)
        if r["status"] != 0 or m == 0 or m > (1 << 20):
            assert (rows[x] == -1).all(), x
            continue
        rank = O.draw(seed, j0 + x, 15, m)
        want = P.list_instance(r["eid"], rank)
        assert (rows[x][:l] == want).all() and (rows[x][l:] == -1).all(), (x, rows[x], want)
        listed += 1
    assert listed > 0
    w.close()
