"""Pins for validation (Alg. 4) and derivation (Alg. 5) in the oracle.

Exact identity from the unbiasedness proof (Lemma "unbiased-estimate"): the
sum of M_phi over all partial matches phi that pass validation equals C.  And
every single M_phi equals the brute-force count of completions of phi.
"""
import pytest

import oracle as O
from oracle_helpers import all_tree_choices
from paper_2507_20441_amd import workloads as W

CASES = [
    ("3cycle", W.MOTIFS["3cycle"], 50, 110, 8, 250),
    ("4cycle", W.MOTIFS["4cycle"], 70, 120, 7, 250),
    ("4star", W.MOTIFS["4star"], 40, 90, 8, 250),
    ("scatter_gather", W.MOTIFS["scatter_gather"], 90, 120, 6, 160),
    ("6chain", W.MOTIFS["6chain"], 70, 80, 8, 200),
    ("lead_trail", ((0, 1), (1, 2), (2, 3), (3, 0), (0, 2)), 90, 110, 6, 250),
    ("parallel", ((0, 1), (1, 0), (0, 1)), 40, 100, 6, 300),
    ("in_star", ((1, 0), (2, 0), (0, 3)), 40, 100, 8, 300),
]


@pytest.mark.parametrize("name,edges,delta,m,n,span", CASES, ids=[c[0] for c in CASES])
def test_sum_of_m_phi_over_valid_partial_matches_is_exact_count(name, edges, delta, m, n, span):
    g = W.small_graph(m, 3, n=n, span=span)
    G = O.Graph(g.src, g.dst, g.t, g.n)
    mo = O.make_motif(edges, delta)
    C = G.brute_count(mo)
    trees = list(all_tree_choices(edges))
    assert C > 0 or name == "scatter_gather"
    for tr in trees[:16]:
        P = O.Prep(G, mo, tr)
        eids, nphi, status, mb = G.brute_partial_matches(mo, tr)
        assert int(nphi.sum()) == P.W
        total = 0
        for a in range(len(nphi)):
            d = P.derive_cnt(eids[a][: tr.n_edges])
            if status[a] == 0:
                assert d == mb[a], (eids[a], d, mb[a])
                total += d
            else:
                assert d is None and mb[a] == 0
        assert total == C, (list(tr.edge)[: tr.n_edges], tr.center)


def test_scatter_gather_has_completions():
    """Denser graph so that the two middle non-tree edges of the fan-out/fan-in
    motif do complete some samples."""
    g = W.small_graph(160, 12, n=5, span=120)
    G = O.Graph(g.src, g.dst, g.t, g.n)
    mo = O.make_motif(W.MOTIFS["scatter_gather"], 100)
    C = G.brute_count(mo)
    assert C > 0
    tr = O.default_tree(mo)
    P = O.Prep(G, mo, tr)
    eids, nphi, status, mb = G.brute_partial_matches(mo, tr)
    total = 0
    for a in range(len(nphi)):
        if status[a] == 0:
            d = P.derive_cnt(eids[a][: tr.n_edges])
            assert d == mb[a]
            total += d
    assert total == C
