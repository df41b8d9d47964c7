"""Random instance listing (Sec. 4.3): the r-th completion of a valid tree
image.  Over every valid partial match phi and every rank r < M_phi the
listed instances are temporal matches (Def. "temporal match"), pairwise
distinct, and exactly C of them: listing is a bijection onto the matches."""
import pytest

import oracle as O
from oracle_helpers import all_tree_choices
from paper_2507_20441_amd import workloads as W

CASES = [
    ("4cycle", W.MOTIFS["4cycle"], 400, 600, 25, 3000),
    ("scatter_gather", W.MOTIFS["scatter_gather"], 700, 500, 15, 2500),
    ("lead_trail", ((0, 1), (1, 2), (2, 3), (3, 0), (0, 2)), 600, 600, 20, 3000),
    ("parallel", ((0, 1), (1, 0), (0, 1)), 300, 500, 15, 3000),
    ("3cycle", W.MOTIFS["3cycle"], 300, 600, 30, 3000),
]


def is_match(edges, delta, inst, src, dst, t):
    img = {}
    for (a, b), e in zip(edges, inst):
        for mv, gv in ((a, int(src[e])), (b, int(dst[e]))):
            if img.setdefault(mv, gv) != gv:
                return False
    if len(set(img.values())) != len(img):
        return False
    ts = [int(t[e]) for e in inst]
    return all(x < y for x, y in zip(ts, ts[1:])) and ts[-1] - ts[0] <= delta


@pytest.mark.parametrize("name,edges,delta,m,n,span", CASES, ids=[c[0] for c in CASES])
def test_listing_is_a_bijection_onto_matches(name, edges, delta, m, n, span):
    g = W.small_graph(m, 61, n=n, span=span)
    og = O.Graph(g.src, g.dst, g.t, g.n)
    src, dst, t = og.edges()
    mo = O.make_motif(edges, delta)
    C = og.brute_count(mo)
    for tr in list(all_tree_choices(edges))[:2]:
        P = O.Prep(og, mo, tr)
        eids, nphi, status, mphi = og.brute_partial_matches(mo, tr)
        seen = set()
        for e, st, mp in zip(eids, status, mphi):
            if st != 0:
                continue
            for r in range(mp):
                inst = tuple(int(x) for x in P.list_instance(e, r))
                assert is_match(edges, delta, inst, src, dst, t), (name, inst)
                seen.add(inst)
            with pytest.raises(O.OracleError):
                P.list_instance(e, mp)
        assert len(seen) == C, (name, len(seen), C)
