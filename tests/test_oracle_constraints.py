"""Constraint ablation (Sec. "A Closer Look at Preprocessing", Tab.
"constraints"): constraint 1 alone, with constraint 2 (distinct end vertices
of adjacent edges), with constraint 3 (2 delta intervals), and all three.
Every mode is pinned against brute force: W is the number of partial matches
under that mode's rules; over the partial matches, the completions of the
valid ones sum to the exact count (so the estimate stays unbiased); and every
sampled record is one of those partial matches with the brute-force
validation cause, N_phi and M_phi."""
import numpy as np
import pytest

import oracle as O
from oracle_helpers import all_tree_choices
from paper_2507_20441_amd import workloads as W

MODES = {"C1": 0, "C1+3": O.C_WINDOWS, "C1+2": O.C_EXCLUDE, "C1+2+3": O.C_ALL}
CASES = [
    ("3cycle", W.MOTIFS["3cycle"], 300, 500, 30, 3000),
    ("4cycle", W.MOTIFS["4cycle"], 400, 500, 25, 3000),
    ("scatter_gather", W.MOTIFS["scatter_gather"], 600, 400, 20, 3000),
    ("4star", W.MOTIFS["4star"], 300, 300, 15, 2000),
    ("6chain", W.MOTIFS["6chain"], 500, 300, 20, 3000),
]


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("name,edges,delta,m,n,span", CASES, ids=[c[0] for c in CASES])
def test_mode_against_brute_force(mode, name, edges, delta, m, n, span):
    flags = MODES[mode]
    g = W.small_graph(m, 11, n=n, span=span)
    og = O.Graph(g.src, g.dst, g.t, g.n)
    mo = O.make_motif(edges, delta)
    C = og.brute_count(mo)
    for tr in list(all_tree_choices(edges))[:2]:
        P = O.Prep(og, mo, tr, constraints=flags)
        assert P.W == og.brute_tree_weight(mo, tr, constraints=flags), (mode, name)
        eids, nphi, status, mphi = og.brute_partial_matches(mo, tr, constraints=flags)
        assert sum(mp for mp, st in zip(mphi, status) if st == 0) == C
        if flags & O.C_WINDOWS == 0:
            assert np.all(nphi == 1)
        if P.W == 0:
            continue
        table = {tuple(e[e >= 0]): (int(s), int(n_), mp) for e, s, n_, mp in zip(eids, status, nphi, mphi)}
        _, recs = P.sample(3, 400, records=True)
        for r in recs:
            key = tuple(int(x) for x in r["eid"] if x >= 0)
            st, n_, mp = table[key]
            assert int(r["status"]) == st
            if st == 0:
                assert int(r["n_phi"]) == n_ and (int(r["m_lo"]) | (int(r["m_hi"]) << 64)) == mp


def test_constraints_shrink_the_tree_weight():
    """Each constraint only removes partial matches: W(C1) >= W(C1+2) and
    W(C1) >= W(C1+3) >= ... per interval family."""
    g = W.small_graph(800, 12, n=30, span=4000)
    og = O.Graph(g.src, g.dst, g.t, g.n)
    mo = O.make_motif(W.MOTIFS["4cycle"], 500)
    w = {k: O.Prep(og, mo, constraints=v).W for k, v in MODES.items()}
    assert w["C1"] >= w["C1+2"] and w["C1+3"] >= w["C1+2+3"]


def test_stored_ablation_counts():
    """The exact counts the ablation benchmark compares against are the
    oracle's brute-force counts of that workload."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ablation_counts.txt")
    want = {}
    for line in open(path):
        if line.startswith("count "):
            _, name, c = line.split()
            want[name] = int(c)
    g = W.ablation_graph()
    og = O.Graph(g.src, g.dst, g.t, g.n)
    for name in W.ABLATION["motifs"]:
        assert og.brute_count(O.make_motif(W.MOTIFS[name], W.ABLATION["delta"])) == want[name]
