"""Pins for partial-order motifs in the oracle (the paper's generalisation to
"a partial order of time constraints", Sec. 1.1 remark and Sec. 6).

A motif under a partial order P requires t(p) < t(q) only for the pairs of P
(and the pairs they imply); every other pair may come in either order or at
equal times.  Pins:
  * hand-worked counts (tests/golden/po_*_hand.txt);
  * a chain order is the total order: the same counts, weights, samples and
    estimate as the total-order path;
  * on graphs whose timestamps are all distinct, every match of P orders its
    edges in exactly one way, which is a linear extension of P, so C_P is the
    sum over the linear extensions L of the total-order count of the motif
    listed in L's order (the total-order brute force is pinned on its own);
  * W equals the brute-force count of partial matches (each parent/child pair
    within [t - delta, t + delta] when P leaves it unordered), every s-weight
    equals its brute-force count, the valid partial matches' completions sum
    to C_P and each equals its brute-force completions;
  * the estimator is unbiased over seeds.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from golden_io import load
from oracle_helpers import all_tree_choices
from paper_2507_20441_amd import workloads as W

PO = W.PO_MOTIFS


def po_motif(name, delta):
    edges, before = PO[name]
    return O.make_motif(edges, delta, before=before)


def closure(l, before):
    R = {(p, q) for p, q in before}
    changed = True
    while changed:
        changed = False
        for (a, b), (c, d) in itertools.product(list(R), list(R)):
            if b == c and (a, d) not in R:
                R.add((a, d))
                changed = True
    return R


def linear_extensions(l, before):
    R = closure(l, before)
    for perm in itertools.permutations(range(l)):
        pos = {p: x for x, p in enumerate(perm)}
        if all(pos[p] < pos[q] for p, q in R):
            yield perm


def distinct_time_graph(m, seed, n, span):
    g = W.small_graph(m, seed, n=n, span=span)
    rng = np.random.default_rng(seed + 1000)
    # distinct times: a random injection into [0, span)
    t = np.sort(rng.choice(span, size=m, replace=False)).astype(np.int64)
    t = t[rng.permutation(m)]
    return W.TemporalGraph(g.src, g.dst, t, g.n)


@pytest.mark.parametrize("fixture", ["po_star2_hand.txt", "po_cycle3_hand.txt"])
def test_hand_worked_counts(fixture):
    fx = load(fixture)
    G = O.Graph(fx["src"], fx["dst"], fx["t"], fx["n"])
    mo = O.make_motif(fx["motif"], fx["delta"], before=fx["before"])
    assert G.brute_count(mo) == fx["expect_count"]
    # and through the estimator's exact identity: sum of M_phi over the valid
    # partial matches of every tree
    for tr in all_tree_choices(fx["motif"]):
        P = O.Prep(G, mo, tr)
        eids, nphi, status, mb = G.brute_partial_matches(mo, tr)
        assert int(nphi.sum()) == P.W
        total = sum(P.derive_cnt(eids[a][: tr.n_edges]) for a in range(len(nphi)) if status[a] == 0)
        assert total == fx["expect_count"]


@pytest.mark.parametrize("name", list(W.MOTIFS))
def test_chain_order_is_the_total_order(name):
    """before = consecutive pairs only: its closure is the total order, and
    the partial-order code paths give the total-order results."""
    edges = W.MOTIFS[name]
    g = W.small_graph(150, 4, n=7, span=300)
    G = O.Graph(g.src, g.dst, g.t, g.n)
    tot = O.make_motif(edges, 80)
    chain = O.make_motif(edges, 80, before=[(p, p + 1) for p in range(len(edges) - 1)])
    assert G.brute_count(tot) == G.brute_count(chain)
    for tr in list(all_tree_choices(edges))[:4]:
        A, B = O.Prep(G, tot, tr), O.Prep(G, chain, tr)
        assert A.W == B.W and A.interval_weights() == B.interval_weights()
        ra, reca = A.sample(3, 2000, records=True)
        rb, recb = B.sample(3, 2000, records=True)
        assert (reca == recb).all()
        assert (ra.acc2.value, ra.acc2_sq.value, ra.estimate, ra.std_error) == \
               (rb.acc2.value, rb.acc2_sq.value, rb.estimate, rb.std_error)


@pytest.mark.parametrize("name,delta,m,n,span", [("po_fan3", 40, 70, 6, 200), ("po_cycle3", 60, 90, 6, 250),
                                                  ("po_free2", 60, 80, 5, 250), ("po_diamond", 60, 80, 6, 250),
                                                  ("po_parallel", 50, 70, 5, 250)])
def test_count_is_sum_over_linear_extensions(name, delta, m, n, span):
    edges, before = PO[name]
    g = distinct_time_graph(m, 7, n, span)
    G = O.Graph(g.src, g.dst, g.t, g.n)
    C = G.brute_count(po_motif(name, delta))
    total = 0
    for perm in linear_extensions(len(edges), before):
        total += G.brute_count(O.make_motif([edges[p] for p in perm], delta))
    assert C == total and C > 0, (C, total)


def test_ties_are_counted_for_unordered_pairs_only():
    """Equal times: an unordered pair may share a time, an ordered one may not."""
    src = np.array([0, 0, 0], np.int32)
    dst = np.array([1, 2, 3], np.int32)
    t = np.array([5, 5, 5], np.int64)
    G = O.Graph(src, dst, t, 4)
    # unordered 2-leaf fan-out: 3 heads pairwise, both roles: 6
    assert G.brute_count(O.make_motif(((0, 1), (0, 2)), 3, before=[])) == 6
    assert G.brute_count(O.make_motif(((0, 1), (0, 2)), 3)) == 0
    assert G.brute_count(O.make_motif(((0, 1), (0, 2), (0, 3)), 3, before=[])) == 6


PO_CASES = [("po_fan3", 40, 90, 7, 250), ("po_cycle3", 50, 110, 7, 250), ("po_sg", 100, 140, 6, 160),
            ("po_free2", 60, 110, 6, 250), ("po_diamond", 60, 110, 7, 250), ("po_parallel", 50, 100, 5, 250)]


@pytest.mark.parametrize("name,delta,m,n,span", PO_CASES, ids=[c[0] for c in PO_CASES])
def test_weights_and_completions_against_brute_force(name, delta, m, n, span):
    edges, before = PO[name]
    g = W.small_graph(m, 3, n=n, span=span)
    G = O.Graph(g.src, g.dst, g.t, g.n)
    mo = po_motif(name, delta)
    C = G.brute_count(mo)
    assert C > 0
    s_, d_, tt = G.edges()
    for tr in list(all_tree_choices(edges))[:12]:
        P = O.Prep(G, mo, tr)
        eids, nphi, status, mb = G.brute_partial_matches(mo, tr)
        assert int(nphi.sum()) == P.W
        total = 0
        for a in range(len(nphi)):
            d = P.derive_cnt(eids[a][: tr.n_edges])
            if status[a] == 0:
                assert d == mb[a]
                total += d
            else:
                assert d is None and mb[a] == 0
        assert total == C, (list(tr.edge)[: tr.n_edges], tr.center)
        # s-weights of non-leaf tree edges on a sample of (edge, slot)
        for sidx in list(tr.edge)[: tr.n_edges]:
            for slot in (0, 1):
                ws = P.weights(sidx, slot)
                for e in range(0, G.m, 7):
                    i = int(tt[e]) // delta - slot
                    if i < 0 or i >= P.q:
                        continue
                    want = G.brute_edge_weight(mo, tr, i, sidx, e)
                    assert int(ws[e]["lo"]) + (int(ws[e]["hi"]) << 64) == want, (sidx, slot, e)


@pytest.mark.parametrize("name,delta,m,n,span", [("po_cycle3", 60, 110, 7, 250), ("po_free2", 70, 100, 6, 250)])
def test_unbiased_over_seeds(name, delta, m, n, span):
    g = W.small_graph(m, 8, n=n, span=span)
    G = O.Graph(g.src, g.dst, g.t, g.n)
    mo = po_motif(name, delta)
    C = G.brute_count(mo)
    tr = O.default_tree(mo)
    P = O.Prep(G, mo, tr)
    eids, nphi, status, mb = G.brute_partial_matches(mo, tr)
    Wt = P.W
    y = np.array([2 * mb[a] / nphi[a] if status[a] == 0 and nphi[a] else 0.0 for a in range(len(nphi))])
    p = nphi / Wt
    ey, ey2 = float((p * y).sum()), float((p * y * y).sum())
    assert abs(Wt * ey / 2 - C) < 1e-9 * max(C, 1)
    k, seeds = 200, 600
    ests = [P.sample(seed=s, k=k)[0].estimate for s in range(1, seeds + 1)]
    sigma = math.sqrt((Wt / 2) ** 2 * (ey2 - ey ** 2) / k / seeds)
    assert abs(float(np.mean(ests)) - C) <= 3 * sigma, (np.mean(ests), C, sigma)


def test_partial_order_errors():
    g = W.small_graph(100, 3, n=6, span=200)
    G = O.Graph(g.src, g.dst, g.t, g.n)
    bad = [
        O.make_motif(((0, 1), (1, 2)), 10, before=[(1, 0)]),          # a pair against the listing order
        O.make_motif(((0, 1), (0, 1), (1, 2)), 10, before=[]),        # parallel edges left unordered
    ]
    m2 = O.make_motif(((0, 1), (1, 2)), 10)
    m2.partial = 2
    bad.append(m2)
    m3 = O.make_motif(((0, 1), (1, 2)), 10, before=[])
    m3.before[5] = 1                                                  # a pair beyond the motif's edges
    bad.append(m3)
    for mo in bad:
        with pytest.raises(O.OracleError):
            O.Prep(G, mo)
        with pytest.raises(O.OracleError):
            G.brute_count(mo)
