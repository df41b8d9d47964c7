"""GPU parity for partial-order motifs (a partial order of time constraints,
Sec. 1.1 remark and Sec. 6): every s-weight, W and W_i, every per-sample
record, the exact sums, the estimate and its standard error, bit for bit
against the oracle's partial-order path, for every (tree, center) choice;
the root-sorted launch with kept windows; batched jobs; the chain order
running as the total order."""
import numpy as np
import pytest

import oracle as O
from oracle_helpers import all_tree_choices
from paper_2507_20441_amd import workloads as W

pytestmark = pytest.mark.gpu

PO = W.PO_MOTIFS


def say(*a):
    print("[gpu-po]", *a, flush=True)


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "no HIP device"
    from paper_2507_20441_amd import timest
    timest.lib()
    return timest


def check(T, og, tg, edges, before, delta, otr, seeds=(1,), k=3000, constraints=None):
    omo = O.make_motif(edges, delta, before=before)
    tmo = T.make_motif(edges, delta, before=before)
    ttr = T.make_tree(list(otr.edge)[: otr.n_edges], otr.center)
    c = O.C_ALL if constraints is None else constraints
    P = O.Prep(og, omo, otr, constraints=c)
    Wt = T.Weights(tg, tmo, ttr, constraints=c)
    assert Wt.W == P.W and Wt.info()["q"] == P.q
    assert Wt.interval_weights() == P.interval_weights()
    for s in list(otr.edge)[: otr.n_edges]:
        for slot in (0, 1):
            a, b = P.weights(s, slot), Wt.weights(s, slot)
            assert (a["lo"] == b["lo"]).all() and (a["hi"] == b["hi"]).all(), (s, slot)
    for seed in seeds:
        ro, reco = P.sample(seed, k, records=True)
        rg, recg = Wt.sample(seed, k, records=True)
        assert (reco == recg).all(), seed
        assert rg.acc2.value == ro.acc2.value and rg.acc2_sq.value == ro.acc2_sq.value
        assert (rg.n_valid, rg.n_bad_vertex, rg.n_bad_delta, rg.n_bad_order, rg.n_nonzero) == \
               (ro.n_valid, ro.n_bad_vertex, ro.n_bad_delta, ro.n_bad_order, ro.n_nonzero)
        assert rg.estimate == ro.estimate and rg.std_error == ro.std_error
    return P, Wt, ro


CASES = [("po_fan3", 40), ("po_cycle3", 60), ("po_sg", 120), ("po_free2", 70), ("po_diamond", 70),
         ("po_parallel", 50)]


@pytest.mark.parametrize("name,delta", CASES, ids=[c[0] for c in CASES])
def test_every_tree_matches_oracle(T, name, delta):
    edges, before = PO[name]
    g = W.small_graph(2500, 31, n=60, span=40 * delta)
    og, tg = O.Graph(g.src, g.dst, g.t, g.n), T.Graph(g.src, g.dst, g.t, g.n)
    trees = list(all_tree_choices(edges))
    say(name, len(trees), "trees")
    valid = 0
    for otr in trees[:10]:
        _, _, ro = check(T, og, tg, edges, before, delta, otr)
        valid += ro.n_nonzero
    assert valid > 0


@pytest.mark.parametrize("name,delta", CASES, ids=[c[0] for c in CASES])
def test_root_sorted_launch_with_kept_windows(T, name, delta):
    """70,000 samples: root draws, the sort by root and the root-sorted
    sampler reading the kept child windows (unordered children included)."""
    edges, before = PO[name]
    g = W.small_graph(20011, 32, n=400, span=20 * 20011)
    og, tg = O.Graph(g.src, g.dst, g.t, g.n), T.Graph(g.src, g.dst, g.t, g.n)
    mo = O.make_motif(edges, delta * 30, before=before)
    say("sorted", name)
    check(T, og, tg, edges, before, delta * 30, O.default_tree(mo), seeds=(5,), k=70000)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_constraint_modes(T, mode):
    edges, before = PO["po_free2"]
    g = W.small_graph(2500, 33, n=60, span=2800)
    og, tg = O.Graph(g.src, g.dst, g.t, g.n), T.Graph(g.src, g.dst, g.t, g.n)
    for otr in list(all_tree_choices(edges))[:4]:
        check(T, og, tg, edges, before, 70, otr, seeds=(2,), k=3000, constraints=mode)


def test_chain_order_runs_as_the_total_order(T):
    """A partial order whose closure is total: the GPU results equal the
    oracle's total-order run (the GPU takes the total-order path)."""
    g = W.small_graph(5000, 34, n=150, span=100000)
    og, tg = O.Graph(g.src, g.dst, g.t, g.n), T.Graph(g.src, g.dst, g.t, g.n)
    for name in ("4cycle", "scatter_gather"):
        edges = W.MOTIFS[name]
        chain = [(p, p + 1) for p in range(len(edges) - 1)]
        P = O.Prep(og, O.make_motif(edges, 3000))
        Wt = T.Weights(tg, T.make_motif(edges, 3000, before=chain))
        ro, reco = P.sample(3, 20000, records=True)
        rg, recg = Wt.sample(3, 20000, records=True)
        assert Wt.W == P.W and (reco == recg).all() and rg.estimate == ro.estimate


def test_batched_partial_order_jobs_match_oracle(T):
    g1 = W.small_graph(3000, 35, n=80, span=60000)
    g2 = W.small_graph(12000, 36, n=300, span=240000)
    og = [O.Graph(g.src, g.dst, g.t, g.n) for g in (g1, g2)]
    tg = [T.Graph(g.src, g.dst, g.t, g.n) for g in (g1, g2)]
    jobs = []
    for j, (name, delta) in enumerate(CASES):
        edges, before = PO[name]
        gi = j % 2
        jobs.append((gi, edges, before, delta * 20, 4000 + 1000 * j, 100 + j))
    jobs.append((0, W.MOTIFS["4cycle"], None, 3000, 5000, 7))   # a total-order job in the mix
    ws = [T.Weights(tg[gi], T.make_motif(e, d, before=b)) for gi, e, b, d, _, _ in jobs]
    say("batch", len(ws))
    got = T.sample_batch(ws, [k for *_, k, _ in jobs], [s for *_, s in jobs])
    est = T.estimate_batch([tg[gi] for gi, *_ in jobs], [T.make_motif(e, d, before=b) for _, e, b, d, _, _ in jobs],
                           [k for *_, k, _ in jobs], [s for *_, s in jobs])
    for i, (gi, e, b, d, k, seed) in enumerate(jobs):
        ro, _ = O.Prep(og[gi], O.make_motif(e, d, before=b)).sample(seed, k)
        for r in (got[i], est[i]):
            assert r.status == 0 and r.acc2.value == ro.acc2.value and r.acc2_sq.value == ro.acc2_sq.value
            assert r.n_valid == ro.n_valid and r.n_bad_order == ro.n_bad_order and r.W.value == ro.W.value
            assert r.estimate == ro.estimate and r.std_error == ro.std_error, i


def test_partial_order_errors(T):
    g = W.small_graph(500, 37, n=30, span=5000)
    tg = T.Graph(g.src, g.dst, g.t, g.n)
    bad = [T.make_motif(((0, 1), (1, 2)), 10, before=[(1, 0)]),
           T.make_motif(((0, 1), (0, 1), (1, 2)), 10, before=[]),
           # six non-tree edges unordered: beyond the GPU's completion counter
           T.make_motif(((0, 1), (1, 0), (0, 1), (1, 0), (0, 1), (1, 0), (0, 1)), 10,
                        before=[(0, 2), (2, 4), (4, 6), (1, 3), (3, 5)])]
    for mo in bad:
        with pytest.raises(T.TimestError) as e:
            T.Weights(tg, mo)
        assert e.value.code == T.TM_EINVAL
    edges, before = PO["po_cycle3"]
    w = T.Weights(tg, T.make_motif(edges, 100, before=before))
    with pytest.raises(T.TimestError):
        T.list_instances(w, 1, 10)
    with pytest.raises(T.TimestError):
        T.sample_family(w, [T.make_motif(edges, 100, before=before)], 1, 100)
