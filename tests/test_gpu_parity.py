"""GPU parity: the HIP path, called through the C ABI, against the oracle.

Integers are compared bit for bit: the CSR arrays, every s-weight, W and
every W_i, every per-sample record, the exact accumulators; the FP64
estimate is the same formula on the same integers and must be identical.
"""
import sys

import numpy as np
import pytest

import oracle as O
from oracle_helpers import all_tree_choices
from paper_2507_20441_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-parity]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "no HIP device"
    from paper_2507_20441_amd import timest
    timest.lib()
    return timest


def pair(T, g):
    return O.Graph(g.src, g.dst, g.t, g.n), T.Graph(g.src, g.dst, g.t, g.n)


def motifs_for(T, edges, delta):
    return O.make_motif(edges, delta), T.make_motif(edges, delta)


def trees_for(T, otr):
    return otr, T.make_tree(list(otr.edge)[: otr.n_edges], otr.center)


def rec_equal(a, b):
    return bool((a == b).all())


# ---------------------------------------------------------------------------
# CSR build
# ---------------------------------------------------------------------------
# 4096 and 8192: whole sort tiles only (4096 keys), no ragged last tile; the
# last two: 2 bn + bt > 64 (bn the vertex-id bits, bt the time bits), so
# the canonical order takes two sorts (by (u, v), then by time), with an odd
# and an even number of digit passes in the first
@pytest.mark.parametrize("m,seed,n,span", [(1, 1, 2, 10), (777, 2, 40, 300), (5000, 3, 300, 20000),
                                           (4096, 8, 500, 10**5), (8192, 9, 1500, 10**6),
                                           (40000, 4, 2000, 10**6), (30000, 6, 600_000, 2**30),
                                           (30000, 7, 3_000_000, 2**35)])
def test_csr_matches_oracle(T, m, seed, n, span):
    say("csr", m, seed, n, span)
    g = W.small_graph(m, seed, n=n, span=span)
    og, tg = pair(T, g)
    s, d, t = og.edges()
    assert (tg.export("src") == s).all() and (tg.export("dst") == d).all()
    assert (tg.export("t") == t).all()
    info = tg.info()
    assert info["t_shift"] == og.shift
    bt = max(1, int(info["t_span"]).bit_length())
    for name, direction, own, nbr in (("out", +1, s, d), ("in", -1, d, s)):
        off = tg.export(f"{name}_off")
        teid = tg.export(f"{name}_eid")
        neid = tg.export(f"{name}n_eid")
        assert off[0] == 0 and off[-1] == g.m
        # per-vertex lists: the oracle's, for every vertex that has edges
        # (offsets are checked for all vertices through the degrees)
        deg = np.bincount(own, minlength=g.n)
        assert (np.diff(off) == deg).all(), name
        for v in np.nonzero(deg)[0]:
            want = og.vertex_list(int(v), direction)
            got = teid[off[v]:off[v + 1]]
            assert (got == want).all(), (name, v)
            # N order: the same edges by (neighbour, eid)
            order = np.lexsort((want, nbr[want]))
            assert (neid[off[v]:off[v + 1]] == want[order]).all(), (name, v)
        # the arrays carried along with the eids
        assert (tg.export(f"{name}_t") == t[teid]).all(), name
        assert (tg.export(f"{name}_nbr") == nbr[teid]).all(), name
        pos = tg.export(f"{name}_pos")
        assert (pos[teid] == np.arange(g.m)).all(), name
        key = tg.export(f"{name}n_key")
        assert (key == ((nbr[neid].astype(np.uint64) << np.uint64(bt)) | t[neid].astype(np.uint64))).all(), name
        assert (tg.export(f"{name}n_pos") == pos[neid]).all(), name


def test_graph_from_device_tensors(T):
    import torch
    g = W.small_graph(3000, 5, n=200, span=5000)
    a = T.Graph(g.src, g.dst, g.t, g.n)
    b = T.Graph(torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda(),
                torch.from_numpy(g.t).cuda(), g.n)
    for name in ("src", "dst", "t", "out_off", "in_off", "out_eid", "in_eid", "outn_eid", "inn_eid"):
        assert (a.export(name) == b.export(name)).all(), name


def test_graph_errors_match_oracle(T):
    cases = [
        ([0, 1], [1, 1], [5, 6], 3),          # self loop
        ([0, 0], [1, 1], [5, 5], 3),          # duplicate tuple
        ([0, 4], [1, 2], [5, 6], 3),          # id out of range
        ([0, 1], [1, 2], [-(2**62), 2**62], 3),  # span too large
    ]
    for s, d, t, n in cases:
        say("graph error case", s, d, t)
        with pytest.raises(O.OracleError) as eo:
            O.Graph(np.array(s), np.array(d), np.array(t), n)
        with pytest.raises(T.TimestError) as eg:
            T.Graph(np.array(s), np.array(d), np.array(t), n)
        assert eo.value.code == eg.value.code


# ---------------------------------------------------------------------------
# Weights and samples
# ---------------------------------------------------------------------------
def check_prep(T, og, tg, edges, delta, otr, seeds=(1, 2), k=3000, g=None, constraints=None):
    omo, tmo = motifs_for(T, edges, delta)
    otr, ttr = trees_for(T, otr)
    P = O.Prep(og, omo, otr, constraints=O.C_ALL if constraints is None else constraints)
    Wt = T.Weights(tg, tmo, ttr, constraints=constraints)
    info = Wt.info()
    assert info["W"] == P.W
    assert info["q"] == P.q
    assert Wt.interval_weights() == P.interval_weights()
    for s in list(otr.edge)[: otr.n_edges]:
        for slot in (0, 1):
            a = P.weights(s, slot)
            b = Wt.weights(s, slot)
            assert (a["lo"] == b["lo"]).all() and (a["hi"] == b["hi"]).all(), (s, slot)
    for seed in seeds:
        ro, reco = P.sample(seed, k, records=True)
        rg, recg = Wt.sample(seed, k, records=True)
        assert rec_equal(reco, recg), seed
        assert rg.acc2.value == ro.acc2.value and rg.acc2_sq.value == ro.acc2_sq.value
        assert (rg.n_valid, rg.n_bad_vertex, rg.n_bad_delta, rg.n_bad_order, rg.n_nonzero) == \
               (ro.n_valid, ro.n_bad_vertex, ro.n_bad_delta, ro.n_bad_order, ro.n_nonzero)
        assert rg.estimate == ro.estimate and rg.std_error == ro.std_error
    return P, Wt


MOTIF_CASES = [
    ("3cycle", W.MOTIFS["3cycle"], 50),
    ("4cycle", W.MOTIFS["4cycle"], 70),
    ("4star", W.MOTIFS["4star"], 40),
    ("scatter_gather", W.MOTIFS["scatter_gather"], 90),
    ("6chain", W.MOTIFS["6chain"], 70),
    ("lead_trail", ((0, 1), (1, 2), (2, 3), (3, 0), (0, 2)), 90),
    ("parallel", ((0, 1), (1, 0), (0, 1)), 40),
    ("in_star", ((1, 0), (2, 0), (0, 3)), 40),
    ("single_edge", ((0, 1),), 30),
]


@pytest.mark.parametrize("name,edges,delta", MOTIF_CASES, ids=[c[0] for c in MOTIF_CASES])
def test_every_tree_and_center_small_graph(T, name, edges, delta):
    g = W.small_graph(300, 11, n=12, span=600)
    og, tg = pair(T, g)
    for j, otr in enumerate(all_tree_choices(edges)):
        if j >= 10:
            break
        say(name, "tree", list(otr.edge)[: otr.n_edges], "center", otr.center)
        check_prep(T, og, tg, edges, delta, otr, seeds=(3,), k=2000)


def center_children_ends(edges, otr):
    """Whether some child of the tree's center edge touches its source, its
    destination."""
    ids = list(otr.edge)[: otr.n_edges]
    cu, cv = edges[otr.center]
    others = [edges[i] for i in ids if i != otr.center]
    return any(cu in e for e in others), any(cv in e for e in others)


SORTED_CASES = [c for c in MOTIF_CASES if c[0] in ("3cycle", "4cycle", "4star", "in_star", "6chain", "lead_trail")]


@pytest.mark.parametrize("name,edges,delta", SORTED_CASES, ids=[c[0] for c in SORTED_CASES])
def test_root_sorted_path_both_root_lists(T, name, edges, delta):
    """k >= 2^16 takes the root-sorted sampler, which reads the kept child
    windows; the root keys come from the in-lists when every child of the
    center attaches at its destination, else from the out-lists.  One tree
    of each kind per motif (where the motif has one), sample by sample
    against the oracle."""
    g = W.small_graph(3000, 13, n=60, span=6000)
    og, tg = pair(T, g)
    picked = {}
    for otr in all_tree_choices(edges):
        at_src, at_dst = center_children_ends(edges, otr)
        kind = "in" if at_dst and not at_src else "out"
        picked.setdefault(kind, otr)
        if len(picked) == 2:
            break
    for kind, otr in sorted(picked.items()):
        say(name, "root list", kind, "tree", list(otr.edge)[: otr.n_edges], "center", otr.center)
        check_prep(T, og, tg, edges, delta, otr, seeds=(5,), k=70000)


@pytest.mark.parametrize("name,edges,delta", MOTIF_CASES[:6], ids=[c[0] for c in MOTIF_CASES[:6]])
def test_default_tree_multi_tile_graph(T, name, edges, delta):
    """Several scan and sort tiles with a ragged tail."""
    g = W.small_graph(20011, 12, n=600, span=200000)
    og, tg = pair(T, g)
    say(name, "multi-tile")
    check_prep(T, og, tg, edges, delta * 20, O.default_tree(O.make_motif(edges, 1)), seeds=(1, 9),
               k=20000)


def stretched(g, top):
    """g with its shifted times scaled so that the largest is exactly top."""
    t = g.t - g.t.min()
    scale = top // int(t.max())
    t = t * scale
    t[int(np.argmax(t))] = top
    return W.TemporalGraph(g.src, g.dst, t, g.n), scale


@pytest.mark.parametrize("top", [2**32 - 2, 2**32 - 1, 2**33 + 5], ids=["last_32_bit", "first_64_bit", "beyond"])
def test_time_span_at_and_beyond_32_bits(T, top):
    """Lists hold 32-bit times when every shifted time is below 2^32 - 1 and
    64-bit ones otherwise.  A graph stretched so that its largest shifted
    time is the last value of the 32-bit form, the first of the 64-bit one,
    or beyond: its list times, then weights and samples of three motifs in
    both sampler shapes (k below 2^16, and the root-sorted one reading kept
    windows), against the oracle."""
    g, scale = stretched(W.small_graph(3000, 13, n=60, span=6000), top)
    og, tg = pair(T, g)
    assert tg.info()["t_span"] == top
    s, d, t = og.edges()
    for name in ("out", "in"):
        assert (tg.export(f"{name}_t") == t[tg.export(f"{name}_eid")]).all(), name
    for name, delta in (("3cycle", 50), ("4cycle", 70), ("6chain", 70)):
        edges = W.MOTIFS[name]
        say("span", top, name)
        check_prep(T, og, tg, edges, delta * scale, O.default_tree(O.make_motif(edges, 1)), seeds=(1,), k=3000)
        check_prep(T, og, tg, edges, delta * scale, O.default_tree(O.make_motif(edges, 1)), seeds=(2,), k=70000)


def test_tiny_workload_full_run_is_bit_identical(T):
    """The small workload in full: 1,000 vertices, 20,000 edges, 3-cycle at
    delta = 1,000, 100,000 samples, seed 1."""
    g = W.tiny_graph()
    og, tg = pair(T, g)
    (name, delta), = W.TINY["motifs"]
    omo, tmo = motifs_for(T, W.MOTIFS[name], delta)
    P = O.Prep(og, omo)
    Wt = T.Weights(tg, tmo)
    say("tiny full run")
    ro, reco = P.sample(W.TINY["seed"], W.TINY["k"], records=True)
    rg, recg = Wt.sample(W.TINY["seed"], W.TINY["k"], records=True)
    assert rec_equal(reco, recg)
    assert rg.estimate == ro.estimate and rg.acc2.value == ro.acc2.value and rg.std_error == ro.std_error
    C = og.brute_count(omo)
    assert abs(rg.estimate - C) <= 0.05 * C, (rg.estimate, C)


@pytest.mark.parametrize("hub_n", [1500, 3000])
def test_wide_weights_beyond_64_bits(T, hub_n):
    """An 8-vertex out-star on a hub with hub_n out-edges inside one window.
    1,500: each center weight (up to about 1500^6) fits 64 bits but their
    sum W does not, so the 64-bit tables are widened to 128 bits without
    recomputing a level; 3,000: the weights themselves reach 2^64 and the
    whole set is rebuilt in 128 bits."""
    rng = np.random.default_rng(3)
    src = np.zeros(hub_n, np.int32)
    dst = np.arange(1, hub_n + 1, dtype=np.int32)
    t = rng.integers(0, 50, hub_n).astype(np.int64)
    g = W.TemporalGraph(src, dst, t, hub_n + 1)
    og, tg = pair(T, g)
    edges = tuple((0, j) for j in range(1, 8))
    omo, tmo = motifs_for(T, edges, 100)
    say("wide", hub_n)
    P, Wt = check_prep(T, og, tg, edges, 100, O.default_tree(omo), seeds=(1,), k=4000)
    assert P.W >= 2**64 and Wt.info()["wide"]
    # which path ran: one level launch (widened) or two (rebuilt)
    T.profile_read(reset=True)
    T.profile_enable(True)
    again = T.Weights(tg, tmo)
    T.profile_enable(False)
    launches = T.profile_read(reset=True)["launches"][T.STAGES.index("levels")]
    assert launches == (1 if hub_n == 1500 else 2), launches
    assert again.W == P.W


def test_widened_set_keeps_64_bit_list_tables(T):
    """A path center -> middle -> five leaves on a hub of 5,000 out-edges:
    the middle edge's weights (5000^5 each) and its list totals fit 64 bits,
    the center's total W does not.  The set is widened without a second level
    launch; its list tables stay 64-bit while the sampler draws the root in
    128 bits (and, in the root-sorted shape, picks the children in 64), and
    every weight, record and sum equals the oracle's."""
    hub = 5000
    src = np.concatenate([np.arange(10, 20), np.full(2, 1), np.full(hub, 2)]).astype(np.int32)
    dst = np.concatenate([np.full(10, 1), np.full(2, 2), np.arange(100, 100 + hub)]).astype(np.int32)
    t = np.concatenate([np.arange(10), 20 + np.arange(2), 30 + np.arange(hub)]).astype(np.int64)
    g = W.TemporalGraph(src, dst, t, 100 + hub)
    og, tg = pair(T, g)
    edges = ((0, 1), (1, 2)) + tuple((2, j) for j in range(3, 8))
    delta = 6000
    otr = O.make_tree(list(range(len(edges))), 0)
    say("widened list tables")
    P, Wt = check_prep(T, og, tg, edges, delta, otr, seeds=(1, 2), k=4000)
    check_prep(T, og, tg, edges, delta, otr, seeds=(3,), k=70000)  # root-sorted, kept windows
    info = Wt.info()
    assert P.W >= 2**64 and info["wide"]
    _, tmo = motifs_for(T, edges, delta)
    ttr = T.make_tree(list(range(len(edges))), 0)
    assert T.weights_footprint(tg, tmo, ttr, wide=False) < info["bytes"] < T.weights_footprint(tg, tmo, ttr, wide=True)
    T.profile_read(reset=True)
    T.profile_enable(True)
    again = T.Weights(tg, tmo, ttr)
    T.profile_enable(False)
    launches = T.profile_read(reset=True)["launches"][T.STAGES.index("levels")]
    assert again.W == P.W and launches == 2, launches  # one per non-leaf level, no rebuild


def test_zero_weight_and_empty_graph(T):
    # no 2-path can exist: every edge leaves vertex 0
    g = W.TemporalGraph(np.zeros(5, np.int32), np.arange(1, 6, dtype=np.int32),
                        np.arange(5, dtype=np.int64), 6)
    og, tg = pair(T, g)
    omo, tmo = motifs_for(T, W.MOTIFS["3cycle"], 10)
    P, Wt = O.Prep(og, omo), T.Weights(tg, tmo)
    ro, reco = P.sample(1, 50, records=True)
    rg, recg = Wt.sample(1, 50, records=True)
    assert P.W == 0 and Wt.W == 0 and rg.flags & T.TM_F_W_ZERO and rg.estimate == 0.0
    assert rec_equal(reco, recg)
    e = np.zeros(0, np.int64)
    eg = T.Graph(e.astype(np.int32), e.astype(np.int32), e, 4)
    res = T.estimate(eg, tmo, 100, 1)
    assert res.W.value == 0 and res.estimate == 0.0


@pytest.mark.parametrize("m,delta,k", [(3000, 300, 5000), (30000, 2000, 70000)])
def test_estimate_records_match_oracle(T, m, delta, k):
    """tm_estimate with records (70,000 samples take the root-sorted launch)
    and without (the enqueued build-and-sample form below 2^23 edges): every
    record and sum against the oracle's run."""
    g = W.small_graph(m, 23, n=max(60, m // 25), span=40 * delta)
    og, tg = pair(T, g)
    for name in ("4cycle", "lead_trail"):
        edges = dict((c[0], c[1]) for c in MOTIF_CASES)[name]
        omo, tmo = motifs_for(T, edges, delta)
        say("estimate records", m, name)
        ro, reco = O.Prep(og, omo).sample(9, k, records=True)
        rg, recg = T.estimate(tg, tmo, k, 9, records=True)
        assert rec_equal(reco, recg)
        for r in (rg, T.estimate(tg, tmo, k, 9)):
            assert r.acc2.value == ro.acc2.value and r.acc2_sq.value == ro.acc2_sq.value
            assert r.estimate == ro.estimate and r.std_error == ro.std_error


def test_sample_ranges_compose(T):
    g = W.small_graph(20000, 13, n=500, span=100000)
    tg = T.Graph(g.src, g.dst, g.t, g.n)
    Wt = T.Weights(tg, T.make_motif(W.MOTIFS["4cycle"], 2000))
    say("ranges")
    whole, rw = Wt.sample(7, 100000, records=True)
    parts = [Wt.sample(7, 100000, j0=a, count=b - a, records=True)
             for a, b in ((0, 1), (1, 40000), (40000, 99999), (99999, 100000))]
    assert sum(p[0].acc2.value for p in parts) == whole.acc2.value
    assert rec_equal(np.concatenate([p[1] for p in parts]), rw)
    again, _ = Wt.sample(7, 100000)
    assert again.acc2.value == whole.acc2.value and again.estimate == whole.estimate


# ---------------------------------------------------------------------------
# The benchmark workload at full size
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def medium(T):
    g = W.medium_graph()
    og, tg = pair(T, g)
    return g, og, tg


@pytest.mark.parametrize("name", ["4cycle", "4star"])
def test_medium_workload_full_size(T, medium, name):
    """100,000 vertices, 2,000,000 edges; 10^7 samples in the launch shape the
    benchmark times; every weight, W_i, the first 200,000 samples' sum and
    records of four sampled windows against the oracle."""
    g, og, tg = medium
    delta = dict(W.MEDIUM["motifs"])[name]
    omo, tmo = motifs_for(T, W.MOTIFS[name], delta)
    P = O.Prep(og, omo)
    Wt = T.Weights(tg, tmo)
    say("medium", name, "W", P.W)
    assert Wt.W == P.W
    assert Wt.interval_weights() == P.interval_weights()
    for s in list(P.tr.edge)[: P.tr.n_edges]:
        for slot in (0, 1):
            a, b = P.weights(s, slot), Wt.weights(s, slot)
            assert (a["lo"] == b["lo"]).all() and (a["hi"] == b["hi"]).all()
    k, seed = W.MEDIUM["k"], W.MEDIUM["seed"]
    full, _ = Wt.sample(seed, k)
    head_o, _ = P.sample(seed, k, j0=0, count=200_000)
    head_g, _ = Wt.sample(seed, k, j0=0, count=200_000)
    assert head_o.acc2.value == head_g.acc2.value and head_o.n_valid == head_g.n_valid
    for j0 in (0, 3_333_331, 7_000_000, k - 5000):
        ro, reco = P.sample(seed, k, j0=j0, count=5000, records=True)
        rg, recg = Wt.sample(seed, k, j0=j0, count=5000, records=True)
        assert rec_equal(reco, recg), j0
    # the whole run is the sum of its pieces
    pieces = [Wt.sample(seed, k, j0=a, count=b - a)[0] for a, b in
              ((0, 2_500_000), (2_500_000, 6_000_001), (6_000_001, k))]
    assert sum(p.acc2.value for p in pieces) == full.acc2.value
    assert sum(p.n_valid for p in pieces) == full.n_valid
    assert sum(p.acc2_sq.value for p in pieces) == full.acc2_sq.value
    assert full.estimate == float(P.W) * (float(full.acc2.value) / (2.0 * k))
    # the standard error of the whole run: the oracle's evaluation of the same sums
    assert full.std_error == O.std_error(P.W, full.acc2.value, full.acc2_sq.value, k, full.flags)
    assert 0 < full.std_error < 0.05 * full.estimate


# ---------------------------------------------------------------------------
# Constraint ablation: every mode, bit-exact against the oracle's same mode
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", [0, 1, 2, 3], ids=["C1", "C1+2", "C1+3", "C1+2+3"])
@pytest.mark.parametrize("name,edges,delta", MOTIF_CASES[:6], ids=[c[0] for c in MOTIF_CASES[:6]])
def test_constraint_modes_match_oracle(T, mode, name, edges, delta):
    say("constraints", name, mode)
    g = W.small_graph(2500, 41, n=70, span=40 * delta)
    og, tg = pair(T, g)
    for otr in list(all_tree_choices(edges))[:3]:
        check_prep(T, og, tg, edges, delta, otr, seeds=(4,), k=4000, constraints=mode)
    # the root-sorted launch shape (2^16 samples or more)
    check_prep(T, og, tg, edges, delta, O.default_tree(O.make_motif(edges, delta)), seeds=(5,), k=70000,
               constraints=mode)


# ---------------------------------------------------------------------------
# Stage timing
# ---------------------------------------------------------------------------
def test_stage_timing_mask(T):
    """Only the stages selected with tm_profile_stages record time; the
    sums are the same with timing on or off."""
    say("stage timing mask")
    g = W.small_graph(5000, 3, n=300, span=20000)
    mo = T.make_motif(W.MOTIFS["4cycle"], 600)
    k = 1 << 17  # large enough for the root-sorted path (its roots stage)

    def run():
        tg = T.Graph(g.src, g.dst, g.t, g.n)
        w = T.Weights(tg, mo)
        r, _ = w.sample(7, k)
        out = (r.acc2.value, r.n_valid)
        w.close()
        tg.close()
        return out

    T.profile_read(reset=True)
    try:
        plain = run()
        T.profile_stages(["sample"])
        T.profile_enable(True)
        only = run()
        T.profile_enable(False)
        p = dict(zip(T.STAGES, T.profile_read(reset=True)["launches"]))
        assert p["sample"] == 1, p
        assert all(p[s] == 0 for s in T.STAGES if s != "sample"), p
        T.profile_stages(None)
        T.profile_enable(True)
        every = run()
        T.profile_enable(False)
        prof = T.profile_read(reset=True)
        p = dict(zip(T.STAGES, prof["launches"]))
        # the 4-cycle's center has children at both ends: two level passes
        assert all(p[s] == (2 if s == "levels" else 1) for s in T.STAGES), p
        assert all(ms > 0 for ms in prof["ms"]), prof
        assert plain == only == every
    finally:
        T.profile_enable(False)
        T.profile_stages(None)
        T.profile_read(reset=True)


# ---------------------------------------------------------------------------
# Access-model bytes of the level kernels
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scale", [1, 1 << 14], ids=["32_bit_times", "64_bit_times"])
@pytest.mark.parametrize("tree_edges,attach", [([0, 1], "out-list of the center's destination"),
                                               ([0, 2], "in-list of the center's source")])
def test_level_model_bytes_match_host_count(T, tree_edges, attach, scale):
    """tm_weights_model_bytes against the access model counted on the host.

    3-cycle a->b, b->c, c->a with a two-edge tree centred on a->b: one level
    launch over every edge e, whose one leaf child is searched in one list of
    length L_e (b->c: the out-list of e's destination; c->a: the in-list of
    e's source).  Per edge: the walked entry (owner, neighbour, eid: 12 B,
    and its time), the list offsets (8 B), ceil(log2 L) + 1 probes (none for
    an empty list) of each of six bounds: three list times and three 8 B
    keys, the two kept windows (32 B) and the two products (16 B).  A time
    is 4 B when every shifted time is below 2^32 - 1 (the graph as drawn),
    else 8 B (its times scaled by 2^14)."""
    say("level model bytes", tree_edges, scale)
    g = W.small_graph(40000, 4, n=2000, span=10**6)
    t = (g.t - g.t.min()) * scale
    tg = T.Graph(g.src, g.dst, t, g.n)
    tsz = 4 if tg.info()["t_span"] < 2**32 - 1 else 8
    assert tsz == (4 if scale == 1 else 8)
    mo = T.make_motif(W.MOTIFS["3cycle"], 3600 * scale)
    got = T.weights_model_bytes(tg, mo, T.make_tree(tree_edges, 0))
    assert got == T.weights_model_bytes(tg, mo, T.make_tree(tree_edges, 0))
    src, dst = tg.export("src").astype(np.int64), tg.export("dst").astype(np.int64)
    if tree_edges == [0, 1]:
        L = np.bincount(src, minlength=g.n)[dst]
    else:
        L = np.bincount(dst, minlength=g.n)[src]
    steps = np.zeros_like(L)
    n = L.copy()
    while (n > 1).any():
        live = n > 1
        steps[live] += 1
        n[live] -= n[live] >> 1
    expect = int(np.sum(12 + tsz + 8 + (3 * tsz + 24) * (steps + (L > 0)) + 32 + 16))
    tg.close()
    assert got == expect, (attach, got, expect)


# ---------------------------------------------------------------------------
# tm_estimate's enqueued path (weights and sampling with one synchronisation)
# ---------------------------------------------------------------------------
def _same_result(a, b):
    return (a.W.value == b.W.value and a.acc2.value == b.acc2.value and a.acc2_sq.value == b.acc2_sq.value
            and a.n_valid == b.n_valid and a.n_bad_vertex == b.n_bad_vertex and a.n_bad_delta == b.n_bad_delta
            and a.n_bad_order == b.n_bad_order and a.n_nonzero == b.n_nonzero and a.q == b.q and a.k == b.k
            and a.flags == b.flags and a.estimate == b.estimate and a.std_error == b.std_error)


@pytest.mark.parametrize("name,delta,k", [("3cycle", 3600, 5000), ("4cycle", 3600, 100000),
                                          ("6chain", 86400, 70000), ("scatter_gather", 20000, 3000)])
def test_estimate_equals_weights_then_sample(T, name, delta, k):
    """tm_estimate enqueues the 64-bit build and the sampling together and
    reads W with the sums; the result equals a separate build and tm_sample,
    below and above the count that sorts roots."""
    say("estimate enqueued", name, k)
    g = W.small_graph(40000, 4, n=2000, span=10**6)
    tg = T.Graph(g.src, g.dst, g.t, g.n)
    mo = T.make_motif(W.MOTIFS[name], delta)
    one = T.estimate(tg, mo, k, 11)
    w = T.Weights(tg, mo)
    two, _ = w.sample(11, k)
    w.close()
    tg.close()
    assert _same_result(one, two)


def test_estimate_enqueued_falls_back_to_128_bits(T):
    """The hub graph whose weights pass 2^64: the enqueued 64-bit build
    overflows, the kernels draw nothing, and tm_estimate runs the 128-bit
    path; the result equals a separate build and tm_sample."""
    say("estimate 128-bit fallback")
    rng = np.random.default_rng(3)
    hub_n = 1500
    src = np.zeros(hub_n, np.int32)
    dst = np.arange(1, hub_n + 1, dtype=np.int32)
    t = rng.integers(0, 50, hub_n).astype(np.int64)
    tg = T.Graph(src, dst, t, hub_n + 1)
    mo = T.make_motif(tuple((0, j) for j in range(1, 8)), 100)
    one = T.estimate(tg, mo, 70000, 5)
    w = T.Weights(tg, mo)
    assert w.info()["wide"]
    two, _ = w.sample(5, 70000)
    w.close()
    tg.close()
    assert one.W.value >= 2**64 and _same_result(one, two)


def test_estimate_enqueued_zero_weight(T):
    """W = 0 on a non-empty graph (every edge leaves vertex 0): the enqueued
    path reads W = 0 with the sums and returns what tm_sample returns."""
    g = W.TemporalGraph(np.zeros(5, np.int32), np.arange(1, 6, dtype=np.int32),
                        np.arange(5, dtype=np.int64), 6)
    tg = T.Graph(g.src, g.dst, g.t, g.n)
    mo = T.make_motif(W.MOTIFS["3cycle"], 10)
    one = T.estimate(tg, mo, 100, 1)
    w = T.Weights(tg, mo)
    two, _ = w.sample(1, 100)
    w.close()
    tg.close()
    assert one.W.value == 0 and one.flags & T.TM_F_W_ZERO and _same_result(one, two)


def test_estimate_enqueued_two_chunks(T):
    """More samples than one chunk (2^28): the enqueued path keeps reading W
    from the table for the second chunk; the result equals a separate build
    and tm_sample over the same ids."""
    say("estimate enqueued, two chunks")
    g = W.small_graph(5000, 3, n=300, span=20000)
    tg = T.Graph(g.src, g.dst, g.t, g.n)
    mo = T.make_motif(W.MOTIFS["3cycle"], 600)
    k = (1 << 28) + 4096
    one = T.estimate(tg, mo, k, 9)
    w = T.Weights(tg, mo)
    two, _ = w.sample(9, k)
    w.close()
    tg.close()
    assert one.k == k and one.n_valid > 0 and _same_result(one, two)


def test_level_model_bytes_two_passes(T):
    """A level of two passes: the 4-cycle a->b, b->c, c->d, d->a on the path
    tree centred on b->c, whose leaf children attach at both ends.  Pass 0
    walks the out-lists (child a->b: the in-list of e's source, L0 entries);
    pass 1 walks the in-lists (child c->d: the out-list of e's destination,
    L1 entries) and reads the first pass's products through the position
    index (4 B, 8 B per interval of e: two unless e lies in the first
    block); each pass writes its windows at its own walk positions.  List times are
    4 B here (every shifted time is below 2^32 - 1)."""
    say("level model bytes, two passes")
    delta = 3600
    g = W.small_graph(40000, 4, n=2000, span=10**6)
    tg = T.Graph(g.src, g.dst, g.t, g.n)
    mo = T.make_motif(W.MOTIFS["4cycle"], delta)
    got = T.weights_model_bytes(tg, mo, T.make_tree([0, 1, 2], 1))
    src, dst = tg.export("src").astype(np.int64), tg.export("dst").astype(np.int64)
    t = tg.export("t")
    tg.close()

    def steps(L):
        s = np.zeros_like(L)
        n = L.copy()
        while (n > 1).any():
            live = n > 1
            s[live] += 1
            n[live] -= n[live] >> 1
        return s

    L0 = np.bincount(dst, minlength=g.n)[src]
    L1 = np.bincount(src, minlength=g.n)[dst]
    has_b = (t // delta) >= 1
    pass0 = 16 + 8 + 36 * (steps(L0) + (L0 > 0)) + 32 + 16
    pass1 = 16 + 4 + 8 * (1 + has_b) + 8 + 36 * (steps(L1) + (L1 > 0)) + 32 + 16
    expect = int(np.sum(pass0 + pass1))
    assert got == expect, (got, expect)
