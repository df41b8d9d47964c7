"""Parity at the large workload's full size: 2e6 vertices, 1e8 edges (90M
Chung-Lu gamma 2.0 + 10M reciprocated), scatter-gather and 6-chain at delta
86400, sampled in the launch shape the benchmark uses (1e8 samples).

The oracle cannot build whole weight tables at this size, so it checks what
it can compute one by one, and the rest is checked by properties:

* CSR: edges in (time, src, dst) order, the same multiset as generated,
  every vertex list exactly its edges in eid order;
* weights: w_i(s, e) only depends on G_i (every candidate of an edge in I_i
  lies in I_i), so the oracle works on the slice G_i alone (times shifted so
  that I_i becomes its first interval, eids offset by the first eid of I_i):
  sampled weights by its table-free recursive rule, and for two whole
  intervals its full tables against every weight of I_i;
* interval totals W_i: exact sums of the exported center weights;
* samples: a window of per-sample records from the root-sorted path is
  re-derived on the host from the definitions -- the root pair from Philox
  draw 0 over the (interval, eid) prefix, each child by inverse CDF over its
  candidate list (window of the shared vertex's list clipped to I_i, minus
  the excluded far endpoint) with draw index = pre-order slot -- and the
  validation cause and N_phi recomputed (records of the two whole intervals
  among them, so that their picks rest on oracle-fixed weights); M_phi of
  valid samples comes from the oracle on a time slice holding every edge
  within delta of the sample;
* sums: a window's accumulators equal the sums over its records, and the
  full run equals the sum of its two halves.
"""
import itertools
import time

import numpy as np
import pytest

import oracle as O
from paper_2507_20441_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

DELTA = 86400
K = 100_000_000
SEED = 1
M32 = np.uint64(0xFFFFFFFF)


_T0 = time.monotonic()


def say(*a):
    print("[gpu-large] %.1fs" % (time.monotonic() - _T0), *a, flush=True)


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available()
    from paper_2507_20441_amd import timest
    timest.lib()
    return timest


@pytest.fixture(scope="module")
def large(T):
    import torch
    say("generating 1e8 edges on the device")
    u, v, t = W.large_graph_device()
    torch.cuda.synchronize()
    gen = (u.cpu().numpy(), v.cpu().numpy(), t.cpu().numpy())
    g = T.Graph(u, v, t, 2_000_000)
    del u, v, t
    torch.cuda.empty_cache()
    say("exporting")
    H = {k: g.export(k) for k in ("src", "dst", "t", "out_off", "in_off", "out_eid", "in_eid")}
    return g, H, gen


def test_large_csr(T, large):
    g, H, (gu, gv, gt) = large
    src, dst, t = H["src"], H["dst"], H["t"]
    # (time, src, dst) strictly increasing along eids
    dt, ds, dd = np.diff(t), np.diff(src.astype(np.int64)), np.diff(dst.astype(np.int64))
    assert np.all((dt > 0) | ((dt == 0) & ((ds > 0) | ((ds == 0) & (dd > 0)))))
    # the generated multiset, shifted to start at 0
    shift = int(gt.min())
    assert int(t[0]) == 0 and g.m == gu.size

    def fingerprint(a, b, c):
        x = (a.astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15)) ^ (b.astype(np.uint64) * np.uint64(0xC2B2AE3D27D4EB4F))
        x ^= (c.astype(np.uint64) * np.uint64(0x165667B19E3779F9))
        x ^= x >> np.uint64(29)
        return int(np.bitwise_xor.reduce(x)), int(x.sum(dtype=np.uint64))

    assert fingerprint(src, dst, t) == fingerprint(gu, gv, gt - shift)
    # every list: its owner's edges, in eid order
    n = H["out_off"].size - 1
    for off, eid, key in ((H["out_off"], H["out_eid"], src), (H["in_off"], H["in_eid"], dst)):
        owner = np.repeat(np.arange(n, dtype=np.int32), np.diff(off))
        assert np.array_equal(key[eid], owner)
        inc = np.diff(eid.astype(np.int64)) > 0
        starts = np.zeros(eid.size, bool)
        starts[off[1:-1][off[1:-1] < eid.size]] = True
        assert np.all(inc | starts[1:])


# ---------------------------------------------------------------------------
# host side of the definitions
# ---------------------------------------------------------------------------
def rooted(edges, tree):
    """Pre-order slots of the tree rooted at its center: per slot the motif
    edge, its parent slot and the attach vertex (children in increasing pi,
    each subtree before the next sibling)."""
    tset = [tree.edge[x] for x in range(tree.n_edges)]
    c = tree.center
    slots = []

    def visit(s, parent, attach):
        me = len(slots)
        slots.append((s, parent, attach))
        if parent is None:
            ends = {edges[s][0], edges[s][1]}
        else:
            a, b = edges[s]
            ends = {b if a == attach else a}
        kids = []
        for x in tset:
            if x == s or (parent is not None and x == slots[parent][0]):
                continue
            common = {edges[x][0], edges[x][1]} & ends
            if common:
                kids.append((x, common.pop()))
        for x, z in sorted(kids):
            visit(x, me, z)

    visit(c, None, None)
    return slots


class Prefix:
    """Exact prefix sums of 128-bit values (four 32-bit limbs, uint64 sums)."""

    def __init__(self, lo, hi):
        ls = [lo & M32, lo >> np.uint64(32), hi & M32, hi >> np.uint64(32)]
        self.c = [np.concatenate([[np.uint64(0)], np.cumsum(x, dtype=np.uint64)]) for x in ls]

    def at(self, i):
        return sum(int(c[i]) << (32 * k) for k, c in enumerate(self.c))

    def pick(self, r):
        """x with P(x) <= r < P(x + 1)."""
        a, b = 0, self.c[0].size - 1  # P(a) <= r < P(b)
        while b - a > 1:
            m = (a + b) // 2
            if self.at(m) <= r:
                a = m
            else:
                b = m
        return a


def slot_weights(w_exp, eids, blk, i):
    """w_i(s, f) for eids f of I_i from the two exported slots."""
    a, b = w_exp
    use_a = blk[eids] == i
    lo = np.where(use_a, a["lo"][eids], b["lo"][eids])
    hi = np.where(use_a, a["hi"][eids], b["hi"][eids])
    return lo, hi


def slice_graph(H, lo_t, hi_t):
    """The edges with time in [lo_t, hi_t) as an oracle graph, times shifted by
    lo_t; returns it and the first eid of the slice."""
    t = H["t"]
    e0 = int(np.searchsorted(t, lo_t, "left"))
    e1 = int(np.searchsorted(t, hi_t, "left"))
    og = O.Graph(H["src"][e0:e1], H["dst"][e0:e1], t[e0:e1] - lo_t, 2_000_000)
    return og, e0


@pytest.mark.parametrize("name", ["scatter_gather", "6chain"])
def test_large_weights_and_samples(T, large, name):
    g, H, _ = large
    src, dst, t = H["src"], H["dst"], H["t"]
    edges = W.MOTIFS[name]
    mo = T.make_motif(edges, DELTA)
    say(name, "weights")
    w = T.Weights(g, mo)
    info = w.info()
    tr = info["tree"]
    slots = rooted(edges, tr)
    q = info["q"]
    blk = t // DELTA
    ilo = np.searchsorted(t, np.arange(q, dtype=np.int64) * DELTA, "left")
    ihi = np.searchsorted(t, (np.arange(q, dtype=np.int64) + 2) * DELTA, "left")
    nonleaf = [s for s, p, z in slots if any(pp is not None and slots[pp][0] == s for _, pp, _ in slots)]
    center = slots[0][0]
    if center not in nonleaf:
        nonleaf = [center] + nonleaf
    exp = {s: (w.weights(s, 0), w.weights(s, 1)) for s in nonleaf}
    say(name, "W", info["W"], "wide", info["wide"], "q", q)

    # interval totals: exact sums of the exported center weights
    Wi = w.interval_weights()
    for i in range(q):
        ids = np.arange(ilo[i], ihi[i])
        lo, hi = slot_weights(exp[center], ids, blk, i)
        assert Prefix(lo, hi).at(ids.size) == Wi[i], i
    assert sum(Wi) == info["W"]

    rng = np.random.default_rng(5)
    # sampled weights against the oracle on slices G_i
    checked = 0
    for i in rng.choice(np.nonzero(np.array(Wi) > 0)[0], size=3, replace=False):
        og, e0 = slice_graph(H, int(i) * DELTA, (int(i) + 2) * DELTA)
        L = O.Prep(og, O.make_motif(edges, DELTA), O.make_tree(list(tr.edge[:tr.n_edges]), tr.center), light=True)
        for e in rng.integers(ilo[i], ihi[i], size=40):
            for s in nonleaf:
                ow = L.edge_weight(0, s, int(e) - e0, work_limit=4_000_000)
                if ow is None:
                    continue
                a, b = exp[s]
                sl = 0 if blk[e] == i else 1
                x = a if sl == 0 else b
                assert ow == int(x["lo"][e]) | (int(x["hi"][e]) << 64), (i, s, e)
                checked += 1
    say(name, "oracle-checked weights", checked)
    assert checked >= 60

    # the launch shape of the benchmark: one run of 1e8 samples, and its halves
    full, _ = w.sample(SEED, K)
    h1, _ = w.sample(SEED, K, j0=0, count=K // 2)
    h2, _ = w.sample(SEED, K, j0=K // 2, count=K - K // 2)
    assert full.acc2.value == h1.acc2.value + h2.acc2.value
    assert full.n_valid == h1.n_valid + h2.n_valid
    say(name, "estimate", full.estimate, "+-", 1.96 * full.std_error)

    # a window of records (root-sorted path) re-derived on the host
    J, CNT = 37_000_000, 1 << 17
    res, recs = w.sample(SEED, K, j0=J, count=CNT, k_total=K, records=True)
    acc2 = sum(2 * (int(r["m_lo"]) | (int(r["m_hi"]) << 64)) // int(r["n_phi"])
               for r in recs if r["status"] == 0)
    assert acc2 == res.acc2.value and int((recs["status"] == 0).sum()) == res.n_valid
    Wtot = info["W"]
    cum = list(itertools.accumulate([0] + Wi))  # exact: W_i may exceed 2^64
    by_pi = sorted(s for s, _, _ in slots)
    slot_of = {s: x for x, (s, _, _) in enumerate(slots)}
    kverts = 1 + max(max(e) for e in edges)
    lists = {0: (H["out_off"], H["out_eid"]), 1: (H["in_off"], H["in_eid"])}
    # whole intervals: for the two intervals holding the most records of the
    # window (slices of at most 7e5 edges), the oracle's full weight tables
    # on G_i against every exported s-weight of I_i; the records of those
    # intervals are then re-derived below from weights the oracle fixed
    ivs, cnts = np.unique(recs["interval"], return_counts=True)
    full_iv = [int(i) for i in ivs[np.argsort(-cnts, kind="stable")] if ihi[i] - ilo[i] <= 700_000][:2]
    for i in full_iv:
        og, e0 = slice_graph(H, i * DELTA, (i + 2) * DELTA)
        assert e0 == ilo[i] and og.m == ihi[i] - ilo[i]
        F = O.Prep(og, O.make_motif(edges, DELTA), O.make_tree(list(tr.edge[:tr.n_edges]), tr.center))
        assert F.interval_weights()[0] == Wi[i], i
        ids = np.arange(ilo[i], ihi[i])
        # interval 0 of the slice is I_i; the oracle keeps w_0 of an edge of
        # its block b (of its own shifted times) in slot b
        sb = (t[ilo[i]:ihi[i]] - i * DELTA - og.shift) // DELTA
        assert sb.min() >= 0 and sb.max() <= 1
        for s in nonleaf:
            o0, o1 = F.weights(s, 0), F.weights(s, 1)
            lo, hi = slot_weights(exp[s], ids, blk, i)
            assert np.array_equal(np.where(sb == 0, o0["lo"], o1["lo"]), lo), (i, s)
            assert np.array_equal(np.where(sb == 0, o0["hi"], o1["hi"]), hi), (i, s)
        del F, og
    say(name, "intervals with every weight oracle-checked", full_iv,
        [int(ihi[i] - ilo[i]) for i in full_iv])
    assert len(full_iv) == 2
    pick_idx = rng.choice(CNT, size=250, replace=False)
    in_full = np.nonzero(np.isin(recs["interval"], full_iv))[0][:200]
    pick_idx = np.union1d(pick_idx, in_full)
    slices = {}
    n_valid_checked = 0
    for x in pick_idx:
        r = recs[x]
        j = J + int(x)
        i = int(r["interval"])
        m_of = {by_pi[a]: int(r["eid"][a]) for a in range(len(by_pi))}
        # root: draw 0 over the (interval, eid) prefix
        r0 = O.draw(SEED, j, 0, Wtot)
        assert cum[i] <= r0 < cum[i + 1], j
        ids = np.arange(ilo[i], ihi[i])
        lo, hi = slot_weights(exp[center], ids, blk, i)
        assert ids[Prefix(lo, hi).pick(r0 - cum[i])] == m_of[center], j
        # children in pre-order, draw index = slot
        for d in range(1, len(slots)):
            s, p, z = slots[d]
            ps = slots[p][0]
            pe = m_of[ps]
            pu, pv = int(src[pe]), int(dst[pe])
            gv, ov = (pu, pv) if z == edges[ps][0] else (pv, pu)
            dirn = 0 if edges[s][0] == z else 1
            off, leid = lists[dirn]
            cand = leid[off[gv]:off[gv + 1]]
            ct = t[cand]
            pt = int(t[pe])
            wlo, whi = (pt - DELTA, pt) if s < ps else (pt, pt + DELTA)
            wlo, whi = max(wlo, i * DELTA), min(whi, (i + 2) * DELTA - 1)
            cand = cand[(ct >= wlo) & (ct <= whi)]
            far = dst[cand] if dirn == 0 else src[cand]
            cand = cand[far != ov]
            if s in exp:
                clo, chi = slot_weights(exp[s], cand, blk, i)
            else:
                clo, chi = np.ones(cand.size, np.uint64), np.zeros(cand.size, np.uint64)
            P = Prefix(clo, chi)
            n = P.at(cand.size)
            assert n > 0, (j, s)
            rr = O.draw(SEED, j, d, n)
            assert cand[P.pick(rr)] == m_of[s], (j, s)
        # validation cause and N_phi
        img = {}
        bad_vertex = False
        for s, e in m_of.items():
            for mv, gvv in ((edges[s][0], int(src[e])), (edges[s][1], int(dst[e]))):
                if img.setdefault(mv, gvv) != gvv:
                    bad_vertex = True
        times = [int(t[m_of[s]]) for s in by_pi]
        if bad_vertex or len(set(img.values())) < kverts:
            want = 1
        elif max(times) - min(times) > DELTA:
            want = 2
        elif any(a >= b for a, b in zip(times, times[1:])):
            want = 3
        else:
            want = 0
        assert int(r["status"]) == want, j
        if want == 0:
            tmin, tmax = min(times), max(times)
            nphi = sum(1 for ii in range(max(0, tmin // DELTA - 1), tmin // DELTA + 2)
                       if ii < q and ii * DELTA <= tmin and tmax < (ii + 2) * DELTA)
            assert int(r["n_phi"]) == nphi, j
            key = i
            if key not in slices:
                og, e0 = slice_graph(H, max(0, i * DELTA - DELTA), (i + 2) * DELTA + DELTA)
                slices[key] = (og, e0, O.Prep(og, O.make_motif(edges, DELTA),
                                              O.make_tree(list(tr.edge[:tr.n_edges]), tr.center), light=True))
            og, e0, L = slices[key]
            mphi = L.derive_cnt(np.array([int(r["eid"][a]) - e0 for a in range(len(by_pi))] + [-1] * (8 - len(by_pi)),
                                         np.int32))
            assert mphi == (int(r["m_lo"]) | (int(r["m_hi"]) << 64)), j
            n_valid_checked += 1
    say(name, "records re-derived", len(pick_idx), "of them in oracle-checked intervals", in_full.size,
        "valid", n_valid_checked)
    assert in_full.size >= 100
    w.close()
