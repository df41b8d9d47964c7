"""Serving loop: queries answered by the server are bit-identical to the same
query run alone with tm_estimate, whatever else is in the mix, however the
budget forces weight sets out and back in, and however a query's samples are
split across passes; a few are also checked against the oracle."""
import threading

import numpy as np
import pytest

import oracle as O
from paper_2507_20441_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-serve]", *a, flush=True)


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available()
    from paper_2507_20441_amd import timest
    timest.lib()
    return timest


def same(a, b):
    return (a.acc2.value == b.acc2.value and a.acc2_sq.value == b.acc2_sq.value
            and a.n_valid == b.n_valid and a.n_bad_vertex == b.n_bad_vertex
            and a.n_bad_delta == b.n_bad_delta and a.n_bad_order == b.n_bad_order
            and a.n_nonzero == b.n_nonzero and a.W.value == b.W.value
            and a.estimate == b.estimate and a.flags == b.flags and a.k == b.k)


@pytest.fixture(scope="module")
def world(T):
    """Three resident graphs and 40 queries: every motif, several deltas,
    repeated (graph, motif, delta) sets, uneven budgets, a zero-sample query."""
    gs = [W.small_graph(m, s, n=max(50, m // 20), span=20 * m) for m, s in ((4000, 11), (30000, 12), (90000, 13))]
    tg = [T.Graph(g.src, g.dst, g.t, g.n) for g in gs]
    rng = np.random.default_rng(21)
    names = list(W.MOTIFS)
    deltas = [[300, 1500], [2000, 9000], [5000, 40000]]
    qs = []
    for i in range(40):
        gi = int(rng.integers(3))
        name = names[int(rng.integers(len(names)))]
        delta = deltas[gi][int(rng.integers(2))]
        k = int(10 ** rng.uniform(2, 5.3))
        qs.append((gi, name, delta, k, int(rng.integers(1, 2 ** 62))))
    qs.append((0, "4cycle", 300, 0, 5))
    alone = []
    for gi, name, delta, k, seed in qs:
        alone.append(T.estimate(tg[gi], T.make_motif(W.MOTIFS[name], delta), k, seed))
    return gs, tg, qs, alone


def run_mix(T, tg, qs, **opts):
    srv = T.Server(**opts)
    try:
        gids = [srv.add_graph(g) for g in tg]
        tickets = [srv.submit(gids[gi], T.make_motif(W.MOTIFS[name], delta), k, seed)
                   for gi, name, delta, k, seed in qs]
        out = [srv.wait(t) for t in tickets]
        return out, srv.stats()
    finally:
        srv.close()


@pytest.mark.parametrize("fifo", [False, True])
def test_mix_matches_alone(T, world, fifo):
    gs, tg, qs, alone = world
    say("mix fifo", fifo)
    out, st = run_mix(T, tg, qs, budget_bytes=1 << 32, pass_samples=1 << 15, job_chunk=1 << 12, fifo=fifo)
    for i, ((r, info), a) in enumerate(zip(out, alone)):
        assert r.status == 0 and same(r, a), (i, qs[i])
        assert info.latency_ms >= info.queued_ms >= 0
    assert st["completed"] == len(qs) and st["failed"] == 0
    assert st["passes"] > 1 and st["weight_hits"] > 0
    assert max(info.passes for _, info in out) > 1


def test_budget_forces_eviction(T, world):
    gs, tg, qs, alone = world
    # room for the largest single weight set and little more
    wide = [bool(a.flags & T.TM_F_WIDE) for a in alone]
    # a build holds one slot's 64-bit values per parity on top of the tables
    extra = [2 * ((tg[gi].m * 8 + 255) & ~255) for gi, *_ in qs]
    need = max(T.weights_footprint(tg[gi], T.make_motif(W.MOTIFS[name], delta), wide=wd) + x
               for (gi, name, delta, _, _), wd, x in zip(qs, wide, extra))
    budget = 24 * (1 << 14) + need + need // 4
    say("evict budget", budget, "wide sets", sum(wide))
    out, st = run_mix(T, tg, qs, budget_bytes=budget, pass_samples=1 << 14, job_chunk=1 << 11)
    for i, ((r, _), a) in enumerate(zip(out, alone)):
        assert r.status == 0 and same(r, a), (i, qs[i])
    assert st["evictions"] > 0 and st["admission_waits"] > 0
    # the budget is a hard bound, 128-bit sets included
    assert st["peak_bytes"] <= budget


def test_wide_set_reserves_its_128_bit_size(T):
    """A set that needs 128 bits (an 8-vertex star on a 1,500-edge hub) in
    a server whose budget holds it only after the 64-bit sets are evicted:
    the 64-bit attempt stops, the query comes back with the 128-bit
    reservation, later queries of that set reserve 128 bits at once, every
    result equals its run alone and the budget holds throughout."""
    rng = np.random.default_rng(3)
    hub = 1500
    star = W.TemporalGraph(np.zeros(hub, np.int32), np.arange(1, hub + 1, dtype=np.int32),
                           rng.integers(0, 50, hub).astype(np.int64), hub + 1)
    gs = T.Graph(star.src, star.dst, star.t, star.n)
    g2 = W.small_graph(20000, 81, n=500, span=400000)
    gt = T.Graph(g2.src, g2.dst, g2.t, g2.n)
    smo = T.make_motif(tuple((0, j) for j in range(1, 8)), 100)
    big = T.weights_footprint(gs, smo, wide=True) + 4 * ((hub * 16 + 255) & ~255) + (1 << 20)
    mos = [T.make_motif(W.MOTIFS[nm], d) for nm, d in (("4cycle", 3000), ("3cycle", 2000), ("4star", 1000))]
    small = max(T.weights_footprint(gt, mo) for mo in mos) + 4 * ((20000 * 8 + 255) & ~255) + (1 << 20)
    reserve = 24 * (1 << 14)
    budget = reserve + max(big, 2 * small) + small // 2
    say("wide budget", budget, big, small)
    srv = T.Server(budget, pass_samples=1 << 14, job_chunk=1 << 12)
    a, b = srv.add_graph(gs), srv.add_graph(gt)
    jobs = [(b, mos[0], 30000, 1), (a, smo, 20000, 5), (b, mos[1], 20000, 2), (b, mos[2], 10000, 3),
            (a, smo, 7000, 6), (b, mos[0], 5000, 4)]
    tickets = [srv.submit(g, mo, k, s) for g, mo, k, s in jobs]
    outs = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    for (g, mo, k, s), (r, _) in zip(jobs, outs):
        alone = T.estimate(gs if g == a else gt, mo, k, s)
        assert r.status == 0 and same(r, alone)
    assert outs[1][0].flags & T.TM_F_WIDE
    assert st["peak_bytes"] <= budget and st["failed"] == 0


def test_pass_retry_after_a_failed_allocation(T):
    """A sampling pass whose device allocation fails (injected through the
    server's allocator once its weight sets are resident) waits for any build
    in flight, returns cached blocks and runs again; every result still
    equals the same query alone."""
    g = W.small_graph(20000, 82, n=500, span=400000)
    tg = T.Graph(g.src, g.dst, g.t, g.n)
    A = T.TorchAllocator()
    srv = T.Server(4 << 30, pass_samples=1 << 16, job_chunk=1 << 14, allocator=A)
    gid = srv.add_graph(tg)
    mos = [T.make_motif(W.MOTIFS[nm], 3000) for nm in ("4cycle", "3cycle")]
    for mo in mos:
        srv.wait(srv.submit(gid, mo, 0, 1))   # sets resident
    A.fail_next = 1                           # the next allocation fails: a pass's
    jobs = [(mos[0], 200000, 7), (mos[1], 100000, 8)]
    tickets = [srv.submit(gid, mo, k, s) for mo, k, s in jobs]
    outs = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["pass_retries"] >= 1 and A.failed == 1
    for (mo, k, s), (r, _) in zip(jobs, outs):
        assert r.status == 0 and same(r, T.estimate(tg, mo, k, s))
    assert A.live_bytes == 0


def test_footprint_matches_build(T, world):
    gs, tg, qs, alone = world
    for gi, name, delta, _, _ in qs[:10]:
        mo = T.make_motif(W.MOTIFS[name], delta)
        w = T.Weights(tg[gi], mo)
        info = w.info()
        if info["wide"]:
            # widened after a 64-bit build: 64-bit list tables, 128-bit center
            assert T.weights_footprint(tg[gi], mo, wide=False) < info["bytes"] <= \
                T.weights_footprint(tg[gi], mo, wide=True)
        else:
            assert T.weights_footprint(tg[gi], mo, wide=False) == info["bytes"]
        w.close()


def test_oracle_agrees(T, world):
    gs, tg, qs, alone = world
    g = gs[0]
    og = O.Graph(g.src, g.dst, g.t, g.n)
    srv = T.Server(1 << 30, pass_samples=1 << 13, job_chunk=1 << 10)
    try:
        gid = srv.add_graph(tg[0])
        cases = [("3cycle", 300, 5000, 3), ("4cycle", 1500, 7000, 4), ("scatter_gather", 1500, 3000, 5)]
        tickets = [srv.submit(gid, T.make_motif(W.MOTIFS[n], d), k, s) for n, d, k, s in cases]
        for (n, d, k, s), t in zip(cases, tickets):
            r, _ = srv.wait(t)
            P = O.Prep(og, O.make_motif(W.MOTIFS[n], d))
            o = P.sample(s, k)[0]
            assert r.acc2.value == o.acc2.value and r.W.value == P.W and r.n_valid == o.n_valid, n
            assert r.estimate == o.estimate and r.std_error == o.std_error
    finally:
        srv.close()


def test_oracle_agrees_beyond_32_bit_times(T):
    """Server sets search their child windows (they keep none): on a graph
    whose shifted times exceed 32 bits the lists hold 64-bit times, and
    served results still equal the oracle's."""
    g = W.small_graph(4000, 11, n=200, span=80000)
    t = (g.t - g.t.min()) * (1 << 17)
    og = O.Graph(g.src, g.dst, t, g.n)
    tg = T.Graph(g.src, g.dst, t, g.n)
    assert tg.info()["t_span"] >= 2**32
    srv = T.Server(1 << 30, pass_samples=1 << 13, job_chunk=1 << 10)
    try:
        gid = srv.add_graph(tg)
        cases = [("3cycle", 300 << 17, 5000, 3), ("4cycle", 1500 << 17, 7000, 4),
                 ("scatter_gather", 1500 << 17, 3000, 5)]
        tickets = [srv.submit(gid, T.make_motif(W.MOTIFS[n], d), k, s) for n, d, k, s in cases]
        for (n, d, k, s), tk in zip(cases, tickets):
            r, _ = srv.wait(tk)
            P = O.Prep(og, O.make_motif(W.MOTIFS[n], d))
            o = P.sample(s, k)[0]
            assert r.acc2.value == o.acc2.value and r.W.value == P.W and r.n_valid == o.n_valid, n
            assert r.estimate == o.estimate and r.std_error == o.std_error
    finally:
        srv.close()


def test_release_cached_returns_blocks(T):
    """tm_release_cached: the blocks a graph build released go back to HIP
    (free device memory rises), and later calls still give the same results."""
    import torch
    g = W.small_graph(400000, 17, n=20000, span=4000000)
    tg = T.Graph(g.src, g.dst, g.t, g.n)
    mo = T.make_motif(W.MOTIFS["4cycle"], 3600)
    a = T.estimate(tg, mo, 50000, 7)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    T.release_cached()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 > free0, (free0, free1)
    b = T.estimate(tg, mo, 50000, 7)
    assert same(a, b)
    tg.close()


def test_concurrent_submitters(T, world):
    gs, tg, qs, alone = world
    srv = T.Server(1 << 32, pass_samples=1 << 15, job_chunk=1 << 12)
    gids = [srv.add_graph(g) for g in tg]
    results = [None] * len(qs)

    def client(part):
        for i in range(part, len(qs), 4):
            gi, name, delta, k, seed = qs[i]
            t = srv.submit(gids[gi], T.make_motif(W.MOTIFS[name], delta), k, seed)
            results[i] = srv.wait(t)

    th = [threading.Thread(target=client, args=(p,)) for p in range(4)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    srv.close()
    for i, (r, _) in enumerate(results):
        assert same(r, alone[i]), i


def test_errors(T, world):
    gs, tg, qs, alone = world
    with pytest.raises(T.TimestError) as e:
        T.Server(1000, pass_samples=1 << 10)
    assert e.value.code == T.TM_EINVAL
    srv = T.Server(24 * (1 << 10) + 4096, pass_samples=1 << 10, job_chunk=1 << 10)
    try:
        gid = srv.add_graph(tg[2])
        with pytest.raises(T.TimestError) as e:
            srv.submit(gid, T.make_motif(W.MOTIFS["6chain"], 5000), 100, 1)
        assert e.value.code == T.TM_EADMIT
        with pytest.raises(T.TimestError) as e:
            srv.submit(7, T.make_motif(W.MOTIFS["3cycle"], 5000), 100, 1)
        assert e.value.code == T.TM_EINVAL
        with pytest.raises(T.TimestError) as e:
            srv.wait(12345)
        assert e.value.code == T.TM_EINVAL
    finally:
        srv.close()


def test_shutdown_with_pending(T, world):
    gs, tg, qs, alone = world
    srv = T.Server(1 << 32, pass_samples=1 << 12, job_chunk=1 << 10)
    gid = srv.add_graph(tg[2])
    for i in range(8):
        srv.submit(gid, T.make_motif(W.MOTIFS["4star"], 40000), 200000, i + 1)
    srv.close()


def test_torch_allocator_serves_every_device_block(T):
    """A graph and a server given PyTorch's caching allocator (tm_allocator):
    every device block of the graph, its weight sets, the calls' temporaries
    and the server's sets and passes comes from it and goes back to it, and
    every result is bit-identical to the library's own allocator."""
    import torch
    g = W.small_graph(20011, 71, n=400, span=20 * 20011)
    plain = T.Graph(g.src, g.dst, g.t, g.n)
    A = T.TorchAllocator()
    base = torch.cuda.memory_allocated()
    hooked = T.Graph(g.src, g.dst, g.t, g.n, allocator=A)
    assert A.allocs > 0 and A.live_bytes > 0
    assert torch.cuda.memory_allocated() - base >= A.live_bytes   # torch accounts for them
    graph_bytes = A.live_bytes
    for name in ("4cycle", "scatter_gather"):
        mo = T.make_motif(W.MOTIFS[name], 4000)
        for k in (5000, 70000):
            a = T.estimate(plain, mo, k, 3)
            b = T.estimate(hooked, mo, k, 3)
            assert same(a, b), (name, k)
        wa, wb = T.Weights(plain, mo), T.Weights(hooked, mo)
        assert A.live_bytes > graph_bytes
        assert same(wa.sample(5, 80000)[0], wb.sample(5, 80000)[0])
        assert (wa.weights(1, 0) == wb.weights(1, 0)).all()
        wa.close()
        wb.close()
    assert A.live_bytes == graph_bytes          # the weight sets gave theirs back
    bat = T.estimate_batch([hooked, hooked], [T.make_motif(W.MOTIFS["3cycle"], 2000)] * 2, [30000, 70000], [1, 2])
    ref = T.estimate_batch([plain, plain], [T.make_motif(W.MOTIFS["3cycle"], 2000)] * 2, [30000, 70000], [1, 2])
    assert all(same(x, y) for x, y in zip(bat, ref))
    # a server with its own torch allocator
    S = T.TorchAllocator()
    srv = T.Server(8 << 30, allocator=S)
    gid = srv.add_graph(plain)
    mo = T.make_motif(W.MOTIFS["4cycle"], 4000)
    tickets = [srv.submit(gid, mo, k, s) for k, s in ((20000, 1), (300000, 2))]
    for t, (k, s) in zip(tickets, ((20000, 1), (300000, 2))):
        r, _ = srv.wait(t)
        assert same(r, T.estimate(plain, mo, k, s))
    assert S.allocs > 0
    srv.close()
    assert S.live_bytes == 0
    hooked.close()
    assert A.live_bytes == 0 and A.frees == A.allocs
