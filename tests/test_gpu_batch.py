"""Batched estimation: each job's result in a batch is bit-identical to the
oracle's run of the same job (graph, motif, default tree, k, seed) and to
the same job run alone on the GPU (the draws are keyed by (seed, sample id);
the batch only changes the schedule)."""
import numpy as np
import pytest

import oracle as O
from paper_2507_20441_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-batch]", *a, flush=True)


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
            and a.estimate == b.estimate and a.flags == b.flags)


@pytest.fixture(scope="module")
def mix(T):
    """Jobs over four graphs: every motif, a general-run motif, a 128-bit job,
    a zero-weight job and a zero-sample job, uneven budgets.  Each job also
    carries the oracle's result for it."""
    graphs = [W.small_graph(m, s, n=max(50, m // 20), span=20 * m)
              for m, s in ((3000, 1), (20011, 2), (120000, 3), (700, 4))]
    rng = np.random.default_rng(5)
    hub = 1500
    graphs.append(W.TemporalGraph(np.zeros(hub, np.int32), np.arange(1, hub + 1, dtype=np.int32),
                                  rng.integers(0, 50, hub).astype(np.int64), hub + 1))
    graphs.append(W.TemporalGraph(np.zeros(5, np.int32), np.arange(1, 6, dtype=np.int32),
                                  np.arange(5, dtype=np.int64), 6))
    tg = [T.Graph(g.src, g.dst, g.t, g.n) for g in graphs]
    og = [O.Graph(g.src, g.dst, g.t, g.n) for g in graphs]
    spec = []
    names = list(W.MOTIFS)
    for i in range(14):
        gi = i % 4
        name = names[i % len(names)]
        delta = [400, 3000, 20000, 150][gi]
        spec.append((gi, W.MOTIFS[name], delta, int(rng.integers(1, 3)) * 10 ** int(rng.integers(3, 6)),
                     int(rng.integers(1, 2 ** 62))))
    spec.append((1, ((0, 1), (1, 2), (2, 3), (3, 0), (0, 2)), 5000, 30000, 77))
    spec.append((4, tuple((0, j) for j in range(1, 8)), 100, 20000, 5))
    spec.append((5, W.MOTIFS["3cycle"], 10, 1000, 3))
    spec.append((0, W.MOTIFS["4cycle"], 400, 0, 9))
    jobs, ref = [], []
    for gi, edges, delta, k, seed in spec:
        jobs.append((tg[gi], T.make_motif(edges, delta), k, seed))
        P = O.Prep(og[gi], O.make_motif(edges, delta))
        ref.append(P.sample(seed, k)[0])
    say("oracle results ready", len(ref))
    return tg, jobs, ref


def same_as_oracle(g, o):
    """Every field of the GPU result against the oracle's, bit for bit."""
    return (g.status == 0 and g.W.value == o.W.value and g.acc2.value == o.acc2.value
            and g.acc2_sq.value == o.acc2_sq.value and g.n_valid == o.n_valid
            and g.n_bad_vertex == o.n_bad_vertex and g.n_bad_delta == o.n_bad_delta
            and g.n_bad_order == o.n_bad_order and g.n_nonzero == o.n_nonzero and g.k == o.k
            and g.q == o.q and g.estimate == o.estimate and g.std_error == o.std_error
            and (g.flags & 3) == (o.flags & 3))


@pytest.mark.parametrize("tile,blocks", [(8192, 0), (256, 7), (1024, 64)])
def test_sample_batch_matches_single_runs(T, mix, tile, blocks):
    tg, jobs, ref = mix
    prev = T.batch_config(tile, blocks)
    try:
        ws = [T.Weights(g, mo) for g, mo, _, _ in jobs]
        say("batch", tile, blocks, len(ws))
        got = T.sample_batch(ws, [k for *_, k, _ in jobs], [s for *_, s in jobs])
        for i, ((g, mo, k, seed), w) in enumerate(zip(jobs, ws)):
            alone, _ = w.sample(seed, k)
            assert got[i].status == 0 and same(got[i], alone), i
            assert same_as_oracle(got[i], ref[i]), i
        assert ws[15].info()["wide"] and got[16].flags & T.TM_F_W_ZERO
    finally:
        T.batch_config(*prev)


def test_estimate_batch_matches_estimate(T, mix):
    tg, jobs, ref = mix
    say("estimate_batch")
    got = T.estimate_batch([g for g, *_ in jobs], [mo for _, mo, _, _ in jobs],
                           [k for *_, k, _ in jobs], [s for *_, s in jobs])
    for i, (g, mo, k, seed) in enumerate(jobs):
        alone = T.estimate(g, mo, k, seed)
        assert got[i].status == 0 and same(got[i], alone), i
        assert same_as_oracle(got[i], ref[i]), i


@pytest.mark.parametrize("limit", [1, 60000, 300000])
def test_batch_split_into_many_passes_matches_oracle(T, mix, limit):
    """A small per-pass limit of root keys and samples splits the batch into
    several passes (limit 1: every job in a pass of its own; 60,000: jobs on
    the 120,000-edge graph alone, small ones grouped), through both the eager
    batch and the recorded plan; each job still equals the oracle's run."""
    tg, jobs, ref = mix
    prev = T.batch_options(group_limit=limit, tile=2048)
    try:
        say("split", limit)
        gs = [g for g, *_ in jobs]
        mos = [mo for _, mo, _, _ in jobs]
        ks = [k for *_, k, _ in jobs]
        ss = [s for *_, s in jobs]
        got = T.estimate_batch(gs, mos, ks, ss)
        for i in range(len(jobs)):
            assert same_as_oracle(got[i], ref[i]), (limit, i)
        plan = T.BatchPlan(gs, mos, ks, ss)
        try:
            for rep in range(2):
                got = plan.run()
                for i in range(len(jobs)):
                    assert same_as_oracle(got[i], ref[i]), (limit, rep, i)
        finally:
            plan.close()
    finally:
        T.batch_options(**prev)


def test_root_lds_staging_sizes_give_identical_results(T, mix):
    """The root draws' LDS staging of W_i (root_lds) changes no result."""
    tg, jobs, ref = mix
    ws = [T.Weights(g, mo) for g, mo, _, _ in jobs[:8]]
    ks = [k for *_, k, _ in jobs[:8]]
    ss = [s for *_, s in jobs[:8]]
    for lds in (0, 4096, 65536):
        prev = T.batch_options(root_lds=lds)
        try:
            say("root_lds", lds)
            got = T.sample_batch(ws, ks, ss)
            for i in range(8):
                assert same_as_oracle(got[i], ref[i]), (lds, i)
        finally:
            T.batch_options(**prev)


def test_batch_repeats_identically(T, mix):
    tg, jobs, ref = mix
    ws = [T.Weights(g, mo) for g, mo, _, _ in jobs[:6]]
    ks = [k for *_, k, _ in jobs[:6]]
    ss = [s for *_, s in jobs[:6]]
    first = T.sample_batch(ws, ks, ss)
    for rep in range(3):
        ws[0].sample(123, 5000)  # eager work in between
        again = T.sample_batch(ws, ks, ss)
        assert all(same(a, b) for a, b in zip(first, again)), rep


def test_batch_plan_replays(T, mix):
    """The recorded pipeline, replayed three times with other library work and
    synchronisations between the replays, equals the eager batch every time;
    the 128-bit job is re-run eagerly after each replay."""
    import torch
    tg, jobs, oref = mix
    gs = [g for g, *_ in jobs]
    mos = [mo for _, mo, _, _ in jobs]
    ks = [k for *_, k, _ in jobs]
    ss = [s for *_, s in jobs]
    ref = T.estimate_batch(gs, mos, ks, ss)
    say("plan create")
    plan = T.BatchPlan(gs, mos, ks, ss)
    prev = T.batch_config(512, 3)  # a later schedule change does not touch the recording
    try:
        for rep in range(3):
            say("replay", rep)
            got = plan.run()
            for i, (a, b) in enumerate(zip(got, ref)):
                assert a.status == b.status and same(a, b), (rep, i)
                assert same_as_oracle(a, oref[i]), (rep, i)
            T.estimate(gs[1], mos[1], 5000, 3 + rep)
            torch.cuda.synchronize()
    finally:
        T.batch_config(*prev)
        plan.close()


def test_batch_of_many_jobs_reads_back_directly(T, mix):
    """220 jobs: their sums (over 16 KiB) are read back straight into host
    memory instead of through the pinned staging block; each job still equals
    its run alone."""
    tg, jobs, ref = mix
    ws = [T.Weights(tg[0], T.make_motif(W.MOTIFS["3cycle"], 400)),
          T.Weights(tg[1], T.make_motif(W.MOTIFS["4cycle"], 3000))]
    n = 220
    batch_ws = [ws[i % 2] for i in range(n)]
    ks = [1000 + 37 * i for i in range(n)]
    seeds = [1000003 * i + 17 for i in range(n)]
    say("many jobs", n)
    got = T.sample_batch(batch_ws, ks, seeds)
    for i in range(n):
        alone, _ = batch_ws[i].sample(seeds[i], ks[i])
        assert got[i].status == 0 and same(got[i], alone), i
