"""tm_sample_noalloc (sampling with its temporaries in a fixed device array,
for callers that cannot allocate) against tm_sample through the C ABI: the
same records and the same exact sums on consecutive calls, the second
smaller than the first, for 64- and 128-bit weight sets; the per-call limit
is enforced."""
import numpy as np
import pytest

from paper_2507_20441_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-noalloc]", *a, flush=True)


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "no HIP device"
    from paper_2507_20441_amd import timest
    timest.lib()
    return timest


def recs_of(T, count):
    import torch
    return torch.empty(max(1, count) * T.REC_DTYPE.itemsize, dtype=torch.uint8, device="cuda")


def same_sums(a, b):
    return (a.acc2.value == b.acc2.value and a.acc2_sq.value == b.acc2_sq.value and a.n_valid == b.n_valid
            and a.n_bad_vertex == b.n_bad_vertex and a.n_bad_delta == b.n_bad_delta
            and a.n_bad_order == b.n_bad_order and a.n_nonzero == b.n_nonzero and a.W.value == b.W.value
            and a.k == b.k and a.flags == b.flags and a.estimate == b.estimate and a.std_error == b.std_error)


def weight_sets(T):
    g = W.small_graph(20011, 61, n=400, span=20 * 20011)
    tg = T.Graph(g.src, g.dst, g.t, g.n)
    rng = np.random.default_rng(3)
    hub = 1500
    star = W.TemporalGraph(np.zeros(hub, np.int32), np.arange(1, hub + 1, dtype=np.int32),
                           rng.integers(0, 50, hub).astype(np.int64), hub + 1)
    sg = T.Graph(star.src, star.dst, star.t, star.n)
    return [("4cycle", tg, T.Weights(tg, T.make_motif(W.MOTIFS["4cycle"], 4000))),
            ("lead_trail", tg, T.Weights(tg, T.make_motif(((0, 1), (1, 2), (2, 3), (3, 0), (0, 2)), 4000))),
            ("wide_star", sg, T.Weights(sg, T.make_motif(tuple((0, j) for j in range(1, 8)), 100)))]


def test_noalloc_equals_sample_on_consecutive_calls(T):
    sets = weight_sets(T)
    assert sets[2][2].info()["wide"]
    for name, _, w in sets:
        # first a root-sorted run (2^16 samples or more), then a smaller one
        for j0, count in ((1000, 300_000), (77, 5000)):
            say(name, j0, count)
            buf = recs_of(T, count)
            got = T.sample_noalloc(w, 9, count, j0=j0, k_total=count, recs_ptr=buf.data_ptr())
            recs = buf[: count * T.REC_DTYPE.itemsize].cpu().numpy().view(T.REC_DTYPE)
            ref, rrec = w.sample(9, count, j0=j0, count=count, k_total=count, records=True)
            assert same_sums(got, ref), (name, count)
            assert (recs == rrec).all(), (name, count)
            assert got.status == 0


def test_noalloc_limit_and_edges(T):
    name, _, w = weight_sets(T)[0]
    big = 1 << 21
    say("limit", big)
    got = T.sample_noalloc(w, 4, big)
    ref, _ = w.sample(4, big)
    assert same_sums(got, ref)
    with pytest.raises(T.TimestError) as e:
        T.sample_noalloc(w, 4, big + 1)
    assert e.value.code == T.TM_EINVAL
    z = T.sample_noalloc(w, 4, 0)
    assert z.acc2.value == 0 and z.n_valid == 0
