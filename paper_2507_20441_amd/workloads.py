"""Seeded synthetic temporal graphs and motifs shaped like TIMEST's workloads.

The paper evaluates on wiki-talk, stackoverflow, bitcoin and reddit-reply
(Tab. "dataset"): power-law degree distributions, bursty activity, spans of
years, delta of hours to weeks.  Those datasets are not available here, so
these seeded generators stand in for them at matching scale and shape.  This
module only draws inputs; it holds none of the estimator's arithmetic and is
the one piece of code shared by the GPU path's tests and the oracle's.

Graph recipe (per config):
  * Chung-Lu: vertex r has weight (r+1)^(-1/(gamma-1)); ids are a seeded
    permutation; source and destination are drawn independently in
    proportion to weight; self loops are redrawn.
  * Times: uniform integers, or bursty per-source renewal processes with
    Pareto(alpha=1.5) gaps (mean span S per source, wrapped modulo S).
  * Duplicate (u, v, t) tuples get a fresh time until every tuple is unique
    (Sec. 1.1: each tuple appears once).
"""
from dataclasses import dataclass, field

import numpy as np

# Motifs as ordered edge lists: edge p is the p-th edge in time (the order pi
# of Def. "temporal motif").  The paper's own motif figures are not recoverable,
# so these are the shapes the workloads name.
MOTIFS = {
    # a->b, b->c, c->a
    "3cycle": ((0, 1), (1, 2), (2, 0)),
    # a->b, b->c, c->d, d->a
    "4cycle": ((0, 1), (1, 2), (2, 3), (3, 0)),
    # 4-leaf out-star a->b < a->c < a->d < a->e
    "4star": ((0, 1), (0, 2), (0, 3), (0, 4)),
    # fan-out then fan-in: a->b < a->c < a->d < b->e < c->e < d->e
    "scatter_gather": ((0, 1), (0, 2), (0, 3), (1, 4), (2, 4), (3, 4)),
    # a->b->c->d->e->f
    "6chain": ((0, 1), (1, 2), (2, 3), (3, 4), (4, 5)),
}


# Partial-order motifs (the paper's remark on a partial order of time
# constraints, Sec. 1.1 and Sec. 6): (edges, pairs (p, q) meaning edge p is
# strictly earlier than edge q); pairs not implied by these are unordered.
PO_MOTIFS = {
    # a->b, a->c, a->d in any order (an unordered 3-leaf fan-out)
    "po_fan3": (((0, 1), (0, 2), (0, 3)), ()),
    # two payments a->b, b->c in any order, then the return c->a
    "po_cycle3": (((0, 1), (1, 2), (2, 0)), ((0, 2), (1, 2))),
    # scatter-gather with each intermediate receiving before forwarding:
    # a->b < b->e, a->c < c->e, a->d < d->e, the three paths unordered
    "po_sg": (((0, 1), (0, 2), (0, 3), (1, 4), (2, 4), (3, 4)), ((0, 3), (1, 4), (2, 5))),
    # a->b < b->c, then c->a and a->c anywhere within delta (two unordered
    # non-tree edges that may lead, trail or sit between the tree edges)
    "po_free2": (((0, 1), (1, 2), (2, 0), (0, 2)), ((0, 1),)),
    # two paths a->b->d and a->c->d, each in order, unordered to each other
    "po_diamond": (((0, 1), (0, 2), (1, 3), (2, 3)), ((0, 2), (1, 3))),
    # two ordered a->b edges and b->c unordered to both
    "po_parallel": (((0, 1), (0, 1), (1, 2)), ((0, 1),)),
}


def motif_vertices(edges) -> int:
    return 1 + max(max(e) for e in edges)


@dataclass
class TemporalGraph:
    src: np.ndarray          # int32
    dst: np.ndarray          # int32
    t: np.ndarray            # int64
    n: int
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def _chung_lu_pairs(rng, n, m, gamma):
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    ids = rng.permutation(n).astype(np.int32)

    def draw(size):
        r = np.searchsorted(cdf, rng.random(size), side="right")
        return ids[np.minimum(r, n - 1)]

    u = draw(m)
    v = draw(m)
    bad = np.nonzero(u == v)[0]
    while bad.size:
        u[bad] = draw(bad.size)
        v[bad] = draw(bad.size)
        bad = bad[u[bad] == v[bad]]
    return u, v


def _bursty_times(rng, u, span, alpha=1.5):
    """Per-source renewal process: start s_u ~ U[0, span), gaps x_u * U^(-1/alpha)
    with x_u = span / (3 d_u) (mean gap 3 x_u), times wrapped modulo span."""
    m = u.shape[0]
    order = np.argsort(u, kind="stable")
    us = u[order]
    starts = np.flatnonzero(np.r_[True, us[1:] != us[:-1]])
    counts = np.diff(np.r_[starts, m])
    group = np.repeat(np.arange(starts.size), counts)
    x = span / (3.0 * counts.astype(np.float64))
    gaps = x[group] * rng.random(m) ** (-1.0 / alpha)
    c = np.cumsum(gaps)
    before = np.r_[0.0, c[starts[1:] - 1]]
    within = c - before[group]
    s0 = rng.random(starts.size) * span
    ts = np.floor(s0[group] + within) % span
    t = np.empty(m, np.int64)
    t[order] = ts.astype(np.int64)
    return t


def _dedup(rng, u, v, t, redraw):
    """Give a fresh time to every repeated (u, v, t) until all are unique."""
    while True:
        key_order = np.lexsort((t, v, u))
        us, vs, ts = u[key_order], v[key_order], t[key_order]
        dup = np.nonzero((us[1:] == us[:-1]) & (vs[1:] == vs[:-1]) & (ts[1:] == ts[:-1]))[0] + 1
        if dup.size == 0:
            return t
        idx = key_order[dup]
        t[idx] = redraw(idx.size)


def chung_lu_graph(n, m, gamma, seed, times="uniform", tmax=100_000, span=10_000_000,
                   reciprocal=0, recip_gap=600, name="") -> TemporalGraph:
    rng = np.random.default_rng(seed)
    base = m - reciprocal
    u, v = _chung_lu_pairs(rng, n, base, gamma)
    if times == "uniform":
        t = rng.integers(0, tmax + 1, size=base, dtype=np.int64)
        redraw = lambda k: rng.integers(0, tmax + 1, size=k, dtype=np.int64)  # noqa: E731
    elif times == "bursty":
        t = _bursty_times(rng, u, float(span))
        redraw = lambda k: rng.integers(0, span, size=k, dtype=np.int64)  # noqa: E731
    else:
        raise ValueError(times)
    t = _dedup(rng, u, v, t, redraw)
    if reciprocal:
        pick = rng.choice(base, size=reciprocal, replace=False)
        ru, rv = v[pick].copy(), u[pick].copy()
        rt = t[pick] + rng.integers(1, recip_gap + 1, size=reciprocal, dtype=np.int64)
        u = np.concatenate([u, ru])
        v = np.concatenate([v, rv])
        t = _dedup(rng, u, v, np.concatenate([t, rt]), redraw)
    meta = dict(n=n, m=m, gamma=gamma, seed=seed, times=times, tmax=tmax, span=span,
                reciprocal=reciprocal)
    return TemporalGraph(u.astype(np.int32), v.astype(np.int32), t.astype(np.int64), n, name, meta)


# ---------------------------------------------------------------------------
# The named workloads.
# ---------------------------------------------------------------------------
def tiny_graph() -> TemporalGraph:
    """1,000 vertices, 20,000 edges, Chung-Lu gamma=2.3, times U{0..100000}."""
    return chung_lu_graph(1000, 20_000, 2.3, seed=101, times="uniform", tmax=100_000, name="tiny")


TINY = dict(motifs=(("3cycle", 1000),), k=100_000, seed=1)


def medium_graph() -> TemporalGraph:
    """100,000 vertices, 2,000,000 edges, gamma=2.1, bursty times over 1e7 s."""
    return chung_lu_graph(100_000, 2_000_000, 2.1, seed=102, times="bursty", span=10_000_000,
                          name="medium")


MEDIUM = dict(motifs=(("4cycle", 3600), ("4star", 3600)), k=10_000_000, seed=1)


def large_graph() -> TemporalGraph:
    """2,000,000 vertices, 100,000,000 edges (90M Chung-Lu gamma=2.0 plus 10M
    reciprocated at +U{1..600} s), bursty times over 3e7 s."""
    return chung_lu_graph(2_000_000, 100_000_000, 2.0, seed=103, times="bursty",
                          span=30_000_000, reciprocal=10_000_000, name="large")


LARGE = dict(motifs=(("scatter_gather", 86400), ("6chain", 86400)), k=100_000_000, seed=1)


def small_graph(m, seed, n=None, gamma=2.1, times="bursty", span=None) -> TemporalGraph:
    """A graph of the medium shape scaled down to m edges (tests)."""
    n = n if n is not None else max(50, m // 20)
    span = span if span is not None else max(1000, 5 * m)
    return chung_lu_graph(n, m, gamma, seed=seed, times=times, span=span, tmax=span,
                          name=f"small{m}")


def batched_jobs(n_jobs=64, seed=1000, m_lo=1e4, m_hi=5e6):
    """The batched workload: graph sizes log-uniform in [1e4, 5e6] edges (medium
    shape, span 1e7 s), motifs uniform over MOTIFS, delta log-uniform in
    [600, 86400], sample budgets log-uniform in [1e5, 1e7]."""
    rng = np.random.default_rng(seed)
    names = list(MOTIFS)
    jobs = []
    for j in range(n_jobs):
        m = int(round(10 ** rng.uniform(np.log10(m_lo), np.log10(m_hi))))
        jobs.append(dict(
            graph_seed=seed + j,
            m=m,
            n=max(50, m // 20),
            motif=names[int(rng.integers(len(names)))],
            delta=int(round(10 ** rng.uniform(np.log10(600), np.log10(86400)))),
            k=int(round(10 ** rng.uniform(5, 7))),
            seed=int(rng.integers(1, 2**63 - 1)),
        ))
    return jobs


def batched_graph(job) -> TemporalGraph:
    return chung_lu_graph(job["n"], job["m"], 2.1, seed=job["graph_seed"], times="bursty",
                          span=10_000_000, name=f"job{job['graph_seed']}")


# ---------------------------------------------------------------------------
# Serving: graphs too large to draw on the host in reasonable time are drawn
# on the device with torch's seeded generator (same recipe, different random
# stream from the numpy generator above).
# ---------------------------------------------------------------------------
SERVE_DELTAS = (600, 1800, 3600, 7200, 14400, 28800, 43200, 86400)
# the large graph's weight sets take 7-40 GB each: an hour and a day keep its
# ten (motif, delta) sets resident together
SERVE_DELTAS_LARGE = (3600, 86400)


def device_graph(n, m, gamma, seed, span=10_000_000, device="cuda", reciprocal=0, recip_gap=600):
    """Chung-Lu pairs with bursty per-source times, drawn on the device; the
    last `reciprocal` edges reverse distinct earlier ones at +U{1..recip_gap} s.
    Returns (src int32, dst int32, t int64) device tensors with every
    (u, v, t) unique."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    base = m - reciprocal
    u, v, t = _device_base(n, base, gamma, gen, span, device)
    if reciprocal:
        pick = torch.randperm(base, generator=gen, device=device)[:reciprocal]
        gap = torch.randint(1, recip_gap + 1, (reciprocal,), generator=gen, device=device)
        u, v, t = torch.cat([u, v[pick]]), torch.cat([v, u[pick]]), torch.cat([t, t[pick] + gap])
        del pick, gap
        _device_dedup(u, v, t, n, span, gen, device)
    return u, v, t


def _device_base(n, m, gamma, gen, span, device):
    import torch
    f64 = torch.float64
    # the vertex-weight distribution on the host: a device prefix sum of
    # floats need not round the same way every run
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    cdf_h = np.cumsum(w)
    cdf_h /= cdf_h[-1]
    cdf = torch.from_numpy(cdf_h).to(device)
    del w, cdf_h
    ids = torch.randperm(n, generator=gen, device=device).to(torch.int32)

    def draw(size):
        r = torch.searchsorted(cdf, torch.rand(size, generator=gen, device=device, dtype=f64), right=True)
        return ids[r.clamp_(max=n - 1)]

    u, v = draw(m), draw(m)
    while True:
        bad = torch.nonzero(u == v).flatten()
        if bad.numel() == 0:
            break
        u[bad], v[bad] = draw(bad.numel()), draw(bad.numel())
    del cdf, ids
    # bursty times: per-source renewal process, Pareto(1.5) gaps, mean span ~
    # span, wrapped modulo span.  Gaps are summed as exact fixed-point
    # integers (1/1024 s), each reduced modulo the span first, so the sums do
    # not depend on the order of a parallel scan.
    q = 1024
    order = torch.argsort(u, stable=True)
    us = u[order].long()
    counts = torch.bincount(us, minlength=n)
    first = torch.cumsum(counts, 0) - counts
    gaps = (span / (3.0 * counts[us].to(f64))) * torch.rand(m, generator=gen, device=device, dtype=f64) ** (-1.0 / 1.5)
    g = torch.floor(torch.fmod(gaps * q, float(span) * q)).to(torch.int64)
    del gaps
    c = torch.cumsum(g, 0)
    before = (c - g)[first.clamp(max=m - 1)]
    s0 = torch.floor(torch.rand(n, generator=gen, device=device, dtype=f64) * span * q).to(torch.int64)
    ts = torch.div(s0[us] + (c - before[us]), q, rounding_mode="floor") % span
    del g, c, before, counts, first, s0
    t = torch.empty(m, dtype=torch.int64, device=device)
    t[order] = ts
    del ts, us, order
    _device_dedup(u, v, t, n, span, gen, device)
    return u, v, t


def _device_dedup(u, v, t, n, span, gen, device):
    """Unique (u, v, t): redraw the time of every repeat, in place."""
    import torch
    while True:
        key = u.long() * n + v.long()
        idx = torch.argsort(t, stable=True)
        idx = idx[torch.argsort(key[idx], stable=True)]
        ks, tsr = key[idx], t[idx]
        dup = torch.nonzero((ks[1:] == ks[:-1]) & (tsr[1:] == tsr[:-1])).flatten() + 1
        del key, ks, tsr
        if dup.numel() == 0:
            break
        t[idx[dup]] = torch.randint(0, span, (dup.numel(),), generator=gen, device=device)
        del idx, dup


def large_graph_device():
    """The large workload drawn on the device (a host draw of 1e8 edges takes
    minutes): 2,000,000 vertices, 100,000,000 edges = 90M Chung-Lu gamma 2.0
    plus 10M reciprocated at +U{1..600} s, bursty times over 3e7 s."""
    return device_graph(2_000_000, 100_000_000, 2.0, 103, span=30_000_000, reciprocal=10_000_000)


def serving_graph_specs(scale=1.0):
    """The resident graphs: one of 2e7 vertices and 5e8 edges, eight of 5e4
    vertices and 1e6 edges (gamma 2.1, medium-style times over 1e7 s);
    scale shrinks the large one for quick runs."""
    big = dict(n=max(1000, int(2e7 * scale)), m=max(20_000, int(5e8 * scale)), seed=2000)
    small = [dict(n=50_000, m=1_000_000, seed=2001 + g) for g in range(8)]
    return [big] + small


def serving_queries(seconds=60.0, rate=200.0, n_graphs=9, seed=3000):
    """Poisson arrivals at `rate` per second for `seconds`: graph uniform over
    the resident ones (graph 0 is the large one), motif uniform over MOTIFS,
    delta uniform over SERVE_DELTAS_LARGE on graph 0 and over SERVE_DELTAS
    elsewhere, sample budget log-uniform in [1e5, 1e7]."""
    rng = np.random.default_rng(seed)
    names = list(MOTIFS)
    out, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            return out
        g = int(rng.integers(n_graphs))
        grid = SERVE_DELTAS_LARGE if g == 0 else SERVE_DELTAS
        out.append(dict(at=t, graph=g, motif=names[int(rng.integers(len(names)))],
                        delta=grid[int(rng.integers(len(grid)))],
                        k=int(round(10 ** rng.uniform(5, 7))), seed=int(rng.integers(1, 2**63 - 1))))


# ---------------------------------------------------------------------------
# Constraint ablation (Tab. "constraints" of the paper, on a synthetic graph
# small enough for exact counts): 5,000 vertices, 200,000 edges, gamma 2.1,
# bursty times over 3e6 s; delta 3600; 1e6 samples per (motif, mode).
# ---------------------------------------------------------------------------
def ablation_graph() -> TemporalGraph:
    return chung_lu_graph(5000, 200_000, 2.1, seed=104, times="bursty", span=3_000_000, name="ablation")


ABLATION = dict(motifs=("3cycle", "4cycle", "6chain"), delta=3600, k=1_000_000, seed=1)
