"""Pins for the oracle's sampler and estimator (Alg. 3, Alg. 6).

Lemma "sample-subtree-overall": a partial match phi is drawn with probability
N_phi / W.  Lemma "unbiased-estimate": E[C^] = C.  Both are checked against
brute-force enumeration of the partial matches (with their N_phi and M_phi).
"""
import math
import statistics
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_2507_20441_amd import workloads as W


def _setup(edges, delta, m, n, span, seed):
    g = W.small_graph(m, seed, n=n, span=span)
    G = O.Graph(g.src, g.dst, g.t, g.n)
    mo = O.make_motif(edges, delta)
    tr = O.default_tree(mo)
    P = O.Prep(G, mo, tr)
    eids, nphi, status, mb = G.brute_partial_matches(mo, tr)
    index = {tuple(e[: tr.n_edges]): a for a, e in enumerate(eids)}
    return G, mo, tr, P, index, nphi, status, mb


@pytest.mark.parametrize("name,delta,m,n,span", [("3cycle", 40, 90, 8, 300),
                                                  ("4cycle", 50, 80, 7, 250),
                                                  ("4star", 25, 60, 8, 250)])
def test_sampling_distribution_is_n_phi_over_w(name, delta, m, n, span):
    G, mo, tr, P, index, nphi, status, mb = _setup(W.MOTIFS[name], delta, m, n, span, 21)
    Wt = P.W
    assert Wt == int(nphi.sum()) and 20 <= len(nphi) <= 3000
    k = 60 * Wt
    res, recs = P.sample(seed=99, k=k, records=True)
    counts = np.zeros(len(nphi))
    for r in recs:
        a = index[tuple(r["eid"][: tr.n_edges])]   # every sample is a partial match
        counts[a] += 1
    # a partial match spread over 2*delta or more fits no interval (N_phi = 0)
    # and must never be drawn
    live = nphi > 0
    assert counts[~live].sum() == 0
    exp = k * nphi[live] / Wt
    chi2 = float(((counts[live] - exp) ** 2 / exp).sum())
    dof = int(live.sum()) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof), (chi2, dof)


def test_records_agree_with_brute_force():
    G, mo, tr, P, index, nphi, status, mb = _setup(W.MOTIFS["3cycle"], 40, 120, 8, 300, 5)
    res, recs = P.sample(seed=3, k=5000, records=True)
    _, _, tt = G.edges()
    for r in recs:
        a = index[tuple(r["eid"][: tr.n_edges])]
        assert r["status"] == status[a]
        times = tt[r["eid"][: tr.n_edges]]
        i = int(r["interval"])
        assert (times >= i * mo.delta).all() and (times < (i + 2) * mo.delta).all()
        if status[a] == 0:
            assert r["n_phi"] == nphi[a]
            assert int(r["m_lo"]) + (int(r["m_hi"]) << 64) == mb[a]
    assert res.n_valid + res.n_bad_vertex + res.n_bad_delta + res.n_bad_order == 5000
    acc2 = sum((2 // int(r["n_phi"])) * (int(r["m_lo"]) + (int(r["m_hi"]) << 64))
               for r in recs if r["status"] == 0)
    assert res.acc2.value == acc2
    assert res.estimate == float(P.W) * (float(acc2) / (2.0 * 5000))


def test_sample_ranges_compose_exactly():
    G, mo, tr, P, *_ = _setup(W.MOTIFS["4cycle"], 50, 120, 7, 250, 6)
    whole, rw = P.sample(seed=17, k=3000, records=True)
    a, ra = P.sample(seed=17, k=3000, j0=0, count=1234, records=True)
    b, rb = P.sample(seed=17, k=3000, j0=1234, count=3000 - 1234, records=True)
    assert whole.acc2.value == a.acc2.value + b.acc2.value
    assert whole.n_valid == a.n_valid + b.n_valid
    assert (np.concatenate([ra, rb]) == rw).all()


@pytest.mark.parametrize("name,delta,m,n,span", [("3cycle", 40, 110, 8, 300),
                                                  ("4cycle", 70, 120, 7, 250)])
def test_unbiased_over_1000_seeds(name, delta, m, n, span):
    """Mean of C^ over 1000 independent seeds within 3 sigma of C, with sigma
    computed exactly from the brute-force distribution of 2*M_phi/N_phi."""
    G, mo, tr, P, index, nphi, status, mb = _setup(W.MOTIFS[name], delta, m, n, span, 8)
    C = G.brute_count(mo)
    assert C > 0
    Wt = P.W
    y = np.array([2 * mb[a] / nphi[a] if status[a] == 0 else 0.0 for a in range(len(nphi))])
    p = nphi / Wt
    ey, ey2 = float((p * y).sum()), float((p * y * y).sum())
    assert abs(Wt * ey / 2 - C) < 1e-9 * C          # E[C^] = C exactly
    k, seeds = 200, 1000
    var_single = (Wt / 2) ** 2 * (ey2 - ey ** 2) / k
    runs = [P.sample(seed=s, k=k)[0] for s in range(1, seeds + 1)]
    ests = [r.estimate for r in runs]
    sigma = math.sqrt(var_single / seeds)
    assert abs(float(np.mean(ests)) - C) <= 3 * sigma, (np.mean(ests), C, sigma)
    # The squared standard error is an unbiased estimate of Var(C^) (Sec. 4.4):
    # its mean over the seeds lies within 4 sigma of the exact variance, sigma
    # from the exact fourth central moment of the same distribution.
    mu = ey
    m2 = float((p * (y - mu) ** 2).sum())
    m4 = float((p * (y - mu) ** 4).sum())
    var_s2 = (m4 - (k - 3) / (k - 1) * m2 * m2) / k      # variance of the sample variance
    scale = (Wt / 2) ** 2 / k
    se2 = [r.std_error ** 2 for r in runs]
    sd_mean = scale * math.sqrt(var_s2 / seeds)
    assert abs(float(np.mean(se2)) - scale * m2) <= 4 * sd_mean, (np.mean(se2), scale * m2, sd_mean)


def _terms(recs):
    return [(2 // int(r["n_phi"])) * (int(r["m_lo"]) + (int(r["m_hi"]) << 64)) if r["status"] == 0 else 0
            for r in recs]


@pytest.mark.parametrize("name,delta,k", [("3cycle", 40, 2), ("3cycle", 40, 3000), ("4cycle", 50, 777)])
def test_std_error_is_the_sample_standard_deviation(name, delta, k):
    """SE = (W/2) * stdev(Y) / sqrt(k), Y = 2 M_phi / N_phi per sample, with
    stdev the library's sample standard deviation (exact rational sums)."""
    g = W.small_graph(120, 6, n=7, span=250)
    G = O.Graph(g.src, g.dst, g.t, g.n)
    P = O.Prep(G, O.make_motif(W.MOTIFS[name], delta))
    res, recs = P.sample(seed=11, k=k, records=True)
    y = _terms(recs)
    want = (P.W / 2) * statistics.stdev([Fraction(v) for v in y]) / math.sqrt(k)
    want = float(want)
    assert res.std_error == pytest.approx(want, rel=1e-12, abs=0.0 if want else 1e-300)


def test_std_error_degenerate_cases():
    g = W.small_graph(120, 6, n=7, span=250)
    G = O.Graph(g.src, g.dst, g.t, g.n)
    P = O.Prep(G, O.make_motif(W.MOTIFS["3cycle"], 40))
    assert P.sample(seed=1, k=1)[0].std_error == 0.0            # one sample: no spread measurable
    Z = O.Prep(G, O.make_motif(W.MOTIFS["3cycle"], 1))          # no partial match at delta 1
    if Z.W == 0:
        r = Z.sample(seed=1, k=100)[0]
        assert r.std_error == 0.0 and r.estimate == 0.0


def _exact_se(Wt, S1, S2, k):
    """(W/2) sqrt((k S2 - S1^2) / (k^2 (k-1))) to 40 significant digits."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    D = k * S2 - S1 * S1
    v = Decimal(D) / Decimal(k * k * (k - 1))
    return Decimal(Wt) / 2 * v.sqrt()


def test_std_error_wide_sums_against_exact_arithmetic():
    """Sums whose D = k sum Y^2 - (sum Y)^2 needs up to 256 bits, against the
    exact value (rational D, 60-digit square root): within 4 ulp, the bound of
    the conversion of D plus the four rounded floating-point steps after it."""
    import random
    rng = random.Random(7)
    cases = [(2, 3, 5, 2), (12345, 10**20, 10**38, 1000)]
    for _ in range(300):
        k = rng.choice([2, 3, 1000, 10**7, 2**40 + 5, 2**63 + 1])
        # k terms with sum S1 and sum of squares S2 >= S1^2 / k
        S1 = rng.randrange(0, 2**rng.randrange(1, 127))
        lo = -(-S1 * S1 // k)
        S2 = lo + rng.randrange(0, 2**rng.randrange(1, 127))
        if S2 >= 2**128:
            continue
        cases.append((rng.randrange(1, 2**rng.randrange(1, 128)), S1, S2, k))
    wide = 0
    for Wt, S1, S2, k in cases:
        got = O.std_error(Wt, S1, S2, k)
        want = float(_exact_se(Wt, S1, S2, k))
        wide += (k * S2 - S1 * S1) >= 2**128
        assert got == pytest.approx(want, rel=4 * 2.0**-52, abs=0.0), (Wt, S1, S2, k)
    assert wide > 20
    assert O.std_error(10, 4, 16, 1) == 0.0             # k < 2
    assert O.std_error(10, 4, 2**128 - 1, 9, flags=2) == 0.0   # squares saturated
    assert O.std_error(0, 0, 0, 9) == 0.0
