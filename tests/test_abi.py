"""The C-ABI library loads on a host without a GPU and exports every entry
point that include/timest.h declares (no compute calls here)."""
import ctypes
import os
import re

from paper_2507_20441_amd import timest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(tm_[a-z0-9_]+)\s*\(", text))
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("tm_graph_create", "tm_weights_create", "tm_sample", "tm_estimate"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(timest.LIB_PATH)
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing


def test_error_strings_without_gpu():
    L = timest.lib()
    assert L.tm_strerror(timest.TM_EDUP).decode() == "duplicate (u, v, t) tuple"
    assert L.tm_strerror(timest.TM_OK).decode() == "ok"


def test_default_tree_on_host_matches_oracle_rule():
    """The plan is host code: the default tree needs no GPU."""
    import oracle as O
    from paper_2507_20441_amd import workloads as W
    for name, edges in W.MOTIFS.items():
        g = timest.default_tree(timest.make_motif(edges, 10))
        o = O.default_tree(O.make_motif(edges, 10))
        assert list(g.edge[: g.n_edges]) == list(o.edge[: o.n_edges]) and g.center == o.center


def test_result_finish_on_host_matches_oracle_std_error():
    """The estimate's standard error is host arithmetic on exact sums: the
    library's 256-bit form equals the oracle's, bit for bit, on random sums
    (including D = k sum Y^2 - (sum Y)^2 well above 2^128 and huge k)."""
    import random
    import oracle as O
    rng = random.Random(3)
    wide = 0
    for _ in range(2000):
        k = rng.choice([2, 3, 17, 1000, 10**7, 2**40 + 5, 2**53 + 1, 2**63 + 1, 2**64 - 1])
        S1 = rng.randrange(0, 2**rng.randrange(1, 128))
        S2 = -(-S1 * S1 // k) + rng.randrange(0, 2**rng.randrange(1, 128))
        if S2 >= 2**128:
            continue
        Wt = rng.randrange(1, 2**rng.randrange(1, 128))
        wide += (k * S2 - S1 * S1) >= 2**128
        r = timest.Result()
        r.W.lo, r.W.hi = Wt & (2**64 - 1), Wt >> 64
        r.acc2.lo, r.acc2.hi = S1 & (2**64 - 1), S1 >> 64
        r.acc2_sq.lo, r.acc2_sq.hi = S2 & (2**64 - 1), S2 >> 64
        r.k = k
        timest.result_finish(r)
        assert r.std_error == O.std_error(Wt, S1, S2, k), (Wt, S1, S2, k)
        assert r.estimate == float(Wt) * (float(S1) / (2.0 * float(k)))
    assert wide > 100
    # ties of the 256-bit rounding: D = 2 S2 with S1 = 0 and k = 2
    for S2 in (2**127 + 2**74, 2**127 + 3 * 2**74, 2**127 + 2**74 + 1, 2**126 + 2**73):
        r = timest.Result()
        r.W.lo, r.acc2_sq.lo, r.acc2_sq.hi, r.k = 2, S2 & (2**64 - 1), S2 >> 64, 2
        timest.result_finish(r)
        assert r.std_error == O.std_error(2, 0, S2, 2)
