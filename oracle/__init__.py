"""Python view of the TIMEST reference oracle -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over liboracle.so (oracle.cpp, brute.cpp).  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
this package; the GPU library never does.
"""
import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

OR_OK, OR_EINVAL, OR_ESELFLOOP, OR_EDUP, OR_EOVERFLOW, OR_ERANGE = 0, -1, -2, -3, -4, -5


C_EXCLUDE, C_WINDOWS, C_ALL = 1, 2, 3  # constraints 2 and 3 (constraint 1 always)


class U128(C.Structure):
    _fields_ = [("lo", C.c_uint64), ("hi", C.c_uint64)]

    @property
    def value(self) -> int:
        return int(self.lo) | (int(self.hi) << 64)

    @staticmethod
    def of(x: int) -> "U128":
        return U128(x & ((1 << 64) - 1), x >> 64)


class Motif(C.Structure):
    _fields_ = [("k", C.c_int32), ("l", C.c_int32), ("src", C.c_int32 * 16),
                ("dst", C.c_int32 * 16), ("delta", C.c_int64), ("partial", C.c_uint32),
                ("before", C.c_uint16 * 16)]


class Tree(C.Structure):
    _fields_ = [("n_edges", C.c_int32), ("edge", C.c_int32 * 8), ("center", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("estimate", C.c_double), ("std_error", C.c_double), ("W", U128), ("acc2", U128),
                ("acc2_sq", U128), ("k", C.c_uint64), ("n_valid", C.c_uint64),
                ("n_bad_vertex", C.c_uint64), ("n_bad_delta", C.c_uint64),
                ("n_bad_order", C.c_uint64), ("n_nonzero", C.c_uint64), ("q", C.c_int64),
                ("flags", C.c_uint32)]


# Per-sample record, the same 64-byte layout the GPU library uses.
REC_DTYPE = np.dtype([("interval", "<u4"), ("status", "<u4"), ("n_phi", "<u4"), ("pad", "<u4"),
                      ("eid", "<i4", (8,)), ("m_lo", "<u8"), ("m_hi", "<u8")])
U128_DTYPE = np.dtype([("lo", "<u8"), ("hi", "<u8")])

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
        L.or_graph_create.argtypes = [vp, vp, vp, i64, i32, C.POINTER(vp)]
        L.or_graph_destroy.argtypes = [vp]
        L.or_graph_edges.argtypes = [vp, vp, vp, vp]
        L.or_graph_shift.argtypes = [vp]
        L.or_graph_shift.restype = i64
        L.or_graph_list.argtypes = [vp, i32, C.c_int, vp, i64]
        L.or_graph_list.restype = i64
        L.or_default_tree.argtypes = [C.POINTER(Motif), C.POINTER(Tree)]
        L.or_prepare.argtypes = [vp, C.POINTER(Motif), C.POINTER(Tree), C.POINTER(vp)]
        L.or_prep_destroy.argtypes = [vp]
        L.or_prep_W.argtypes = [vp]
        L.or_prep_W.restype = U128
        L.or_prep_q.argtypes = [vp]
        L.or_prep_q.restype = i64
        L.or_prep_interval_weights.argtypes = [vp, vp]
        L.or_prep_weights.argtypes = [vp, i32, C.c_int, vp]
        L.or_sample.argtypes = [vp, u64, u64, u64, u64, C.POINTER(Result), vp]
        L.or_std_error.argtypes = [U128, U128, U128, u64, C.c_uint32]
        L.or_std_error.restype = C.c_double
        L.or_derive_cnt.argtypes = [vp, vp, C.POINTER(U128)]
        L.or_list_instance.argtypes = [vp, vp, U128, vp]
        L.or_tree_candidates.argtypes = [C.POINTER(Motif), C.POINTER(Tree), C.POINTER(C.c_int64), C.c_int,
                                         C.POINTER(C.c_int)]
        L.or_choose_tree.argtypes = [vp, C.POINTER(Motif), C.c_int, C.POINTER(Tree), C.POINTER(U128),
                                     C.POINTER(C.c_int)]
        L.or_prepare_ex.argtypes = [vp, C.POINTER(Motif), C.POINTER(Tree), C.c_uint32, C.POINTER(vp)]
        L.or_prepare_light_ex.argtypes = [vp, C.POINTER(Motif), C.POINTER(Tree), C.c_uint32, C.POINTER(vp)]
        L.or_brute_tree_weight_ex.argtypes = [vp, C.POINTER(Motif), C.POINTER(Tree), C.c_uint32, C.POINTER(U128)]
        L.or_brute_partial_matches_ex.argtypes = [vp, C.POINTER(Motif), C.POINTER(Tree), C.c_uint32, i64, vp,
                                                  vp, vp, vp]
        L.or_brute_partial_matches_ex.restype = i64
        L.or_prepare_light.argtypes = [vp, C.POINTER(Motif), C.POINTER(Tree), C.POINTER(vp)]
        L.or_edge_weight.argtypes = [vp, C.c_int64, C.c_int32, C.c_int32, C.c_uint64, C.POINTER(U128)]
        L.or_philox4x32_10.argtypes = [vp, vp, vp]
        L.or_draw.argtypes = [u64, u64, C.c_uint32, U128]
        L.or_draw.restype = U128
        L.or_brute_count.argtypes = [vp, C.POINTER(Motif), C.POINTER(U128)]
        L.or_brute_tree_weight.argtypes = [vp, C.POINTER(Motif), C.POINTER(Tree), C.POINTER(U128)]
        L.or_brute_edge_weight.argtypes = [vp, C.POINTER(Motif), C.POINTER(Tree), i64, i32, i32,
                                           C.POINTER(U128)]
        L.or_brute_partial_matches.argtypes = [vp, C.POINTER(Motif), C.POINTER(Tree), i64, vp, vp,
                                               vp, vp]
        L.or_brute_partial_matches.restype = i64
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_motif(edges, delta, k=None, before=None) -> Motif:
    """edges: list of (src, dst) in pi order.  before: None for the total
    order of the list, else a partial order as pairs (p, q), edge p strictly
    earlier than edge q (p < q)."""
    mo = Motif()
    mo.l = len(edges)
    mo.k = k if k is not None else 1 + max(max(e) for e in edges)
    for p, (a, b) in enumerate(edges):
        mo.src[p], mo.dst[p] = a, b
    mo.delta = int(delta)
    if before is not None:
        mo.partial = 1
        for p, q in before:
            mo.before[q] |= 1 << p
    return mo


def make_tree(edges, center) -> Tree:
    tr = Tree()
    tr.n_edges = len(edges)
    for j, p in enumerate(edges):
        tr.edge[j] = p
    tr.center = center
    return tr


def default_tree(mo: Motif) -> Tree:
    tr = Tree()
    rc = lib().or_default_tree(C.byref(mo), C.byref(tr))
    if rc != OR_OK:
        raise OracleError(rc, "default_tree")
    return tr


def u128_array_to_int(a) -> list:
    return [int(x["lo"]) | (int(x["hi"]) << 64) for x in a]


class Graph:
    def __init__(self, src, dst, t, n):
        self.src = np.ascontiguousarray(src, dtype=np.int32)
        self.dst = np.ascontiguousarray(dst, dtype=np.int32)
        self.t = np.ascontiguousarray(t, dtype=np.int64)
        self.m = len(self.src)
        self.n = int(n)
        h = C.c_void_p()
        rc = lib().or_graph_create(_ptr(self.src), _ptr(self.dst), _ptr(self.t), self.m, self.n,
                                   C.byref(h))
        if rc != OR_OK:
            raise OracleError(rc, "graph_create")
        self.h = h
        # released with the object, or at exit before module teardown (the
        # finalizer holds the destroy function itself)
        weakref.finalize(self, lib().or_graph_destroy, h)

    def edges(self):
        s = np.empty(self.m, np.int32)
        d = np.empty(self.m, np.int32)
        t = np.empty(self.m, np.int64)
        lib().or_graph_edges(self.h, _ptr(s), _ptr(d), _ptr(t))
        return s, d, t

    @property
    def shift(self) -> int:
        return int(lib().or_graph_shift(self.h))

    def vertex_list(self, v, direction):
        cnt = lib().or_graph_list(self.h, int(v), int(direction), None, 0)
        out = np.empty(max(cnt, 0), np.int32)
        lib().or_graph_list(self.h, int(v), int(direction), _ptr(out), cnt)
        return out

    def brute_count(self, mo: Motif) -> int:
        c = U128()
        rc = lib().or_brute_count(self.h, C.byref(mo), C.byref(c))
        if rc != OR_OK:
            raise OracleError(rc, "brute_count")
        return c.value

    def brute_tree_weight(self, mo: Motif, tr: Tree, constraints=C_ALL) -> int:
        c = U128()
        rc = lib().or_brute_tree_weight_ex(self.h, C.byref(mo), C.byref(tr), int(constraints), C.byref(c))
        if rc != OR_OK:
            raise OracleError(rc, "brute_tree_weight")
        return c.value

    def brute_edge_weight(self, mo, tr, interval, s, eid) -> int:
        c = U128()
        rc = lib().or_brute_edge_weight(self.h, C.byref(mo), C.byref(tr), int(interval), int(s),
                                        int(eid), C.byref(c))
        if rc != OR_OK:
            raise OracleError(rc, "brute_edge_weight")
        return c.value

    def brute_partial_matches(self, mo, tr, constraints=C_ALL):
        cnt = lib().or_brute_partial_matches_ex(self.h, C.byref(mo), C.byref(tr), int(constraints), 0, None,
                                                None, None, None)
        if cnt < 0:
            raise OracleError(cnt, "brute_partial_matches")
        eids = np.empty((cnt, 8), np.int32)
        nphi = np.empty(cnt, np.uint32)
        status = np.empty(cnt, np.uint32)
        mphi = np.empty(cnt, U128_DTYPE)
        lib().or_brute_partial_matches_ex(self.h, C.byref(mo), C.byref(tr), int(constraints), cnt, _ptr(eids),
                                          _ptr(nphi), _ptr(status), _ptr(mphi))
        return eids, nphi, status, u128_array_to_int(mphi)


class Prep:
    """Weights of one (graph, motif, tree) -- Alg. 1 / Alg. 2.  light=True
    builds no tables: only edge_weight and derive_cnt are then available."""

    def __init__(self, g: Graph, mo: Motif, tr: Tree = None, light=False, constraints=C_ALL):
        self.g, self.mo = g, mo
        self.tr = tr if tr is not None else default_tree(mo)
        h = C.c_void_p()
        fn = lib().or_prepare_light_ex if light else lib().or_prepare_ex
        rc = fn(g.h, C.byref(mo), C.byref(self.tr), int(constraints), C.byref(h))
        if rc != OR_OK:
            raise OracleError(rc, "prepare")
        self.h = h
        self._g = g  # the graph outlives its preparations
        weakref.finalize(self, lib().or_prep_destroy, h)

    def edge_weight(self, interval, s, eid, work_limit=1 << 62):
        """w_i(s, e) of one edge by the recursive rule (no tables); None when
        the candidate lists exceed work_limit."""
        out = U128()
        rc = lib().or_edge_weight(self.h, int(interval), int(s), int(eid), int(work_limit), C.byref(out))
        if rc == OR_ERANGE:
            return None
        if rc != OR_OK:
            raise OracleError(rc, "edge_weight")
        return out.value


    @property
    def W(self) -> int:
        return lib().or_prep_W(self.h).value

    @property
    def q(self) -> int:
        return int(lib().or_prep_q(self.h))

    def interval_weights(self):
        out = np.empty(self.q, U128_DTYPE)
        lib().or_prep_interval_weights(self.h, _ptr(out))
        return u128_array_to_int(out)

    def weights(self, s, slot):
        out = np.empty(self.g.m, U128_DTYPE)
        rc = lib().or_prep_weights(self.h, int(s), int(slot), _ptr(out))
        if rc != OR_OK:
            raise OracleError(rc, "prep_weights")
        return out

    def sample(self, seed, k, j0=0, count=None, k_total=None, records=False):
        count = k if count is None else count
        k_total = k if k_total is None else k_total
        res = Result()
        recs = np.zeros(count, REC_DTYPE) if records else None
        rc = lib().or_sample(self.h, int(seed), int(j0), int(count), int(k_total), C.byref(res),
                             _ptr(recs))
        if rc != OR_OK:
            raise OracleError(rc, "sample")
        return res, recs

    def list_instance(self, eids, rank):
        """The rank-th completion of a valid tree image: l eids in pi order."""
        e = np.ascontiguousarray(eids, dtype=np.int32)
        out = np.empty(self.mo.l, np.int32)
        rc = lib().or_list_instance(self.h, _ptr(e), U128.of(int(rank)), _ptr(out))
        if rc != OR_OK:
            raise OracleError(rc, "list_instance")
        return out

    def derive_cnt(self, eids):
        e = np.ascontiguousarray(eids, dtype=np.int32)
        out = U128()
        rc = lib().or_derive_cnt(self.h, _ptr(e), C.byref(out))
        if rc == OR_EINVAL:
            return None
        if rc != OR_OK:
            raise OracleError(rc, "derive_cnt")
        return out.value


def std_error(W, acc2, acc2_sq, k, flags=0) -> float:
    return float(lib().or_std_error(U128.of(int(W)), U128.of(int(acc2)), U128.of(int(acc2_sq)), int(k),
                                    int(flags)))


def philox4x32_10(ctr, key):
    c = np.array(ctr, np.uint32)
    k = np.array(key, np.uint32)
    out = np.empty(4, np.uint32)
    lib().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return [int(x) for x in out]


def draw(seed, j, d, n) -> int:
    return lib().or_draw(int(seed), int(j), int(d), U128.of(int(n))).value


def tree_candidates(mo: Motif):
    """[(Tree, looseness)] for every (spanning tree, center) pair (Alg. 8 order)."""
    n = C.c_int()
    rc = lib().or_tree_candidates(C.byref(mo), None, None, 0, C.byref(n))
    if rc != OR_OK:
        raise OracleError(rc, "tree_candidates")
    trees = (Tree * n.value)()
    loose = (C.c_int64 * n.value)()
    lib().or_tree_candidates(C.byref(mo), trees, loose, n.value, C.byref(n))
    return [(trees[x], int(loose[x])) for x in range(n.value)]


def choose_tree(g: "Graph", mo: Motif, n_c):
    """(best Tree, [W per evaluated candidate]) by Alg. 7."""
    best = Tree()
    Ws = (U128 * max(1, n_c))()
    ne = C.c_int()
    rc = lib().or_choose_tree(g.h, C.byref(mo), int(n_c), C.byref(best), Ws, C.byref(ne))
    if rc != OR_OK:
        raise OracleError(rc, "choose_tree")
    return best, [Ws[x].value for x in range(ne.value)]
