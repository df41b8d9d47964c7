"""Python binding of the TIMEST GPU library (libtimest.so, include/timest.h).

Argument marshalling only: every step of the estimator runs in the library's
HIP kernels.  PyTorch supplies device memory (for inputs and per-sample
records) and the current HIP stream.  Loading fails loudly when the library
is missing; there is no CPU fallback.
"""
import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtimest.so")

TM_OK, TM_EINVAL, TM_ESELFLOOP, TM_EDUP, TM_EOVERFLOW, TM_ERANGE, TM_ENOMEM, TM_EDEVICE = \
    0, -1, -2, -3, -4, -5, -6, -7
TM_EADMIT, TM_EAGAIN, TM_ECANCELED = -8, -9, -10
TM_PTR_HOST, TM_PTR_DEVICE = 0, 1
TM_F_W_ZERO, TM_F_SQ_SATURATED, TM_F_WIDE = 1, 2, 4
TM_C_EXCLUDE, TM_C_WINDOWS, TM_C_ALL = 1, 2, 3
ARRAYS = dict(src=0, dst=1, t=2, out_off=3, in_off=4, out_eid=5, in_eid=6, outn_eid=7, inn_eid=8,
              out_t=9, in_t=10, out_nbr=11, in_nbr=12, out_pos=13, in_pos=14, outn_key=15, inn_key=16,
              outn_pos=17, inn_pos=18)
ARRAY_DTYPES = dict(t="int64", out_t="int64", in_t="int64", outn_key="uint64", inn_key="uint64")


class U128(C.Structure):
    _fields_ = [("lo", C.c_uint64), ("hi", C.c_uint64)]

    @property
    def value(self) -> int:
        return int(self.lo) | (int(self.hi) << 64)


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
                ("flags", C.c_uint32), ("status", C.c_int32)]


class Profile(C.Structure):
    _fields_ = [("ms", C.c_double * 6), ("launches", C.c_uint64 * 6)]


STAGES = ("graph", "weights", "sample", "reduce", "roots", "levels")


class ServerOpts(C.Structure):
    _fields_ = [("pass_samples", C.c_uint64), ("job_chunk", C.c_uint64), ("max_jobs", C.c_int32),
                ("fifo", C.c_int32)]


class QueryInfo(C.Structure):
    _fields_ = [("queued_ms", C.c_double), ("latency_ms", C.c_double), ("weights_hit", C.c_uint32),
                ("passes", C.c_uint32)]


class ServerStats(C.Structure):
    _fields_ = [(f, C.c_uint64) for f in (
        "submitted", "completed", "failed", "passes", "samples", "weight_builds", "weight_hits",
        "evictions", "admission_waits", "budget_bytes", "resident_bytes", "peak_bytes", "cached_sets")] + [
        ("build_ms", C.c_double), ("pass_ms", C.c_double), ("pass_retries", C.c_uint64)]

    def as_dict(self):
        return {f: (round(getattr(self, f), 3) if t is C.c_double else int(getattr(self, f)))
                for f, t in self._fields_}


REC_DTYPE = np.dtype([("interval", "<u4"), ("status", "<u4"), ("n_phi", "<u4"), ("pad", "<u4"),
                      ("eid", "<i4", (8,)), ("m_lo", "<u8"), ("m_hi", "<u8")])
U128_DTYPE = np.dtype([("lo", "<u8"), ("hi", "<u8")])


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)


class Allocator(C.Structure):
    """tm_allocator: alloc(ctx, bytes, stream) -> device pointer or NULL;
    free(ctx, ptr, bytes, stream)."""
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class TorchAllocator:
    """The library's device memory from PyTorch's caching allocator: each
    block is a torch.cuda.caching_allocator_alloc on the stream the library
    names, returned with caching_allocator_delete.  Counts what it served
    (live_bytes, allocs, frees).  Pass it to Graph(..., allocator=) or
    Server(..., allocator=); keep it alive as long as they live (they hold a
    reference)."""

    def __init__(self):
        import torch
        self._torch = torch
        self.live_bytes = 0
        self.peak_bytes = 0
        self.allocs = 0
        self.frees = 0
        self.fail_next = 0   # tests: this many next requests fail (return NULL)
        self.failed = 0
        self._sizes = {}

        def _alloc(ctx, nbytes, stream):
            if self.fail_next > 0:
                self.fail_next -= 1
                self.failed += 1
                return None
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
            except RuntimeError:
                return None
            self._sizes[p] = int(nbytes)
            self.allocs += 1
            self.live_bytes += int(nbytes)
            self.peak_bytes = max(self.peak_bytes, self.live_bytes)
            return p

        def _free(ctx, ptr, nbytes, stream):
            torch.cuda.caching_allocator_delete(int(ptr))
            self.frees += 1
            self.live_bytes -= self._sizes.pop(int(ptr), int(nbytes))

        self._fa = ALLOC_FN(_alloc)
        self._ff = FREE_FN(_free)
        self.struct = Allocator(self._fa, self._ff, None)


class BatchOpts(C.Structure):
    _fields_ = [("tile", C.c_int32), ("blocks", C.c_int32), ("root_lds", C.c_int32), ("pad", C.c_int32),
                ("group_limit", C.c_uint64)]


class TimestError(RuntimeError):
    def __init__(self, code, what, detail):
        super().__init__(f"{what}: {detail} (code {code})")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() or "
                               "python paper_2507_20441_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
        L.tm_strerror.restype = C.c_char_p
        L.tm_strerror.argtypes = [C.c_int]
        L.tm_last_error.restype = C.c_char_p
        L.tm_graph_create.argtypes = [vp, vp, vp, i64, i32, C.c_int, C.POINTER(Allocator), vp, C.POINTER(vp)]
        L.tm_graph_destroy.argtypes = [vp]
        L.tm_graph_destroy.restype = None
        L.tm_graph_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i32), C.POINTER(i64),
                                    C.POINTER(i64), C.POINTER(u64)]
        L.tm_graph_export.argtypes = [vp, C.c_int, vp, vp]
        L.tm_default_tree.argtypes = [C.POINTER(Motif), C.POINTER(Tree)]
        L.tm_weights_create.argtypes = [vp, C.POINTER(Motif), C.POINTER(Tree), vp, C.POINTER(vp)]
        L.tm_weights_create_ex.argtypes = [vp, C.POINTER(Motif), C.POINTER(Tree), C.c_uint32, vp,
                                           C.POINTER(vp)]
        L.tm_estimate_ex.argtypes = [vp, C.POINTER(Motif), C.POINTER(Tree), C.c_uint32, u64, u64, vp,
                                     C.POINTER(Result), vp]
        L.tm_weights_destroy.argtypes = [vp]
        L.tm_weights_destroy.restype = None
        L.tm_weights_info.argtypes = [vp, C.POINTER(U128), C.POINTER(i64), C.POINTER(i32),
                                      C.POINTER(u64), C.POINTER(Tree)]
        L.tm_weights_export.argtypes = [vp, i32, i32, vp, vp]
        L.tm_weights_intervals.argtypes = [vp, vp, vp]
        L.tm_sample.argtypes = [vp, u64, u64, u64, u64, vp, C.POINTER(Result), vp]
        L.tm_result_finish.argtypes = [C.POINTER(Result)]
        L.tm_sample_noalloc.argtypes = [vp, u64, u64, u64, u64, vp, C.POINTER(Result), vp]
        L.tm_estimate.argtypes = [vp, C.POINTER(Motif), C.POINTER(Tree), u64, u64, vp,
                                  C.POINTER(Result), vp]
        L.tm_sample_batch.argtypes = [C.POINTER(vp), C.POINTER(u64), C.POINTER(u64), C.c_int, vp,
                                      C.POINTER(Result)]
        L.tm_estimate_batch.argtypes = [C.POINTER(vp), C.POINTER(Motif), C.POINTER(C.POINTER(Tree)),
                                        C.POINTER(u64), C.POINTER(u64), C.c_int, vp,
                                        C.POINTER(Result)]
        L.tm_batch_config.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.tm_batch_options.argtypes = [C.POINTER(BatchOpts), C.POINTER(BatchOpts)]
        L.tm_list_instances.argtypes = [vp, u64, u64, u64, vp, vp, vp]
        L.tm_sample_family.argtypes = [vp, C.POINTER(Motif), C.c_int, u64, u64, vp, C.POINTER(Result)]
        L.tm_tree_candidates.argtypes = [C.POINTER(Motif), C.POINTER(Tree), C.POINTER(i64), C.c_int,
                                         C.POINTER(C.c_int)]
        L.tm_choose_tree.argtypes = [vp, C.POINTER(Motif), C.c_int, vp, C.POINTER(Tree), C.POINTER(U128),
                                     C.POINTER(C.c_int)]
        L.tm_batch_plan_create.argtypes = [C.POINTER(vp), C.POINTER(Motif), C.POINTER(C.POINTER(Tree)),
                                           C.POINTER(u64), C.POINTER(u64), C.c_int, vp, C.POINTER(vp)]
        L.tm_batch_plan_run.argtypes = [vp, vp, C.POINTER(Result)]
        L.tm_batch_plan_destroy.argtypes = [vp]
        L.tm_batch_plan_destroy.restype = None
        L.tm_release_cached.argtypes = []
        L.tm_profile_enable.argtypes = [C.c_int]
        L.tm_profile_enable.restype = None
        L.tm_profile_stages.argtypes = [C.c_uint32]
        L.tm_profile_stages.restype = None
        L.tm_profile_read.argtypes = [C.POINTER(Profile), C.c_int]
        L.tm_sample_model_bytes.argtypes = [vp, u64, u64, u64, vp, C.POINTER(u64)]
        L.tm_weights_model_bytes.argtypes = [vp, C.POINTER(Motif), C.POINTER(Tree), vp, C.POINTER(u64)]
        L.tm_weights_footprint.argtypes = [vp, C.POINTER(Motif), C.POINTER(Tree), i32, C.POINTER(u64)]
        L.tm_server_create.argtypes = [u64, C.POINTER(ServerOpts), C.POINTER(Allocator), C.POINTER(vp)]
        L.tm_server_add_graph.argtypes = [vp, vp, C.POINTER(i32)]
        L.tm_server_submit.argtypes = [vp, i32, C.POINTER(Motif), C.POINTER(Tree), u64, u64,
                                       C.POINTER(u64)]
        L.tm_server_poll.argtypes = [vp, u64, C.POINTER(Result), C.POINTER(QueryInfo)]
        L.tm_server_wait.argtypes = [vp, u64, C.POINTER(Result), C.POINTER(QueryInfo)]
        L.tm_server_read_stats.argtypes = [vp, C.POINTER(ServerStats)]
        L.tm_server_destroy.argtypes = [vp]
        L.tm_server_destroy.restype = None
        _lib = L
    return _lib


def _release(destroy, h):
    destroy(h)


def _own(obj, destroy, h):
    """Tie handle h to obj: released by obj.close(), when obj is collected, or
    at interpreter exit (before module teardown, latest handle first) -- the
    finalizer holds the destroy function itself, so it needs no module
    globals then."""
    obj.h = h
    obj._fin = weakref.finalize(obj, _release, destroy, h)


def _disown(obj):
    fin = getattr(obj, "_fin", None)
    if fin is not None:
        fin()
    obj.h = None


def _check(rc, what):
    if rc != TM_OK:
        raise TimestError(rc, what, lib().tm_last_error().decode())


def _stream():
    import torch
    if torch.cuda.is_available():
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(0)


def make_motif(edges, delta, k=None, before=None) -> Motif:
    """edges: (src, dst) pairs in pi order; before: None for their total
    order, else pairs (p, q), p < q, of a partial order (edge p strictly
    earlier than edge q)."""
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
    _check(lib().tm_default_tree(C.byref(mo), C.byref(tr)), "default_tree")
    return tr


def u128_ints(a):
    return [int(x["lo"]) | (int(x["hi"]) << 64) for x in a]


class Graph:
    """A temporal graph resident in device memory.

    src, dst, t: numpy arrays (copied from host memory) or torch tensors on
    the GPU (read in place on the current stream).  allocator: None (the
    library's block cache) or a TorchAllocator for the graph and everything
    built on it."""

    def __init__(self, src, dst, t, n, allocator=None):
        import torch
        self.n = int(n)
        self.allocator = allocator
        ap = C.byref(allocator.struct) if allocator is not None else None
        h = C.c_void_p()
        if isinstance(src, torch.Tensor) and src.is_cuda:
            s = src.to(torch.int32).contiguous()
            d = dst.to(torch.int32).contiguous()
            tt = t.to(torch.int64).contiguous()
            self.m = int(s.numel())
            rc = lib().tm_graph_create(C.c_void_p(s.data_ptr()), C.c_void_p(d.data_ptr()),
                                       C.c_void_p(tt.data_ptr()), self.m, self.n, TM_PTR_DEVICE, ap,
                                       _stream(), C.byref(h))
        else:
            s = np.ascontiguousarray(np.asarray(src), dtype=np.int32)
            d = np.ascontiguousarray(np.asarray(dst), dtype=np.int32)
            tt = np.ascontiguousarray(np.asarray(t), dtype=np.int64)
            self.m = int(s.shape[0])
            rc = lib().tm_graph_create(s.ctypes.data_as(C.c_void_p), d.ctypes.data_as(C.c_void_p),
                                       tt.ctypes.data_as(C.c_void_p), self.m, self.n, TM_PTR_HOST, ap,
                                       _stream(), C.byref(h))
        _check(rc, "graph_create")
        _own(self, lib().tm_graph_destroy, h)

    def close(self):
        _disown(self)

    def info(self):
        m, n, sh, sp, b = C.c_int64(), C.c_int32(), C.c_int64(), C.c_int64(), C.c_uint64()
        _check(lib().tm_graph_info(self.h, C.byref(m), C.byref(n), C.byref(sh), C.byref(sp),
                                   C.byref(b)), "graph_info")
        return dict(m=m.value, n=n.value, t_shift=sh.value, t_span=sp.value, bytes=b.value)

    def export(self, name):
        which = ARRAYS[name]
        size = self.n + 1 if name.endswith("_off") else self.m
        out = np.empty(size, np.dtype(ARRAY_DTYPES.get(name, "int32")))
        _check(lib().tm_graph_export(self.h, which, out.ctypes.data_as(C.c_void_p), _stream()),
               "graph_export")
        return out


class Weights:
    """Resident s-weight tables of one (graph, motif, tree) (Alg. 1, Alg. 2)."""

    def __init__(self, g: Graph, mo: Motif, tr: Tree = None, constraints=None):
        self.g, self.mo = g, mo
        h = C.c_void_p()
        c = TM_C_ALL if constraints is None else int(constraints)
        _check(lib().tm_weights_create_ex(g.h, C.byref(mo), C.byref(tr) if tr is not None else None, c,
                                          _stream(), C.byref(h)), "weights_create")
        _own(self, lib().tm_weights_destroy, h)

    def close(self):
        _disown(self)

    def info(self):
        W, q, wide, b, tr = U128(), C.c_int64(), C.c_int32(), C.c_uint64(), Tree()
        _check(lib().tm_weights_info(self.h, C.byref(W), C.byref(q), C.byref(wide), C.byref(b),
                                     C.byref(tr)), "weights_info")
        return dict(W=W.value, q=q.value, wide=bool(wide.value), bytes=b.value, tree=tr)

    @property
    def W(self) -> int:
        return self.info()["W"]

    def weights(self, s, slot):
        out = np.empty(self.g.m, U128_DTYPE)
        _check(lib().tm_weights_export(self.h, int(s), int(slot), out.ctypes.data_as(C.c_void_p),
                                       _stream()), "weights_export")
        return out

    def interval_weights(self):
        q = self.info()["q"]
        out = np.empty(q, U128_DTYPE)
        _check(lib().tm_weights_intervals(self.h, out.ctypes.data_as(C.c_void_p), _stream()),
               "weights_intervals")
        return u128_ints(out)

    def sample(self, seed, k, j0=0, count=None, k_total=None, records=False):
        import torch
        count = k if count is None else count
        k_total = k if k_total is None else k_total
        res = Result()
        recs_dev = None
        ptr = None
        if records and count > 0:
            recs_dev = torch.empty(count * REC_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
            ptr = C.c_void_p(recs_dev.data_ptr())
        _check(lib().tm_sample(self.h, int(seed), int(j0), int(count), int(k_total), _stream(),
                               C.byref(res), ptr), "sample")
        recs = None
        if records:
            recs = (recs_dev.cpu().numpy().view(REC_DTYPE) if recs_dev is not None
                    else np.zeros(0, REC_DTYPE))
        return res, recs


def sample_noalloc(w: "Weights", seed, count, j0=0, k_total=None, recs_ptr=None) -> "Result":
    """tm_sample_noalloc: samples j0 .. j0 + count - 1 with no allocation in
    the library; recs_ptr: None or a device pointer (int) to count records."""
    res = Result()
    k_total = count if k_total is None else k_total
    _check(lib().tm_sample_noalloc(w.h, int(seed), int(j0), int(count), int(k_total), _stream(), C.byref(res),
                                   C.c_void_p(recs_ptr) if recs_ptr else None), "sample_noalloc")
    return res


def estimate(g: Graph, mo: Motif, k, seed, tr: Tree = None, constraints=None, records=False):
    """tm_estimate_ex: a Result, or (Result, records) when records=True."""
    import torch
    res = Result()
    c = TM_C_ALL if constraints is None else int(constraints)
    recs_dev, ptr = None, None
    if records and k > 0:
        recs_dev = torch.empty(int(k) * REC_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        ptr = C.c_void_p(recs_dev.data_ptr())
    _check(lib().tm_estimate_ex(g.h, C.byref(mo), C.byref(tr) if tr is not None else None, c, int(k),
                                int(seed), _stream(), C.byref(res), ptr), "estimate")
    if not records:
        return res
    return res, (recs_dev.cpu().numpy().view(REC_DTYPE) if recs_dev is not None else np.zeros(0, REC_DTYPE))


def result_finish(res: "Result") -> "Result":
    """tm_result_finish: recompute estimate and std_error from the sums."""
    _check(lib().tm_result_finish(C.byref(res)), "result_finish")
    return res


def batch_config(tile, blocks=0):
    """Set the batched kernels' schedule; returns the previous (tile, blocks)."""
    pt, pb = C.c_int(), C.c_int()
    _check(lib().tm_batch_config(int(tile), int(blocks), C.byref(pt), C.byref(pb)), "batch_config")
    return pt.value, pb.value


def batch_options(tile=None, blocks=None, root_lds=None, group_limit=None) -> dict:
    """tm_batch_options: set the given fields (others unchanged); returns the
    previous schedule as a dict (pass it back as **kwargs to restore)."""
    prev = BatchOpts()
    _check(lib().tm_batch_options(None, C.byref(prev)), "batch_options")
    old = dict(tile=prev.tile, blocks=prev.blocks, root_lds=prev.root_lds, group_limit=prev.group_limit)
    new = dict(old)
    for k, v in (("tile", tile), ("blocks", blocks), ("root_lds", root_lds), ("group_limit", group_limit)):
        if v is not None:
            new[k] = int(v)
    o = BatchOpts(new["tile"], new["blocks"], new["root_lds"], 0, new["group_limit"])
    _check(lib().tm_batch_options(C.byref(o), None), "batch_options")
    return old


def sample_batch(weights, ks, seeds):
    """tm_sample_batch over resident weight sets; one Result per job."""
    n = len(weights)
    hs = (C.c_void_p * n)(*[w.h for w in weights])
    kk = (C.c_uint64 * n)(*[int(x) for x in ks])
    ss = (C.c_uint64 * n)(*[int(x) for x in seeds])
    out = (Result * n)()
    _check(lib().tm_sample_batch(hs, kk, ss, n, _stream(), out), "sample_batch")
    return list(out)


def estimate_batch(graphs, motifs, ks, seeds, trees=None):
    """tm_estimate_batch: whole estimates for (graph, motif, k, seed) jobs."""
    n = len(graphs)
    hs = (C.c_void_p * n)(*[g.h for g in graphs])
    mo = (Motif * n)(*motifs)
    kk = (C.c_uint64 * n)(*[int(x) for x in ks])
    ss = (C.c_uint64 * n)(*[int(x) for x in seeds])
    tr = None
    if trees is not None:
        keep = [C.pointer(t) if t is not None else None for t in trees]
        tr = (C.POINTER(Tree) * n)(*keep)
    out = (Result * n)()
    _check(lib().tm_estimate_batch(hs, mo, tr, kk, ss, n, _stream(), out), "estimate_batch")
    return list(out)


def weights_footprint(g: Graph, mo: Motif, tr: Tree = None, wide=False) -> int:
    b = C.c_uint64()
    _check(lib().tm_weights_footprint(g.h, C.byref(mo), C.byref(tr) if tr is not None else None,
                                      1 if wide else 0, C.byref(b)), "weights_footprint")
    return int(b.value)


class Server:
    """tm_server_*: resident graphs, a budgeted weight-set cache and
    continuous batching, driven by the library's worker thread."""

    def __init__(self, budget_bytes, pass_samples=0, job_chunk=0, max_jobs=0, fifo=False, allocator=None):
        o = ServerOpts(int(pass_samples), int(job_chunk), int(max_jobs), 1 if fifo else 0)
        h = C.c_void_p()
        self.allocator = allocator
        ap = C.byref(allocator.struct) if allocator is not None else None
        _check(lib().tm_server_create(int(budget_bytes), C.byref(o), ap, C.byref(h)), "server_create")
        _own(self, lib().tm_server_destroy, h)
        self._graphs = []

    def add_graph(self, g: Graph) -> int:
        gid = C.c_int32()
        _check(lib().tm_server_add_graph(self.h, g.h, C.byref(gid)), "server_add_graph")
        self._graphs.append(g)
        return gid.value

    def submit(self, gid, mo: Motif, k, seed, tr: Tree = None) -> int:
        t = C.c_uint64()
        _check(lib().tm_server_submit(self.h, int(gid), C.byref(mo),
                                      C.byref(tr) if tr is not None else None, int(k), int(seed),
                                      C.byref(t)), "server_submit")
        return t.value

    def poll(self, ticket):
        """(Result, QueryInfo) once finished, else None."""
        r, i = Result(), QueryInfo()
        rc = lib().tm_server_poll(self.h, int(ticket), C.byref(r), C.byref(i))
        if rc == TM_EAGAIN:
            return None
        _check(rc, "server_poll")
        return r, i

    def wait(self, ticket):
        r, i = Result(), QueryInfo()
        _check(lib().tm_server_wait(self.h, int(ticket), C.byref(r), C.byref(i)), "server_wait")
        return r, i

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().tm_server_read_stats(self.h, C.byref(st)), "server_stats")
        return st.as_dict()

    def close(self):
        _disown(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def release_cached():
    """Return the library's cached device blocks to HIP (tm_release_cached)."""
    _check(lib().tm_release_cached(), "release_cached")


def profile_enable(on=True):
    """Stage timing with HIP events (tm_profile_enable)."""
    lib().tm_profile_enable(1 if on else 0)


def profile_stages(stages=None):
    """Which stages are timed (tm_profile_stages): names from STAGES, or None for all."""
    mask = (1 << len(STAGES)) - 1 if stages is None else sum(1 << STAGES.index(s) for s in stages)
    lib().tm_profile_stages(mask)


def profile_read(reset=False) -> dict:
    """Accumulated stage milliseconds and launch counts (tm_profile_read)."""
    p = Profile()
    _check(lib().tm_profile_read(C.byref(p), 1 if reset else 0), "profile_read")
    return {"ms": list(p.ms), "launches": [int(x) for x in p.launches]}


def sample_model_bytes(w: "Weights", seed, count, j0=0) -> int:
    b = C.c_uint64()
    _check(lib().tm_sample_model_bytes(w.h, int(seed), int(j0), int(count), _stream(), C.byref(b)),
           "sample_model_bytes")
    return int(b.value)


def weights_model_bytes(g: "Graph", mo: "Motif", tr: "Tree" = None) -> int:
    """Access-model bytes of a weight build's level kernels (tm_weights_model_bytes)."""
    b = C.c_uint64()
    _check(lib().tm_weights_model_bytes(g.h, C.byref(mo), C.byref(tr) if tr is not None else None, _stream(),
                                        C.byref(b)), "weights_model_bytes")
    return int(b.value)


class BatchPlan:
    """tm_batch_plan_*: the 64-bit pipeline of a fixed job set recorded into
    one HIP graph; run() replays it and returns one Result per job."""

    def __init__(self, graphs, motifs, ks, seeds, trees=None):
        n = len(graphs)
        self._graphs = list(graphs)
        hs = (C.c_void_p * n)(*[g.h for g in graphs])
        mo = (Motif * n)(*motifs)
        kk = (C.c_uint64 * n)(*[int(x) for x in ks])
        ss = (C.c_uint64 * n)(*[int(x) for x in seeds])
        tr = None
        if trees is not None:
            keep = [C.pointer(t) if t is not None else None for t in trees]
            tr = (C.POINTER(Tree) * n)(*keep)
        h = C.c_void_p()
        _check(lib().tm_batch_plan_create(hs, mo, tr, kk, ss, n, _stream(), C.byref(h)), "batch_plan_create")
        _own(self, lib().tm_batch_plan_destroy, h)
        self.n = n

    def run(self):
        out = (Result * self.n)()
        _check(lib().tm_batch_plan_run(self.h, _stream(), out), "batch_plan_run")
        return list(out)

    def close(self):
        _disown(self)


def tree_candidates(mo: Motif):
    """[(Tree, looseness)] for every (spanning tree, center) pair, in the
    library's order (tm_tree_candidates)."""
    n = C.c_int()
    _check(lib().tm_tree_candidates(C.byref(mo), None, None, 0, C.byref(n)), "tree_candidates")
    trees = (Tree * n.value)()
    loose = (C.c_int64 * n.value)()
    _check(lib().tm_tree_candidates(C.byref(mo), trees, loose, n.value, C.byref(n)), "tree_candidates")
    return [(trees[x], int(loose[x])) for x in range(n.value)]


def choose_tree(g: Graph, mo: Motif, n_c):
    """(best Tree, [W of each evaluated candidate]) by tm_choose_tree."""
    best = Tree()
    Ws = (U128 * max(1, n_c))()
    ne = C.c_int()
    _check(lib().tm_choose_tree(g.h, C.byref(mo), int(n_c), _stream(), C.byref(best), Ws, C.byref(ne)),
           "choose_tree")
    return best, [Ws[x].value for x in range(ne.value)]


def sample_family(w: "Weights", motifs, seed, k):
    """tm_sample_family: one tree sample stream completed for every motif."""
    n = len(motifs)
    mo = (Motif * n)(*motifs)
    out = (Result * n)()
    _check(lib().tm_sample_family(w.h, mo, n, int(seed), int(k), _stream(), out), "sample_family")
    return list(out)


def list_instances(w: "Weights", seed, count, j0=0):
    """tm_list_instances: (eids [count x 16] int32, records) of samples
    j0 .. j0 + count - 1."""
    import torch
    eids = torch.empty(max(1, count) * 16, dtype=torch.int32, device="cuda")
    recs = torch.empty(max(1, count) * REC_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    _check(lib().tm_list_instances(w.h, int(seed), int(j0), int(count), _stream(), C.c_void_p(eids.data_ptr()),
                                   C.c_void_p(recs.data_ptr())), "list_instances")
    return (eids.cpu().numpy().reshape(-1, 16)[:count],
            recs.cpu().numpy().view(REC_DTYPE)[:count])
