// Preprocessing: the bottom-up spanning-tree weights (Alg. 1, Alg. 2).
//
// For a tree edge s of height h >= 1, an edge e matched to s and an interval
// I_i holding e, w_i(s, e) is the product over the children s' of s of the
// summed w_i(s', .) over the child's candidate list (Claim
// "overall-num-matches").  The candidate list is a time window of one
// vertex's out- or in-list minus the run of edges to the excluded vertex, so
// each factor is two differences of prefix sums: one along the window (T
// order), one along the excluded run (N order).  A leaf child contributes the
// plain counts.  Levels run bottom-up; after each non-center level the values
// are prefix-summed along the lists the parent searches.
//
// An edge lies in at most two intervals, i = floor(t/delta) and the one
// before, and those have different parities; so each table holds, per eid,
// one value per interval parity.  A window inside I_i only holds edges of
// blocks i and i+1, whose values for interval i are exactly the entries of
// parity i & 1 -- one prefix array per parity serves every interval.
#include <algorithm>
#include <cstring>

#include "tm_primitives.h"

namespace {

struct ChildDesc {
    int side;   // 0: attaches at the source endpoint of the parent's match, 1: destination
    int dir;    // 0: child is an out-edge of the shared vertex, 1: an in-edge
    int beta;   // -1: child precedes the parent in pi, +1: follows it
    int leaf;
    const void* qt[2];
    const void* qn[2];
};

struct LevelArgs {
    DevGraph G;
    int64_t delta;
    int nc;
    ChildDesc c[kMaxSlots];
    void* out[2];
    int* ovf;
};

template <typename W>
__global__ void __launch_bounds__(kBlock) level_kernel(LevelArgs a) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const DevGraph& G = a.G;
    if (e >= G.m) return;
    const int32_t u = G.src[e], v = G.dst[e];
    const int64_t t = G.t[e];
    const int64_t blk = t / a.delta;
    W val[2] = {0, 0};
    bool ovf = false;
    for (int slot = 0; slot < 2; ++slot) {
        const int64_t i = blk - slot;
        if (i < 0) continue;
        const int par = (int)(i & 1);
        const int64_t ilo = i * a.delta, ihi = (i + 2) * a.delta - 1;
        W prod = 1;
        for (int c = 0; c < a.nc; ++c) {
            const ChildDesc& d = a.c[c];
            const int32_t g = d.side ? v : u;
            const int32_t o = d.side ? u : v;
            int64_t wlo = d.beta < 0 ? t - a.delta : t;
            int64_t whi = d.beta < 0 ? t : t + a.delta;
            wlo = wlo > ilo ? wlo : ilo;
            whi = whi < ihi ? whi : ihi;
            const Window w = find_window(G, d.dir, g, o, wlo, whi);
            W f;
            if (d.leaf) {
                f = (W)((w.p1 - w.p0) - (w.q1 - w.q0));
            } else {
                const W* qt = static_cast<const W*>(d.qt[par]);
                const W* qn = static_cast<const W*>(d.qn[par]);
                f = (qt[w.p1] - qt[w.p0]) - (qn[w.q1] - qn[w.q0]);
            }
            if (!mul_ok(prod, f, &prod)) ovf = true;
        }
        val[par] = prod;
    }
    static_cast<W*>(a.out[0])[e] = val[0];
    static_cast<W*>(a.out[1])[e] = val[1];
    if (ovf) atomicOr(a.ovf, 4);
}

// Values of one parity gathered along a list order.
template <typename W>
struct ListGather {
    const W* val;
    const int32_t* eid;
    __device__ W operator()(int64_t p) const { return val[eid[p]]; }
};

template <typename W>
struct Plain {
    const W* val;
    __device__ W operator()(int64_t p) const { return val[p]; }
};

// Interval bounds: I_i = [i delta, (i+2) delta) holds eids [lo_i, hi_i).
__global__ void interval_kernel(const int64_t* t, int64_t m, int64_t q, int64_t delta, int32_t* lo,
                                int32_t* hi) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= q) return;
    lo[i] = lower_bound_pos<int64_t>(t, 0, (int32_t)m, i * delta);
    hi[i] = lower_bound_pos<int64_t>(t, lo[i], (int32_t)m, (i + 2) * delta);
}

// W_i = sum of w_i(c, e) over I_i: a difference of the center's prefix array.
template <typename W>
struct IntervalWeight {
    const W* qc0;
    const W* qc1;
    const int32_t* lo;
    const int32_t* hi;
    __device__ W operator()(int64_t i) const {
        const W* q = (i & 1) ? qc1 : qc0;
        return q[hi[i]] - q[lo[i]];
    }
};

unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <typename W>
int build_typed(tm_weights* w, hipStream_t st, int* ovf) {
    tm_graph* g = w->g;
    const HostPlan& P = w->plan;
    const int64_t m = g->m;
    const int64_t delta = P.mo.delta;
    // bottom-up over heights; leaves other than the center have weight 1 and
    // no table (a lone center edge gets a table of ones)
    for (int h = 0; h <= P.H; ++h) {
        for (int s = 0; s < P.nt; ++s) {
            if (P.height[s] != h || (h == 0 && s != 0)) continue;
            LevelArgs a;
            std::memset(&a, 0, sizeof a);
            a.G = g->d;
            a.delta = delta;
            a.nc = P.n_children[s];
            for (int j = 0; j < a.nc; ++j) {
                const int c = P.children[s][j];
                ChildDesc& d = a.c[j];
                d.side = P.side[c];
                d.dir = P.alpha[c] > 0 ? 0 : 1;
                d.beta = P.beta[c];
                d.leaf = P.n_children[c] == 0;
                for (int par = 0; par < 2; ++par) {
                    d.qt[par] = w->qt[c][par];
                    d.qn[par] = w->qn[c][par];
                }
            }
            for (int par = 0; par < 2; ++par) {
                W* p;
                TM_TRY(arena_alloc(w->arena, &p, (size_t)m));
                w->vals[s][par] = p;
                a.out[par] = p;
            }
            a.ovf = ovf;
            hipLaunchKernelGGL((level_kernel<W>), dim3(grid_for(m)), dim3(kBlock), 0, st, a);
            TM_HIP(hipGetLastError());
            // prefix sums along the lists the parent searches
            if (s != 0) {
                const int dir = P.alpha[s] > 0 ? 0 : 1;
                for (int par = 0; par < 2; ++par) {
                    W *qt, *qn;
                    TM_TRY(arena_alloc(w->arena, &qt, (size_t)m + 1));
                    TM_TRY(arena_alloc(w->arena, &qn, (size_t)m + 1));
                    const W* vp = static_cast<const W*>(w->vals[s][par]);
                    TM_TRY(device_exclusive_scan<W>(ListGather<W>{vp, g->d.leid[dir]}, m, qt, ovf, st));
                    TM_TRY(device_exclusive_scan<W>(ListGather<W>{vp, g->d.neid[dir]}, m, qn, ovf, st));
                    w->qt[s][par] = qt;
                    w->qn[s][par] = qn;
                }
            }
        }
    }
    // the center: prefix sums in eid order (slot 0 is the center)
    for (int par = 0; par < 2; ++par) {
        W* qc;
        TM_TRY(arena_alloc(w->arena, &qc, (size_t)m + 1));
        TM_TRY(device_exclusive_scan<W>(Plain<W>{static_cast<const W*>(w->vals[0][par])}, m, qc,
                                        ovf, st));
        w->qc[par] = qc;
    }
    // intervals and their weights
    TM_TRY(arena_alloc(w->arena, &w->ilo, (size_t)w->q));
    TM_TRY(arena_alloc(w->arena, &w->ihi, (size_t)w->q));
    hipLaunchKernelGGL(interval_kernel, dim3(grid_for(w->q)), dim3(kBlock), 0, st, g->d.t, m, w->q,
                       delta, w->ilo, w->ihi);
    TM_HIP(hipGetLastError());
    W* cum;
    TM_TRY(arena_alloc(w->arena, &cum, (size_t)w->q + 1));
    TM_TRY(device_exclusive_scan<W>(
        IntervalWeight<W>{static_cast<const W*>(w->qc[0]), static_cast<const W*>(w->qc[1]), w->ilo,
                          w->ihi},
        w->q, cum, ovf, st));
    w->cumW = cum;
    W hW;
    TM_HIP(hipMemcpyAsync(&hW, cum + w->q, sizeof(W), hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    w->W = to_u128(hW);
    return TM_OK;
}

void clear_tables(tm_weights* w) {
    w->arena.release();
    std::memset(w->vals, 0, sizeof w->vals);
    std::memset(w->qt, 0, sizeof w->qt);
    std::memset(w->qn, 0, sizeof w->qn);
    std::memset(w->qc, 0, sizeof w->qc);
    w->ilo = w->ihi = nullptr;
    w->cumW = nullptr;
}

}  // namespace

int weights_build(tm_weights* w, hipStream_t st) {
    tm_graph* g = w->g;
    const int64_t delta = w->plan.mo.delta;
    w->q = g->m > 0 ? g->T / delta + 1 : 0;
    if (g->m == 0) {
        w->W = 0;
        w->wide = false;
        return TM_OK;
    }
    if (w->q >= ((int64_t)1 << 31)) return tm_fail(TM_ERANGE, "weights: too many intervals");
    StageTimer timer;
    timer.start(TM_STAGE_WEIGHTS, st);
    int* ovf = nullptr;
    TM_HIP(hipMallocAsync((void**)&ovf, sizeof(int), st));
    int h = 0;
    int rc = TM_OK;
    for (int wide = 0; wide < 2; ++wide) {
        clear_tables(w);
        TM_HIP(hipMemsetAsync(ovf, 0, sizeof(int), st));
        w->wide = wide != 0;
        rc = wide ? build_typed<u128>(w, st, ovf) : build_typed<u64>(w, st, ovf);
        if (rc != TM_OK) break;
        TM_HIP(hipMemcpyAsync(&h, ovf, sizeof(int), hipMemcpyDeviceToHost, st));
        TM_HIP(hipStreamSynchronize(st));
        if (h == 0) break;
        if (wide) rc = tm_fail(TM_EOVERFLOW, "weights: a weight or W reaches 2^128");
    }
    TM_HIP(hipFreeAsync(ovf, st));
    timer.stop();
    TM_HIP(hipStreamSynchronize(st));
    timer.finish();
    if (rc != TM_OK) clear_tables(w);
    return rc;
}
