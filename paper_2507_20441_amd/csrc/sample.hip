// Sampling, validation, completion and reduction (Alg. 3 - Alg. 6).
//
// One lane per sample.  Draw 0 picks (interval, center edge) by inverse CDF
// over the pairs in (interval, eid) order: a search of the interval prefix
// W_i, then of the center's prefix array inside the interval.  Each further
// tree edge, in pre-order, is drawn by inverse CDF over its candidate list:
// the window of the shared vertex's list minus the run of edges to the
// excluded vertex.  The excluded entries sit at known T-order positions
// (xref), so the number J of excluded entries before the answer is found by a
// search over the excluded run, and the answer by one more search of the
// window's prefix array at the target shifted by their weight.
#include <algorithm>
#include <cstring>

#include "tm_primitives.h"

namespace {

struct SampleArgs {
    DevGraph G;
    int64_t delta;
    int64_t q;
    int k;
    int nt;
    int esrc[kMaxSlots], edst[kMaxSlots];  // motif vertices of each slot's edge
    int parent[kMaxSlots], side[kMaxSlots], dir[kMaxSlots], beta[kMaxSlots], leaf[kMaxSlots];
    int new_vertex[kMaxSlots];
    int by_pi[kMaxSlots];
    const void* qt[kMaxSlots][2];
    const void* qn[kMaxSlots][2];
    const void* qc[2];
    const int32_t* ilo;
    const int32_t* ihi;
    const void* cumW;
    u64 W_lo, W_hi;
    int n_free;
    int free_src[TM_MAX_L], free_dst[TM_MAX_L];
    int n_runs;
    int run_first[TM_MAX_L], run_len[TM_MAX_L], run_prev[TM_MAX_L], run_next[TM_MAX_L];
    u64 seed, j0, count;
    tm_sample_rec* recs;
    struct Partial* parts;
    int* ovf;
};

struct Partial {
    u128 acc2, acc2_sq;
    u64 n_valid, n_vertex, n_delta, n_order, n_nonzero;
    u64 flags;  // bit 0: acc2 wrapped, bit 1: acc2_sq saturated
    u64 bytes;  // access-model bytes (counting pass only)
};

// Reads charged to one binary search over L entries: ceil(log2(L + 1)).
__device__ __forceinline__ u64 probes(int64_t L) { return L <= 0 ? 0 : (u64)(64 - __clzll((u64)L)); }

// --------------------------------------------------------------------------
// Completion counting (Alg. 5).  Chains over the multi-edge lists of
// consecutive non-tree motif edges: every list is a run of the source's
// out-list in (destination, time) order, restricted to [lo, hi]; a chain
// takes one edge per list with strictly increasing times.  Merge-sweep over
// the lists in time order; S[j] counts chains ending in list j so far.  On
// equal times the later list goes first, so it never extends an edge of the
// same time.
// --------------------------------------------------------------------------
struct Run {
    int32_t a[TM_MAX_L], b[TM_MAX_L];  // [a, b) in the out-list N order
    int n;
};

template <bool kCount>
__device__ __forceinline__ void run_bounds(const DevGraph& G, const int32_t* img_v, const int* fs,
                                           const int* fd, int first, int len, int64_t lo, int64_t hi,
                                           Run& R, u64& nb) {
    R.n = len;
    if (lo < 0) lo = 0;
    if (hi > G.T) hi = G.T;
    for (int j = 0; j < len; ++j) {
        const int32_t x = img_v[fs[first + j]], y = img_v[fd[first + j]];
        const int32_t a = G.off[0][x], b = G.off[0][x + 1];
        if (lo > hi) {
            R.a[j] = R.b[j] = a;
            continue;
        }
        const u64 base = (u64)y << G.bt;
        R.a[j] = lower_bound_pos<u64>(G.nkey[0], a, b, base | (u64)lo);
        R.b[j] = upper_bound_pos<u64>(G.nkey[0], R.a[j], b, base | (u64)hi);
        if constexpr (kCount) nb += 8 + (probes(b - a) + probes(b - R.a[j])) * 8;
    }
}

template <bool kCount>
__device__ __forceinline__ u128 chain_count(const DevGraph& G, const Run& R, bool* ovf, u64& nb) {
    if (R.n == 0) return 1;
    if (R.n == 1) return (u128)(R.b[0] - R.a[0]);
    if constexpr (kCount)
        for (int j = 0; j < R.n; ++j) nb += (u64)(R.b[j] - R.a[j]) * 8;
    const u64 tmask = (G.bt >= 64) ? ~0ull : ((1ull << G.bt) - 1);
    u128 S[TM_MAX_L];
    int32_t p[TM_MAX_L];
    for (int j = 0; j < R.n; ++j) {
        S[j] = 0;
        p[j] = R.a[j];
    }
    while (true) {
        int best = -1;
        u64 bt = 0;
        for (int j = R.n - 1; j >= 0; --j) {
            if (p[j] < R.b[j]) {
                const u64 tj = G.nkey[0][p[j]] & tmask;
                if (best < 0 || tj < bt) {
                    bt = tj;
                    best = j;
                }
            }
        }
        if (best < 0) break;
        const u128 c = best == 0 ? (u128)1 : S[best - 1];
        if (!add_ok(S[best], c, &S[best])) *ovf = true;
        ++p[best];
    }
    return S[R.n - 1];
}

template <typename W>
__device__ __forceinline__ W child_mass(const Window& w, bool leaf, const W* qt, const W* qn) {
    if (leaf) return (W)((w.p1 - w.p0) - (w.q1 - w.q0));
    return (qt[w.p1] - qt[w.p0]) - (qn[w.q1] - qn[w.q0]);
}

template <typename W, bool kCount>
__global__ void __launch_bounds__(kBlock) sample_kernel(SampleArgs a) {
    const DevGraph& G = a.G;
    const W Wtot = (W)(((u128)a.W_hi << 64) | a.W_lo);
    const W* cumW = static_cast<const W*>(a.cumW);
    Partial acc;
    acc.acc2 = 0;
    acc.acc2_sq = 0;
    acc.n_valid = acc.n_vertex = acc.n_delta = acc.n_order = acc.n_nonzero = 0;
    acc.flags = 0;
    acc.bytes = 0;
    u64 nb = 0;
    bool ovf = false;
    bool bad = false;
    const u64 stride = (u64)gridDim.x * kBlock;
    for (u64 r = (u64)blockIdx.x * kBlock + threadIdx.x; r < a.count; r += stride) {
        const u64 j = a.j0 + r;
        int32_t img_e[kMaxSlots];
        int64_t te[kMaxSlots];
        int32_t eu[kMaxSlots], ev[kMaxSlots];
        int32_t img_v[TM_MAX_K];
        // draw 0: interval, then center edge
        const W r0 = scale(draw_block(a.seed, j, 0), Wtot);
        const int32_t i = upper_bound_pos<W>(cumW, 0, (int32_t)a.q + 1, r0) - 1;
        if (i < 0 || i >= a.q) { bad = true; break; }
        const int par = i & 1;
        const W* qc = static_cast<const W*>(a.qc[par]);
        const int32_t lo = a.ilo[i], hi = a.ihi[i];
        const W target0 = r0 - cumW[i] + qc[lo];
        int32_t e0 = upper_bound_pos<W>(qc, lo + 1, hi + 1, target0) - 1;
        // an interval with positive W_i holds edges; positions stay inside it
        if (hi <= lo) { bad = true; break; }
        e0 = e0 < lo ? lo : (e0 >= hi ? hi - 1 : e0);
        if constexpr (kCount)
            nb += (probes(a.q + 1) + 2 + probes(hi - lo)) * sizeof(W) + 8 + 16;
        img_e[0] = e0;
        te[0] = G.t[e0];
        eu[0] = G.src[e0];
        ev[0] = G.dst[e0];
        img_v[a.esrc[0]] = eu[0];
        img_v[a.edst[0]] = ev[0];
        const int64_t ilo_t = (int64_t)i * a.delta, ihi_t = ((int64_t)i + 2) * a.delta - 1;
        // draws 1..: children in pre-order
        for (int s = 1; s < a.nt; ++s) {
            const int p = a.parent[s];
            const int32_t g = a.side[s] ? ev[p] : eu[p];
            const int32_t o = a.side[s] ? eu[p] : ev[p];
            int64_t wlo = a.beta[s] < 0 ? te[p] - a.delta : te[p];
            int64_t whi = a.beta[s] < 0 ? te[p] : te[p] + a.delta;
            wlo = wlo > ilo_t ? wlo : ilo_t;
            whi = whi < ihi_t ? whi : ihi_t;
            const int d = a.dir[s];
            const Window w = find_window(G, d, g, o, wlo, whi);
            const bool leaf = a.leaf[s] != 0;
            const W* qt = static_cast<const W*>(a.qt[s][par]);
            const W* qn = static_cast<const W*>(a.qn[s][par]);
            const W mass = child_mass<W>(w, leaf, qt, qn);
            // a child of a positive-weight match always has positive mass
            if (mass == 0 || w.p1 <= w.p0) { bad = true; break; }
            const W rr = scale(draw_block(a.seed, j, (uint32_t)s), mass);
            // J: excluded entries whose preceding candidate mass is <= rr
            int32_t lo_j = w.q0, hi_j = w.q1;
            const int32_t* xref = G.nxref[d];
            while (lo_j < hi_j) {
                const int32_t mid = lo_j + ((hi_j - lo_j) >> 1);
                const int32_t pos = xref[mid];
                W F;
                if (leaf) F = (W)((pos - w.p0) - (mid - w.q0));
                else F = (qt[pos] - qt[w.p0]) - (qn[mid] - qn[w.q0]);
                if (F <= rr) lo_j = mid + 1; else hi_j = mid;
            }
            const int32_t J = lo_j - w.q0;
            int32_t pos;
            if (leaf) {
                pos = w.p0 + (int32_t)rr + J;
            } else {
                const W tgt = qt[w.p0] + rr + (qn[w.q0 + J] - qn[w.q0]);
                pos = upper_bound_pos<W>(qt, w.p0 + 1, w.p1 + 1, tgt) - 1;
            }
            pos = pos < w.p0 ? w.p0 : (pos >= w.p1 ? w.p1 - 1 : pos);
            if constexpr (kCount) {
                const int32_t la = G.off[d][g], lb = G.off[d][g + 1];
                nb += 8 + (2 * probes(lb - la) + probes(lb - w.p0) + probes(lb - w.q0)) * 8;
                nb += probes(w.q1 - w.q0) * (4 + (leaf ? 0 : 2 * sizeof(W)));
                if (!leaf) nb += (5 + probes(w.p1 - w.p0)) * sizeof(W);
                nb += 16;
            }
            const int32_t e = G.leid[d][pos];
            const int32_t nb = G.lnbr[d][pos];
            img_e[s] = e;
            te[s] = G.lt[d][pos];
            eu[s] = d == 0 ? g : nb;
            ev[s] = d == 0 ? nb : g;
            img_v[a.new_vertex[s]] = nb;
        }
        if (bad) break;
        // Alg. 4: vertex map 1-1, then delta range, then edge order
        uint32_t status = 0;
        for (int x = 0; x < a.k && status == 0; ++x)
            for (int y = x + 1; y < a.k; ++y)
                if (img_v[x] == img_v[y]) { status = 1; break; }
        int64_t tmin = te[0], tmax = te[0];
        for (int s = 1; s < a.nt; ++s) {
            tmin = te[s] < tmin ? te[s] : tmin;
            tmax = te[s] > tmax ? te[s] : tmax;
        }
        if (status == 0 && tmax - tmin > a.delta) status = 2;
        if (status == 0)
            for (int x = 1; x < a.nt; ++x)
                if (!(te[a.by_pi[x - 1]] < te[a.by_pi[x]])) { status = 3; break; }
        uint32_t n_phi = 0;
        u128 m_phi = 0;
        if (status == 0) {
            // N_phi: intervals holding every tree edge
            const int64_t b = tmin / a.delta;
            for (int64_t ii = b - 1; ii <= b; ++ii)
                if (ii >= 0 && ii < a.q && ii * a.delta <= tmin && tmax < (ii + 2) * a.delta) ++n_phi;
            // Alg. 5: completions over the non-tree edges
            m_phi = 1;
            const int64_t tfirst = te[a.by_pi[0]], tlast = te[a.by_pi[a.nt - 1]];
            int lead = -1, trail = -1;
            Run R;
            for (int rr = 0; rr < a.n_runs && m_phi != 0; ++rr) {
                const int pv = a.run_prev[rr], nx = a.run_next[rr];
                if (pv < 0) { lead = rr; continue; }
                if (nx < 0) { trail = rr; continue; }
                run_bounds<kCount>(G, img_v, a.free_src, a.free_dst, a.run_first[rr], a.run_len[rr],
                           te[pv] + 1, te[nx] - 1, R, nb);
                const u128 c = chain_count<kCount>(G, R, &ovf, nb);
                if (!mul_ok(m_phi, c, &m_phi)) ovf = true;
            }
            if (m_phi != 0 && lead >= 0 && trail < 0) {
                run_bounds<kCount>(G, img_v, a.free_src, a.free_dst, a.run_first[lead], a.run_len[lead],
                           tlast - a.delta, tfirst - 1, R, nb);
                if (!mul_ok(m_phi, chain_count<kCount>(G, R, &ovf, nb), &m_phi)) ovf = true;
            } else if (m_phi != 0 && trail >= 0 && lead < 0) {
                run_bounds<kCount>(G, img_v, a.free_src, a.free_dst, a.run_first[trail], a.run_len[trail],
                           tlast + 1, tfirst + a.delta, R, nb);
                if (!mul_ok(m_phi, chain_count<kCount>(G, R, &ovf, nb), &m_phi)) ovf = true;
            } else if (m_phi != 0 && trail >= 0 && lead >= 0) {
                // the first edge f of the leading chain fixes the window end
                // t(f) + delta of the trailing chain
                Run F;
                run_bounds<kCount>(G, img_v, a.free_src, a.free_dst, a.run_first[lead], 1,
                           tlast - a.delta, tfirst - 1, F, nb);
                const u64 tmask = (G.bt >= 64) ? ~0ull : ((1ull << G.bt) - 1);
                u128 sum = 0;
                for (int32_t x = F.a[0]; x < F.b[0]; ++x) {
                    const int64_t tf = (int64_t)(G.nkey[0][x] & tmask);
                    u128 lc = 1;
                    if (a.run_len[lead] > 1) {
                        run_bounds<kCount>(G, img_v, a.free_src, a.free_dst, a.run_first[lead] + 1,
                                   a.run_len[lead] - 1, tf + 1, tfirst - 1, R, nb);
                        lc = chain_count<kCount>(G, R, &ovf, nb);
                    }
                    if (lc == 0) continue;
                    run_bounds<kCount>(G, img_v, a.free_src, a.free_dst, a.run_first[trail],
                               a.run_len[trail], tlast + 1, tf + a.delta, R, nb);
                    u128 prod;
                    if (!mul_ok(lc, chain_count<kCount>(G, R, &ovf, nb), &prod)) ovf = true;
                    if (!add_ok(sum, prod, &sum)) ovf = true;
                }
                if (!mul_ok(m_phi, sum, &m_phi)) ovf = true;
            }
            ++acc.n_valid;
            if (m_phi != 0) ++acc.n_nonzero;
            u128 term;
            if (!mul_ok(m_phi, (u128)(2 / n_phi), &term)) ovf = true;
            if (!add_ok(acc.acc2, term, &acc.acc2)) acc.flags |= 1;
            u128 sq;
            if (!mul_ok(term, term, &sq) || !add_ok(acc.acc2_sq, sq, &acc.acc2_sq)) {
                acc.acc2_sq = ~(u128)0;
                acc.flags |= 2;
            }
        } else if (status == 1) {
            ++acc.n_vertex;
        } else if (status == 2) {
            ++acc.n_delta;
        } else {
            ++acc.n_order;
        }
        if (a.recs) {
            tm_sample_rec& out = a.recs[r];
            out.interval = (uint32_t)i;
            out.status = status;
            out.n_phi = n_phi;
            out.pad = 0;
            for (int x = 0; x < 8; ++x) out.eid[x] = x < a.nt ? img_e[a.by_pi[x]] : -1;
            out.m_phi.lo = (u64)m_phi;
            out.m_phi.hi = (u64)(m_phi >> 64);
        }
    }
    acc.bytes = nb;
    // block reduction into one partial
    __shared__ Partial red[kBlock];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            Partial& x = red[threadIdx.x];
            const Partial& y = red[threadIdx.x + h];
            if (!add_ok(x.acc2, y.acc2, &x.acc2)) x.flags |= 1;
            if (!add_ok(x.acc2_sq, y.acc2_sq, &x.acc2_sq)) { x.acc2_sq = ~(u128)0; x.flags |= 2; }
            x.n_valid += y.n_valid;
            x.n_vertex += y.n_vertex;
            x.n_delta += y.n_delta;
            x.n_order += y.n_order;
            x.n_nonzero += y.n_nonzero;
            x.flags |= y.flags;
            x.bytes += y.bytes;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) a.parts[blockIdx.x] = red[0];
    if (ovf) atomicOr(a.ovf, 1);
    if (bad) atomicOr(a.ovf, 2);
}

// Sum of the block partials (integers: the order does not matter).
__global__ void __launch_bounds__(kBlock) reduce_kernel(const Partial* parts, int n, Partial* out) {
    Partial acc;
    acc.acc2 = 0;
    acc.acc2_sq = 0;
    acc.n_valid = acc.n_vertex = acc.n_delta = acc.n_order = acc.n_nonzero = 0;
    acc.flags = 0;
    acc.bytes = 0;
    for (int b = threadIdx.x; b < n; b += kBlock) {
        const Partial& y = parts[b];
        if (!add_ok(acc.acc2, y.acc2, &acc.acc2)) acc.flags |= 1;
        if (!add_ok(acc.acc2_sq, y.acc2_sq, &acc.acc2_sq)) { acc.acc2_sq = ~(u128)0; acc.flags |= 2; }
        acc.n_valid += y.n_valid;
        acc.n_vertex += y.n_vertex;
        acc.n_delta += y.n_delta;
        acc.n_order += y.n_order;
        acc.n_nonzero += y.n_nonzero;
        acc.flags |= y.flags;
        acc.bytes += y.bytes;
    }
    __shared__ Partial red[kBlock];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            Partial& x = red[threadIdx.x];
            const Partial& y = red[threadIdx.x + h];
            if (!add_ok(x.acc2, y.acc2, &x.acc2)) x.flags |= 1;
            if (!add_ok(x.acc2_sq, y.acc2_sq, &x.acc2_sq)) { x.acc2_sq = ~(u128)0; x.flags |= 2; }
            x.n_valid += y.n_valid;
            x.n_vertex += y.n_vertex;
            x.n_delta += y.n_delta;
            x.n_order += y.n_order;
            x.n_nonzero += y.n_nonzero;
            x.flags |= y.flags;
            x.bytes += y.bytes;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

__global__ void fill_undrawn_kernel(tm_sample_rec* recs, u64 count) {
    const u64 r = (u64)blockIdx.x * kBlock + threadIdx.x;
    if (r >= count) return;
    tm_sample_rec& out = recs[r];
    out.interval = 0;
    out.status = 4;
    out.n_phi = 0;
    out.pad = 0;
    for (int x = 0; x < 8; ++x) out.eid[x] = -1;
    out.m_phi.lo = out.m_phi.hi = 0;
}

}  // namespace

int sample_run(tm_weights* w, u64 seed, u64 j0, u64 count, u64 k_total, hipStream_t st,
               tm_result* out, tm_sample_rec* recs, u64* model_bytes) {
    if (model_bytes) {
        *model_bytes = 0;
        recs = nullptr;
    }
    const HostPlan& P = w->plan;
    std::memset(out, 0, sizeof *out);
    out->k = k_total;
    out->q = w->q;
    out->W.lo = (u64)w->W;
    out->W.hi = (u64)(w->W >> 64);
    if (w->wide) out->flags |= TM_F_WIDE;
    if (w->W == 0 || count == 0) {
        if (w->W == 0) out->flags |= TM_F_W_ZERO;
        if (recs && count) {
            hipLaunchKernelGGL(fill_undrawn_kernel, dim3((unsigned)((count + kBlock - 1) / kBlock)),
                               dim3(kBlock), 0, st, recs, count);
            TM_HIP(hipGetLastError());
            TM_HIP(hipStreamSynchronize(st));
        }
        return TM_OK;
    }
    SampleArgs a;
    std::memset(&a, 0, sizeof a);
    a.G = w->g->d;
    a.delta = P.mo.delta;
    a.q = w->q;
    a.k = P.mo.k;
    a.nt = P.nt;
    for (int s = 0; s < P.nt; ++s) {
        const int e = P.edge[s];
        a.esrc[s] = P.mo.src[e];
        a.edst[s] = P.mo.dst[e];
        a.parent[s] = P.parent[s];
        a.side[s] = P.side[s];
        a.dir[s] = P.alpha[s] > 0 ? 0 : 1;
        a.beta[s] = P.beta[s];
        a.leaf[s] = P.n_children[s] == 0;
        a.new_vertex[s] = P.new_vertex[s];
        a.by_pi[s] = P.by_pi[s];
        for (int par = 0; par < 2; ++par) {
            a.qt[s][par] = w->qt[s][par];
            a.qn[s][par] = w->qn[s][par];
        }
    }
    a.qc[0] = w->qc[0];
    a.qc[1] = w->qc[1];
    a.ilo = w->ilo;
    a.ihi = w->ihi;
    a.cumW = w->cumW;
    a.W_lo = (u64)w->W;
    a.W_hi = (u64)(w->W >> 64);
    a.n_free = P.n_free;
    for (int f = 0; f < P.n_free; ++f) {
        a.free_src[f] = P.free_src[f];
        a.free_dst[f] = P.free_dst[f];
    }
    a.n_runs = P.n_runs;
    for (int r = 0; r < P.n_runs; ++r) {
        a.run_first[r] = P.run_first[r];
        a.run_len[r] = P.run_len[r];
        a.run_prev[r] = P.run_prev[r];
        a.run_next[r] = P.run_next[r];
    }
    a.seed = seed;
    a.j0 = j0;
    a.count = count;
    a.recs = recs;
    const u64 want = (count + kBlock - 1) / kBlock;
    const int blocks = (int)std::min<u64>(want, 4096);
    Partial* parts = nullptr;
    int* ovf = nullptr;
    TM_HIP(hipMallocAsync((void**)&parts, (size_t)(blocks + 1) * sizeof(Partial), st));
    TM_HIP(hipMallocAsync((void**)&ovf, sizeof(int), st));
    TM_HIP(hipMemsetAsync(ovf, 0, sizeof(int), st));
    a.parts = parts;
    a.ovf = ovf;
    StageTimer t_sample, t_reduce;
    if (!model_bytes) t_sample.start(TM_STAGE_SAMPLE, st);
    if (model_bytes) {
        if (w->wide)
            hipLaunchKernelGGL((sample_kernel<u128, true>), dim3(blocks), dim3(kBlock), 0, st, a);
        else
            hipLaunchKernelGGL((sample_kernel<u64, true>), dim3(blocks), dim3(kBlock), 0, st, a);
    } else if (w->wide) {
        hipLaunchKernelGGL((sample_kernel<u128, false>), dim3(blocks), dim3(kBlock), 0, st, a);
    } else {
        hipLaunchKernelGGL((sample_kernel<u64, false>), dim3(blocks), dim3(kBlock), 0, st, a);
    }
    TM_HIP(hipGetLastError());
    t_sample.stop();
    if (!model_bytes) t_reduce.start(TM_STAGE_REDUCE, st);
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kBlock), 0, st, (const Partial*)parts, blocks,
                       parts + blocks);
    TM_HIP(hipGetLastError());
    t_reduce.stop();
    Partial h;
    int hovf = 0;
    TM_HIP(hipMemcpyAsync(&h, parts + blocks, sizeof h, hipMemcpyDeviceToHost, st));
    TM_HIP(hipMemcpyAsync(&hovf, ovf, sizeof hovf, hipMemcpyDeviceToHost, st));
    TM_HIP(hipFreeAsync(parts, st));
    TM_HIP(hipFreeAsync(ovf, st));
    TM_HIP(hipStreamSynchronize(st));
    t_sample.finish();
    t_reduce.finish();
    if (model_bytes) *model_bytes = h.bytes;
    if (hovf & 2) return tm_fail(TM_EDEVICE, "sample: inconsistent weight tables");
    if (hovf || (h.flags & 1)) return tm_fail(TM_EOVERFLOW, "sample: a count reaches 2^128");
    out->acc2.lo = (u64)h.acc2;
    out->acc2.hi = (u64)(h.acc2 >> 64);
    out->acc2_sq.lo = (u64)h.acc2_sq;
    out->acc2_sq.hi = (u64)(h.acc2_sq >> 64);
    out->n_valid = h.n_valid;
    out->n_bad_vertex = h.n_vertex;
    out->n_bad_delta = h.n_delta;
    out->n_bad_order = h.n_order;
    out->n_nonzero = h.n_nonzero;
    if (h.flags & 2) out->flags |= TM_F_SQ_SATURATED;
    return TM_OK;
}
