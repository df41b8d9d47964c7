// Host-side internals of the TIMEST GPU library: handles, the motif plan,
// error plumbing and the launchers each translation unit provides.
#pragma once

#include <initializer_list>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/timest.h"
#include "tm_common.h"

// ---------------------------------------------------------------------------
// Errors: every failing call records a message for its thread.
// ---------------------------------------------------------------------------
int tm_fail(int code, const char* fmt, ...);

#define TM_HIP(expr)                                                              \
    do {                                                                          \
        hipError_t _e = (expr);                                                   \
        if (_e != hipSuccess)                                                     \
            return tm_fail(_e == hipErrorOutOfMemory ? TM_ENOMEM : TM_EDEVICE,    \
                           "%s: %s (%s:%d)", #expr, hipGetErrorString(_e),        \
                           __FILE__, __LINE__);                                   \
    } while (0)

#define TM_TRY(expr)                    \
    do {                                \
        int _rc = (expr);               \
        if (_rc != TM_OK) return _rc;   \
    } while (0)

// Device allocations owned by a handle; released together.
// Tables owned by a handle, allocated from the library's block cache.
struct DevArena {
    std::vector<void*> blocks;
    uint64_t bytes = 0;
    hipStream_t stream = nullptr;
    int alloc(void** p, size_t nbytes);
    // return one block (work using it must be enqueued on `stream` before)
    void release_one(void* p, size_t nbytes);
    void release();
};

template <typename T>
int arena_alloc(DevArena& A, T** p, size_t count) {
    return A.alloc(reinterpret_cast<void**>(p), count * sizeof(T));
}

// Device block cache (mem.cpp): stream-aware reuse of released blocks.
// While an AllocScope with a caller's allocator is live on a thread,
// dev_alloc takes its blocks from that allocator instead (dev_free returns
// each block to where it came from, on any thread).
class AllocScope {
public:
    explicit AllocScope(const tm_allocator* a);
    ~AllocScope();
    AllocScope(const AllocScope&) = delete;
    AllocScope& operator=(const AllocScope&) = delete;

private:
    const tm_allocator* prev_;
};
hipError_t dev_alloc(void** p, size_t bytes, hipStream_t st);
hipError_t dev_free(void* p, hipStream_t st);
// Synchronise the device and return every cached block to HIP.
void dev_cache_trim();
// Between begin and end, dev_free on this thread appends to keep instead of
// releasing (for work recorded into a graph, which replays on those blocks).
void dev_defer_begin(std::vector<std::pair<void*, hipStream_t>>* keep);
void dev_defer_end();
// Every block released on st becomes reusable by any stream.
void dev_stream_synced(hipStream_t st);
// hipStreamSynchronize, then dev_stream_synced.
hipError_t sync_stream(hipStream_t st);
// Set n_words 32-bit words to v with a kernel (capturable, unlike a memset).
int fill_u32(void* p, int64_t n_words, uint32_t v, hipStream_t st);

// Pinned host blocks of kHostStageBytes for reading a few device words back.
// A copy into pageable memory waits for the device before it returns; copies
// into pinned memory do not, so the reads that end a call share one
// synchronisation.  Blocks come from a process-wide list (null when pinned
// memory cannot be had) and are never given back to HIP.
constexpr size_t kHostStageBytes = 16384;
void* host_stage_acquire();
void host_stage_release(void* p);

// One device-to-host copy of read_back.
struct HostRead {
    void* host;
    const void* dev;
    size_t bytes;
};
// The n copies, in stream order on st, then one synchronisation of st (as
// sync_stream); through one pinned block when they fit in it, else straight
// into the destinations.
hipError_t read_back(const HostRead* r, int n, hipStream_t st);
inline hipError_t read_back(std::initializer_list<HostRead> r, hipStream_t st) {
    return read_back(r.begin(), (int)r.size(), st);
}

// ---------------------------------------------------------------------------
// Graph handle.
// ---------------------------------------------------------------------------
struct tm_graph {
    DevGraph d{};
    int64_t m = 0;
    int32_t n = 0;
    int64_t shift = 0;
    int64_t T = 0;
    int device = 0;
    DevArena arena;
    // the caller's allocator of everything built on this graph (has_alloc)
    tm_allocator alloc{};
    bool has_alloc = false;
};

inline const tm_allocator* alloc_of(const tm_graph* g) { return g && g->has_alloc ? &g->alloc : nullptr; }

// ---------------------------------------------------------------------------
// Motif plan: the spanning tree rooted at its center edge (Sec. 4.1), listed
// in pre-order (center first, children in increasing pi index, each child's
// subtree before the next sibling).  Slots index that pre-order.
// ---------------------------------------------------------------------------
constexpr int kMaxSlots = 8;

struct HostPlan {
    tm_motif mo{};
    tm_tree tree{};
    int nt = 0;                    // tree edges (k - 1)
    int H = 0;                     // height of the center
    int slot_of_edge[TM_MAX_L];    // pre-order slot of a motif edge, -1 if not in the tree
    int edge[kMaxSlots];           // motif edge of a slot
    int parent[kMaxSlots];         // parent slot, -1 for the center
    int side[kMaxSlots];           // 0: attaches at the parent's source, 1: at its destination
    int alpha[kMaxSlots];          // +1: child leaves the shared vertex; -1: enters it
    int beta[kMaxSlots];           // -1: child precedes its parent; +1: follows; 0: unordered
    int height[kMaxSlots];
    int new_vertex[kMaxSlots];     // motif vertex first reached through this slot
    int children[kMaxSlots][kMaxSlots];
    int n_children[kMaxSlots];
    int by_pi[kMaxSlots];          // slots in increasing pi index
    int root_dir;                  // the list whose T positions key the root: 1 (in-lists)
                                   // when every child of the center attaches at its
                                   // destination, else 0 (out-lists)
    int same_window[kMaxSlots];    // 1: same parent, side, direction and time side as
                                   // the previous slot (a leaf sibling): same window
    // non-tree edges in pi order, and maximal runs of consecutive ones
    int n_free = 0;
    int free_src[TM_MAX_L], free_dst[TM_MAX_L];
    int n_runs = 0;
    int run_first[TM_MAX_L], run_len[TM_MAX_L];
    int run_prev[TM_MAX_L], run_next[TM_MAX_L];  // tree slots around a run, -1 at the ends
    // partial-order motifs whose order is not total (po = 1): the relation
    // "strictly earlier" as bit masks -- over tree slots for each tree slot,
    // and for each non-tree edge (n_free index) over tree slots before it,
    // tree slots after it and the non-tree edges before it
    int po = 0;
    uint16_t po_tpred[kMaxSlots];
    uint16_t po_f_tpred[TM_MAX_L], po_f_tsucc[TM_MAX_L], po_f_fpred[TM_MAX_L];
};

// Non-tree edges a partial-order motif may have on the GPU (its completion
// counter keeps one count per set of them).
constexpr int kPoMaxFree = 5;

int plan_build(const tm_motif* mo, const tm_tree* tr, HostPlan* out);
int motif_check(const tm_motif* mo);

// ---------------------------------------------------------------------------
// Per-slot tables of a weight set.  For a non-leaf slot s, the build computes
// per eid e w_i(s, e) for the interval i of parity par that holds e (each
// edge lies in at most one interval of each parity) into vals[s][par], a
// temporary.  What stays are exclusive prefix sums of those values: for
// non-leaf, non-center slots along the lists in which their parent looks them
// up (qt: T order, qn: N order, per parity); for the center along eid order
// (qc).  A value is the difference of two neighbouring prefix entries.
// ---------------------------------------------------------------------------
struct tm_weights {
    tm_graph* g = nullptr;
    HostPlan plan;
    bool wide = false;
    int64_t q = 0;
    u128 W = 0;
    // constraints 2 (exclusion) and 3 (2 delta intervals), TM_C_*; ilen is the
    // interval unit: delta with constraint 3, else T + 1 (one interval)
    uint32_t constraints = TM_C_ALL;
    int64_t ilen = 0;
    void* vals[kMaxSlots][2] = {};  // build temporaries (both parities interleaved in vals[s][0]), null afterwards
    // child windows, per non-center slot and interval parity: the slot's
    // candidate window (p0, p1, q0, q1) for every edge its parent can match,
    // by that edge's position x in the T order of the list the slot attaches
    // to (out-lists for a slot at its parent's source, in-lists at its
    // destination: the order the level kernel walks); null when not kept.
    // The two parities interleave, one 32-byte record per edge:
    // parity par's window of position x is win[s][par][2 x] (win[s][1] is
    // win[s][0] + 1).
    int4* win[kMaxSlots][2] = {};
    bool has_win = false;
    // a server builds its sets for memory over speed: no kept windows and a
    // guide four times coarser
    bool lean = false;
    // which widths a build may use: 0 both (64 bits, widened or rebuilt in
    // 128 when needed), 1 only 64 (a build needing more stops with
    // TM_EOVERFLOW and needs_wide set), 2 only 128
    int width_mode = 0;
    bool needs_wide = false;
    // list prefix tables, per non-center slot and parity (T and N order):
    // 128-bit entries only when the set was built in 128 bits; a set widened
    // after a 64-bit build keeps its 64-bit list tables, which are exact
    // (only center and interval totals outgrew 64 bits)
    void* qt[kMaxSlots][2] = {};
    void* qn[kMaxSlots][2] = {};
    // every kCoarse-th entry of each qt table (m / kCoarse + 1 entries, the
    // table's width): a search over a window goes through it first, so the
    // probes far apart fall in a table 16 times smaller
    void* qtc[kMaxSlots][2] = {};
    bool list_wide = false;
    void* qc[2] = {};
    int32_t* ilo = nullptr;  // [q] first eid of I_i
    int32_t* ihi = nullptr;  // [q] one past the last eid of I_i
    void* cumW = nullptr;    // [q+1] prefix of W_i
    // root pairs (interval << 32 | eid) and their sort keys at the draws
    // X = b 2^(128 - guide_bits), b = 0 .. 2^guide_bits (the last at
    // X = 2^128 - 1): a draw in bucket b picks a pair between entries b and b + 1
    RootGuide* guide = nullptr;
    int guide_bits = 0;
    void* ioff = nullptr;    // [q] cum[i] - qc[lo_i] of the interval's parity
    DevArena arena;
};

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
int graph_build(tm_graph* g, const int32_t* src, const int32_t* dst, const int64_t* t,
                hipStream_t st);
// model_bytes (optional): the level kernels' access-model bytes (every
// attempt, as the level stage timing counts every attempt).
int weights_build(tm_weights* w, hipStream_t st, u64* model_bytes = nullptr);
// The 64-bit weight build enqueued on st with no host synchronisation; a
// product or prefix that does not fit 64 bits sets *ovf (device).  The
// caller reads W from cumW[q] afterwards, or rebuilds with weights_build.
struct StageTimer;
// level_timers (optional): each level launch's stage timer, for the caller to
// finish once the stream is synchronised.
int weights_enqueue(tm_weights* w, hipStream_t st, int* ovf,
                    std::vector<std::unique_ptr<StageTimer>>* level_timers = nullptr);
// wflag (optional): w's 64-bit build was enqueued on st with that overflow
// flag and not waited for (weights_enqueue); W is then read with the sums,
// *overflowed tells whether the tables overflowed (the result is then
// unset), and only plain sampling (no records, no byte count) is allowed.
// sample_run's non-deferred path with its temporaries in a file-scope device
// array instead of allocations (tm_sample_noalloc).
int sample_run_noalloc(tm_weights* w, u64 seed, u64 j0, u64 count, u64 k_total, hipStream_t st, tm_result* out,
                       tm_sample_rec* recs);
int sample_run(tm_weights* w, u64 seed, u64 j0, u64 count, u64 k_total, hipStream_t st,
               tm_result* out, tm_sample_rec* recs, u64* model_bytes, const int* wflag = nullptr,
               bool* overflowed = nullptr);

// Device bytes of a weight set's tables (prefix arrays, intervals) for a
// graph of m edges and q intervals, in 64-bit (wide = false) or 128-bit form,
// and the temporaries a build holds on top of them at its peak (one slot's
// values, per parity).
u64 weights_footprint(const HostPlan& P, int64_t m, int64_t q, bool wide, bool lean = false);
// Whether a weight set keeps its child windows: at most kWinMaxBytes of them
// (servers build lean sets without them).
constexpr u64 kWinMaxBytes = (u64)32 << 30;
u64 weights_window_bytes(const HostPlan& P, int64_t m);
bool weights_keep_windows(const HostPlan& P, int64_t m);
u64 weights_build_extra(int64_t m, bool wide);
// Bits of the root guide for a graph of m edges: about one (interval, edge)
// pair per bucket (lean sets: about eight), between 2^8 and 2^26 buckets (lean
// sets: 2^23).
constexpr int kGuideExtraBits = 1;
constexpr int kCoarseBits = 4;  // list prefix tables: one coarse entry per 2^kCoarseBits
int guide_bits_for(int64_t m, bool lean = false);

// Exact sums over a range of samples of one job.  Sums over disjoint ranges
// add up to the sums over their union, whatever the split.
struct JobSums {
    u128 acc2 = 0, acc2_sq = 0;
    u64 n_valid = 0, n_vertex = 0, n_delta = 0, n_order = 0, n_nonzero = 0;
    u64 flags = 0;  // bit 0: acc2 reached 2^128; bit 1: acc2_sq saturated
    int status = TM_OK;
};
void sums_merge(JobSums& into, const JobSums& x);
// Copy sums into a result (which already holds k, q, W and flags).
void sums_to_result(const JobSums& s, tm_result* out);

// Batched sampling of several weight sets in one pass (tile: samples per work
// item of the persistent kernels; blocks: their grid, 0 = 8 per CU).
struct BatchConfig {
    int tile;          // samples per tile (each of a workgroup's lanes takes tile / kBlock)
    int blocks;        // persistent grid (0: 8 workgroups per CU)
    u64 group_limit;   // root keys and samples per batched pass (0: 2^32)
    int root_lds;      // LDS bytes staging a job's interval prefix in the root draws
};
extern BatchConfig g_batch_config;
// Samples j0[x] .. j0[x] + count[x] - 1 of every job x with W > 0; per-job
// errors go to out[x].status.
int batch_sample_pass(tm_weights* const* ws, const u64* j0, const u64* count, const u64* seeds, int n,
                      hipStream_t st, JobSums* out, const BatchConfig& cfg);

// Motif families: k samples of w's tree, each completed for every member
// plan (same tree slots, own non-tree edges).  sums[f]: acc2, acc2_sq and
// nonzero counts of member f; shared: the validation counts of the stream.
int family_run(tm_weights* w, const HostPlan* plans, int n, u64 seed, u64 k, hipStream_t st, JobSums* sums,
               JobSums* shared);

// Random instance listing of samples j0 .. j0 + count - 1 (eids: device,
// count x TM_MAX_L; recs: device records or NULL).
int list_run(tm_weights* w, u64 seed, u64 j0, u64 count, hipStream_t st, int32_t* eids, tm_sample_rec* recs);

// The captured form of a batched pass over jobs whose 64-bit weights are
// being built earlier on st: every launch and copy is enqueued with no host
// synchronisation or read; W comes from each job's table and a job whose
// wflag is set (overflow) or whose W is 0 draws nothing.  Jobs with
// count[x] = 0 are left out.  The handle owns the buffers (and the pinned
// staging the recorded uploads read) until batch_capture_free.
struct CapturedPass;
int batch_capture_enqueue(tm_weights* const* ws, const int* const* wflag, const u64* count, const u64* seeds,
                          int n, hipStream_t st, const BatchConfig& cfg, CapturedPass** out);
// Sums of every job after the recorded work ran (synchronises st).
int batch_capture_read(CapturedPass* p, hipStream_t st, JobSums* out);
void batch_capture_free(CapturedPass* p, hipStream_t st);

BatchConfig batch_config_now();
int sample_batch_results(tm_weights* const* w, const uint64_t* k, const uint64_t* seed, int n_jobs,
                         hipStream_t st, tm_result* out);
// Estimate and standard error of a result whose W, k, acc2 and acc2_sq are set.
void finish_result(tm_result* r);

// ---------------------------------------------------------------------------
// Stage timing with HIP events on the call's stream (tm_profile_enable).
// ---------------------------------------------------------------------------
bool prof_enabled(int stage);
void prof_add(int stage, double ms);
// Stage timing off on this thread (while recording a graph).
void prof_suspend(bool on);
bool prof_suspended();

// Timing events of the current device from a list kept per device (creating
// and destroying two for every timed stage costs more than recording them).
// Null when no event can be created; *dev receives the device to release on.
hipEvent_t timing_event_acquire(int* dev);
void timing_event_release(hipEvent_t e, int dev);

struct StageTimer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t st = nullptr;
    int stage = 0, dev = 0;
    bool on = false;
    StageTimer() = default;
    StageTimer(const StageTimer&) = delete;
    StageTimer& operator=(const StageTimer&) = delete;
    void start(int stage_, hipStream_t st_) {
        stage = stage_;
        st = st_;
        if (!prof_enabled(stage)) return;
        a = timing_event_acquire(&dev);
        b = a ? timing_event_acquire(&dev) : nullptr;
        on = a && b;
        if (on) (void)hipEventRecord(a, st);
        else release();
    }
    void stop() {
        if (on) (void)hipEventRecord(b, st);
    }
    // after the stream has been synchronised
    void finish() {
        if (!on) return;
        float ms = 0.f;
        if (hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess)
            prof_add(stage, ms);
        release();
    }
    ~StageTimer() { release(); }

   private:
    void release() {
        if (a) timing_event_release(a, dev);
        if (b) timing_event_release(b, dev);
        a = b = nullptr;
        on = false;
    }
};
