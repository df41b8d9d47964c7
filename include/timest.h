/*
 * timest.h -- C ABI of the MI355X (gfx950) TIMEST hot path.
 *
 * TIMEST (arXiv 2507.20441) estimates the number of temporal motif matches
 * in a temporal multigraph by sampling weighted temporal spanning-tree
 * matches.  This library runs its data-parallel hot path on one AMD Instinct
 * MI355X: CSR build of the time-sorted edge lists, the bottom-up spanning-tree
 * weights, the weighted tree sampler, validation and completion counting of
 * each sample, and the reduction into the estimate.  Every stage is a HIP
 * kernel written for CDNA4; the host code here only plans and launches.
 *
 * Conventions shared by every call:
 *   - Return value: TM_OK (0) or a negative TM_E* code; tm_last_error() then
 *     holds a message for the calling thread.  A failed call leaves its
 *     output handles untouched and the library usable.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *     on it; calls that return values to host memory synchronise it first.
 *   - Device memory is allocated through the graph's or server's allocator
 *     (tm_allocator; NULL: the library's own hipMalloc-backed block cache)
 *     and owned by the handle that holds it until its destroy call.
 *   - Sizes: at most 2^31 - 1 edges and 2^31 - 1 vertices; the time span
 *     max(t) - min(t) and delta must stay below 2^62, and the number of bits
 *     of (n - 1) plus the number of bits of the time span must not exceed 64
 *     (the per-vertex neighbour lists are searched on a packed 64-bit key).
 */
#ifndef TIMEST_H
#define TIMEST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TM_MAX_K 8   /* motif vertices */
#define TM_MAX_L 16  /* motif edges */

enum tm_error {
    TM_OK = 0,
    TM_EINVAL = -1,      /* NULL or malformed argument, vertex id out of range,
                            bad motif or tree */
    TM_ESELFLOOP = -2,   /* an edge (u, u, t) */
    TM_EDUP = -3,        /* a tuple (u, v, t) given twice (Sec. 1.1 forbids it) */
    TM_EOVERFLOW = -4,   /* a weight, W or a completion count reaches 2^128 */
    TM_ERANGE = -5,      /* time span or delta too large for the limits above */
    TM_ENOMEM = -6,      /* device allocation failed */
    TM_EDEVICE = -7,     /* HIP runtime error */
    TM_EADMIT = -8,      /* serving: the query's weight set alone exceeds the budget */
    TM_EAGAIN = -9,      /* serving: the query has not finished yet */
    TM_ECANCELED = -10   /* serving: the server shut down before the query finished */
};

enum tm_ptr_kind { TM_PTR_HOST = 0, TM_PTR_DEVICE = 1 };

/* Constraints on the sampled tree matches (Sec. "A Closer Look at
 * Preprocessing"; Tab. "constraints"): constraint 1 -- order and delta
 * between a tree edge and its parent -- always holds; TM_C_EXCLUDE adds
 * constraint 2 (a child's far endpoint differs from the parent's other
 * endpoint), TM_C_WINDOWS constraint 3 (the overlapping 2 delta intervals;
 * without it one interval spans all times and N_phi = 1).  Every mode gives
 * an unbiased estimate; the default is TM_C_ALL. */
#define TM_C_EXCLUDE 1u
#define TM_C_WINDOWS 2u
#define TM_C_ALL 3u

/* result flags */
#define TM_F_W_ZERO 1u        /* no partial match exists: estimate is 0 */
#define TM_F_SQ_SATURATED 2u  /* acc2_sq reached 2^128 - 1 and stopped */
#define TM_F_WIDE 4u          /* weights needed 128 bits (else 64) */

typedef struct { uint64_t lo, hi; } tm_u128;

/* A caller's device memory provider (the Python binding can pass PyTorch's
 * caching allocator).  alloc returns at least `bytes` of device memory on the
 * current device, first used on `stream` (a hipStream_t), or NULL when it
 * cannot; free takes back a block alloc returned, with its size and the
 * stream its last use was enqueued on.  Both may be called from any thread
 * of the library (a server's workers included) and get ctx back.  A graph
 * created with an allocator takes its tables, the tables of every weight set
 * built on it and the temporaries of every call on them (a batch: its first
 * job's graph's) from it; a server created with one takes its weight sets
 * and pass buffers from it.  The functions and ctx must stay valid until
 * every handle using them is destroyed.  tm_sample_noalloc allocates
 * nothing, through any allocator. */
typedef struct {
    void* (*alloc)(void* ctx, size_t bytes, void* stream);
    void (*free)(void* ctx, void* ptr, size_t bytes, void* stream);
    void* ctx;
} tm_allocator;

typedef struct tm_graph tm_graph;
typedef struct tm_weights tm_weights;

/* Temporal motif M = (H, pi, delta) (Def. "temporal motif"): l directed edges
 * src[p] -> dst[p] over vertices 0..k-1, listed in pi order (edge p must be
 * the p-th in time).  2 <= k <= 8, 1 <= l <= 16, no self loop, weakly
 * connected, 1 <= delta < 2^62.  Parallel motif edges are allowed.
 *
 * Partial-order motifs (the generalisation to "a partial order of time
 * constraints", Sec. 1.1 remark and Sec. 6): partial = 1 keeps only the
 * pairs of `before` and the pairs they imply -- bit p of before[q] says edge
 * p must be strictly earlier than edge q -- and leaves every other pair
 * unordered (either order, or equal times).  The list must be a linear
 * extension (bits p < q < l only) and parallel motif edges must be ordered
 * (else two of them could take one graph edge); an unordered pair of tree
 * edges searches the window [t - delta, t + delta].  A relation whose
 * closure orders every pair is the total order and runs as partial = 0.
 * The GPU path completes at most 5 non-tree edges under a partial order
 * (TM_EINVAL beyond); families and instance listing take total orders only.
 * partial = 0 (zero-initialised) is the total order of the list. */
typedef struct {
    int32_t k;
    int32_t l;
    int32_t src[TM_MAX_L];
    int32_t dst[TM_MAX_L];
    int64_t delta;
    uint32_t partial;
    uint16_t before[TM_MAX_L];
} tm_motif;

/* Spanning tree S of the motif (Def. "spanning tree of a temporal motif"):
 * k - 1 distinct motif edge indices forming a tree of the underlying
 * undirected graph, and the center (root) edge, one of them (Sec. 4.1). */
typedef struct {
    int32_t n_edges;
    int32_t edge[8];
    int32_t center;
} tm_tree;

/* Outcome of an estimate (Alg. 6).  acc2 is the exact sum over samples of
 * 2 * M_phi / N_phi (M_phi: motif matches completing the sampled tree match,
 * N_phi in {1, 2}: intervals holding it); estimate = W * acc2 / (2 k), each
 * 128-bit integer converted to double with round-to-nearest-even.
 * std_error = (W / 2) * s / sqrt(k), s the sample standard deviation of the
 * terms 2 M_phi / N_phi (see tm_result_finish for its exact evaluation). */
typedef struct {
    double estimate;
    double std_error;
    tm_u128 W;           /* total sampling weight (Claim "num-matches-entire-tree") */
    tm_u128 acc2;
    tm_u128 acc2_sq;     /* sum of squares of the same terms */
    uint64_t k;
    uint64_t n_valid;     /* samples passing Alg. 4 */
    uint64_t n_bad_vertex;/* vertex map not 1-1 */
    uint64_t n_bad_delta; /* tree edges not within delta */
    uint64_t n_bad_order; /* tree edges not in pi order */
    uint64_t n_nonzero;   /* valid samples with M_phi > 0 */
    int64_t q;            /* number of 2*delta intervals */
    uint32_t flags;       /* TM_F_* */
    int32_t status;       /* TM_OK, or the error of this job in batched calls */
} tm_result;

/* One per sample: the interval drawn, the validation outcome (0 valid,
 * 1 vertex map not 1-1, 2 outside delta, 3 out of order, 4 not drawn because
 * W = 0), N_phi and M_phi (0 unless valid), and the eids matched to the tree
 * edges listed in increasing pi index (-1 past the last tree edge).  An eid
 * is the rank of an edge under the key (time, src, dst). */
typedef struct {
    uint32_t interval;
    uint32_t status;
    uint32_t n_phi;
    uint32_t pad;
    int32_t eid[8];
    tm_u128 m_phi;
} tm_sample_rec;

/* Message of a TM_E* code; static storage. */
const char* tm_strerror(int code);
/* Detail of the last failed call on this thread; static thread-local storage. */
const char* tm_last_error(void);

/* Build the graph (Sec. 4, storage): validate the m edges (src[i], dst[i],
 * t[i]), shift times so the earliest is 0, order edges by (time, src, dst)
 * (that rank is the eid), and build per-vertex out- and in-lists in time
 * order plus the same lists ordered by (neighbour, time), which hold every
 * multi-edge list El_{u,v} (Def. "multi-edge list") as a contiguous run.
 * src, dst, t: m entries each, host or device memory per ptr_kind; the caller
 * keeps ownership and may free them once the call returns.  n: vertex count,
 * ids in [0, n).  m = 0 gives an empty graph.  alloc: NULL (the library's
 * block cache) or the allocator of the graph and of everything built on it
 * (copied; see tm_allocator).  Errors: TM_EINVAL (NULL, m or n out of range,
 * id out of range), TM_ESELFLOOP, TM_ERANGE, TM_EDUP -- the first failing
 * check in that order -- TM_ENOMEM, TM_EDEVICE. */
int tm_graph_create(const int32_t* src, const int32_t* dst, const int64_t* t, int64_t m,
                    int32_t n, int ptr_kind, const tm_allocator* alloc, void* stream, tm_graph** out);

/* Frees the graph's device memory.  Weights built on it must be destroyed
 * first.  NULL is ignored. */
void tm_graph_destroy(tm_graph* g);

/* Sizes of a graph; any output pointer may be NULL. */
int tm_graph_info(const tm_graph* g, int64_t* m, int32_t* n, int64_t* t_shift,
                  int64_t* t_span, uint64_t* device_bytes);

/* Arrays of the built graph, copied to host memory for inspection. */
enum tm_graph_array {
    TM_ARR_SRC = 0,      /* int32[m]  source by eid */
    TM_ARR_DST = 1,      /* int32[m]  destination by eid */
    TM_ARR_T = 2,        /* int64[m]  shifted time by eid */
    TM_ARR_OUT_OFF = 3,  /* int32[n+1] offsets of each vertex's out-lists */
    TM_ARR_IN_OFF = 4,   /* int32[n+1] offsets of each vertex's in-lists */
    TM_ARR_OUT_EID = 5,  /* int32[m]  out-lists in time order (eids) */
    TM_ARR_IN_EID = 6,   /* int32[m]  in-lists in time order (eids) */
    TM_ARR_OUTN_EID = 7, /* int32[m]  out-lists in (destination, time) order */
    TM_ARR_INN_EID = 8,  /* int32[m]  in-lists in (source, time) order */
    TM_ARR_OUT_T = 9,    /* int64[m]  out-lists in time order: times */
    TM_ARR_IN_T = 10,    /* int64[m]  in-lists in time order: times */
    TM_ARR_OUT_NBR = 11, /* int32[m]  out-lists in time order: destinations */
    TM_ARR_IN_NBR = 12,  /* int32[m]  in-lists in time order: sources */
    TM_ARR_OUT_POS = 13, /* int32[m]  by eid: the edge's position in the out-lists' time order */
    TM_ARR_IN_POS = 14,  /* int32[m]  by eid: the edge's position in the in-lists' time order */
    TM_ARR_OUTN_KEY = 15, /* uint64[m] out-lists in N order: destination << b | time, b the
                           * bits of the largest shifted time (at least 1) */
    TM_ARR_INN_KEY = 16, /* uint64[m] in-lists in N order: source << b | time */
    TM_ARR_OUTN_POS = 17, /* int32[m] out-lists in N order: each entry's time-order position */
    TM_ARR_INN_POS = 18  /* int32[m]  in-lists in N order: each entry's time-order position */
};
int tm_graph_export(const tm_graph* g, int which, void* host_out, void* stream);

/* Default spanning tree and center: the tree with the smallest constraint
 * looseness (Alg. 8, taken per tree vertex over pairs of incident tree edges
 * as |pi(e1) - pi(e2)| - 1), ties to the lexicographically smallest edge set;
 * the center minimises the rooted height, ties to the smallest pi index. */
int tm_default_tree(const tm_motif* mo, tm_tree* out);

/* Preprocess (Alg. 1, Alg. 2): for every edge e, every non-leaf tree edge s
 * and both 2*delta intervals I_i = [i delta, (i+2) delta) holding e, the
 * s-weight w_i(s, e) (Def. "s-weight", Claim "overall-num-matches"), exact;
 * then W_i and W (Claim "num-matches-entire-tree").  The tables stay resident
 * in device memory for any number of tm_sample calls.  tr = NULL takes
 * tm_default_tree.  Weights are computed in 64 bits and recomputed in 128
 * bits when any value or prefix sum would reach 2^64.  Errors: TM_EINVAL,
 * TM_ERANGE (bit limits above), TM_EOVERFLOW, TM_ENOMEM, TM_EDEVICE. */
int tm_weights_create(tm_graph* g, const tm_motif* mo, const tm_tree* tr, void* stream,
                      tm_weights** out);
/* tm_weights_create under a subset of the constraints (TM_C_*). */
int tm_weights_create_ex(tm_graph* g, const tm_motif* mo, const tm_tree* tr, uint32_t constraints,
                         void* stream, tm_weights** out);
void tm_weights_destroy(tm_weights* w);

/* W, the interval count q, whether 128-bit weights were needed, the device
 * bytes held and the tree used; any output pointer may be NULL.  A set whose
 * 64-bit build overflowed only in the center's totals along eid order is
 * widened in place: its center and interval tables become 128-bit, its list
 * tables stay 64-bit (exact), and device_bytes is then below the 128-bit
 * footprint of tm_weights_footprint. */
int tm_weights_info(const tm_weights* w, tm_u128* W, int64_t* q, int32_t* wide,
                    uint64_t* device_bytes, tm_tree* tree);

/* w_i(s, e) for every eid e, with i = floor(t(e) / delta) - slot (slot 0 or 1;
 * entries with i < 0 are 0); s is a tree edge's motif index.  Leaf edges give 1.
 * host_out: m entries. */
int tm_weights_export(const tm_weights* w, int32_t s, int32_t slot, tm_u128* host_out,
                      void* stream);

/* W_i for i = 0 .. q-1 into host memory. */
int tm_weights_intervals(const tm_weights* w, tm_u128* host_out, void* stream);

/* Draw samples j = j0 .. j0 + count - 1 (Alg. 3 SampleSubg, Alg. 4, Alg. 5)
 * and reduce them (Alg. 6).  Draw d of sample j is the Philox4x32-10 block
 * for counter (j mod 2^32, j >> 32, d, 0) and key (seed mod 2^32, seed >> 32)
 * read as a 128-bit X; it selects floor(X * n / 2^128) among n.  Draw 0 picks
 * the (interval, center edge) pair by inverse CDF over pairs in (interval,
 * eid) order weighted by w_i(c, e); draw d >= 1 picks the d-th tree edge in
 * pre-order (children in increasing pi index) by inverse CDF over its
 * candidate list (Claim "matching-edges-set") in eid order.  k_total is the k
 * of the estimate formula (count for a whole run).  recs: NULL, or device
 * memory for count records.  Synchronises the stream.  Results for a given
 * (weights, seed, j) never depend on how samples are split across calls. */
int tm_sample(tm_weights* w, uint64_t seed, uint64_t j0, uint64_t count, uint64_t k_total,
              void* stream, tm_result* out, tm_sample_rec* recs);

/* tm_sample for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same draws, kernels and results as tm_sample, but every temporary -- the
 * per-workgroup partial sums, a flag word, the root keys and sample offsets
 * of the sort by root and the sort's histograms, about 36 MiB -- lives in one
 * file-scope device array, never in hipMalloc'd memory; no hipMalloc, hipFree
 * or other allocating routine is called.  Each device the library runs on
 * holds its own copy of the array until the process ends.  At most 2^21
 * samples per call (TM_EINVAL beyond: split the id range, whose sums add up
 * exactly).  Calls that overlap on one device race on the shared array (run
 * them one after another on a device); the caller still provides w, out and
 * recs (NULL, or device memory for count records).  Synchronises the stream.
 * Errors: TM_EINVAL, TM_EOVERFLOW, TM_EDEVICE. */
int tm_sample_noalloc(tm_weights* w, uint64_t seed, uint64_t j0, uint64_t count, uint64_t k_total,
                      void* stream, tm_result* out, tm_sample_rec* recs);

/* Recompute out->estimate and out->std_error from its W, acc2, acc2_sq, k
 * and flags (Alg. 6; the standard error of Sec. 4.4): for results of
 * sample ranges whose exact sums the caller has added up.  Host-only; no
 * device work.  std_error = (W / 2) sqrt(D / (k^2 (k - 1))) with
 * D = k acc2_sq - acc2^2 formed exactly in 256 bits and rounded once to
 * double; 0 when k < 2, W = 0 or TM_F_SQ_SATURATED is set.  Errors:
 * TM_EINVAL (NULL). */
int tm_result_finish(tm_result* out);

/* One whole estimate (Alg. 6, Estimate(M, G, k)): tm_weights_create,
 * tm_sample(j0 = 0, count = k_total = k), tm_weights_destroy.  recs: NULL,
 * or device memory for k records (tm_sample's).  W = 0 gives TM_OK with
 * estimate 0 and TM_F_W_ZERO.  Errors: as tm_weights_create and tm_sample. */
int tm_estimate(tm_graph* g, const tm_motif* mo, const tm_tree* tr, uint64_t k,
                uint64_t seed, void* stream, tm_result* out, tm_sample_rec* recs);
/* tm_estimate under a subset of the constraints (TM_C_*). */
int tm_estimate_ex(tm_graph* g, const tm_motif* mo, const tm_tree* tr, uint32_t constraints, uint64_t k,
                   uint64_t seed, void* stream, tm_result* out, tm_sample_rec* recs);

/* ---- batched estimation (many jobs in one pass) -------------------------
 * Every job's samples are drawn exactly as tm_sample draws them (same seed,
 * same sample ids 0 .. k-1), so each job's result is bit-identical to its
 * own tm_sample / tm_estimate; only the schedule differs.  The root draws of
 * all jobs run in one launch, one radix sort orders all samples by (job,
 * root list position), and persistent kernels pull (job, sample range)
 * tiles from a device counter, with one reduction per job.  Per-job errors
 * go to out[i].status; the call fails only on a device or argument error. */

/* Sample jobs i = 0 .. n_jobs-1 from resident weight sets: k[i] samples with
 * seed seed[i] from w[i].  Synchronises the stream. */
int tm_sample_batch(tm_weights* const* w, const uint64_t* k, const uint64_t* seed, int n_jobs,
                    void* stream, tm_result* out);

/* Whole estimates for n_jobs (graph, motif, tree, k, seed) jobs: the 64-bit
 * weight builds of all jobs are enqueued back to back with a single
 * synchronisation (jobs that overflow 64 bits are rebuilt in 128 bits), then
 * tm_sample_batch.  tr may be NULL (default trees) or hold per-job pointers
 * (NULL entries take the default).  Results equal tm_estimate's per job. */
int tm_estimate_batch(tm_graph* const* g, const tm_motif* mo, const tm_tree* const* tr,
                      const uint64_t* k, const uint64_t* seed, int n_jobs, void* stream,
                      tm_result* out);

/* A batch plan: the 64-bit pipeline of a fixed set of jobs -- every weight
 * build, the root draws, the sort, the sampling and the per-job reductions --
 * recorded once into a HIP graph on streams of the plan's own (the weight
 * builds on four parallel branches, balanced by edge count, joined before
 * the batched pass) and replayed by tm_batch_plan_run with no host work
 * between the stages.  Jobs whose
 * weights need 128 bits draw nothing in the graph and are re-run by
 * tm_estimate after each replay.  The graphs must stay alive and unchanged;
 * tr and its entries may be NULL (default trees).  Results equal
 * tm_estimate's per job.  Errors: TM_EINVAL (as tm_estimate_batch, or a job
 * of 2^32 samples or more), TM_ERANGE, TM_ENOMEM, TM_EDEVICE (recording). */
typedef struct tm_batch_plan tm_batch_plan;
int tm_batch_plan_create(tm_graph* const* g, const tm_motif* mo, const tm_tree* const* tr,
                         const uint64_t* k, const uint64_t* seed, int n_jobs, void* stream,
                         tm_batch_plan** out);
/* Replay on `stream` and write one result per job; synchronises the stream.
 * Replays may not overlap (they share the plan's buffers). */
int tm_batch_plan_run(tm_batch_plan* p, void* stream, tm_result* out);
void tm_batch_plan_destroy(tm_batch_plan* p);

/* Schedule of the batched kernels: samples per tile (>= 256) and the grid of
 * the persistent kernels (0 = 8 workgroups per compute unit).  Process-wide;
 * the autotuner in the Python package searches these.  Returns the previous
 * values through prev_tile / prev_blocks when not NULL. */
int tm_batch_config(int tile, int blocks, int* prev_tile, int* prev_blocks);

/* The full schedule of the batched kernels (tm_batch_config sets the first
 * two fields only).  Process-wide; the autotuner searches these.
 *   tile: samples per tile, >= 256; each lane of a 256-lane workgroup takes
 *     tile / 256 of a tile's samples (the samples per lane);
 *   blocks: workgroups of the persistent kernels (0 = 8 per compute unit);
 *   root_lds: LDS bytes per workgroup that stage a job's interval prefix W_i
 *     for its root draws when it fits (jobs with a root guide read one or
 *     two entries and stage nothing), 0 .. 65536;
 *   group_limit: root keys (two per edge) and samples one batched pass may
 *     hold (0 = 2^32, what 32-bit sort keys allow); a smaller value splits a
 *     batch into more passes without changing any result.
 * in may be NULL (read only); prev may be NULL.  Errors: TM_EINVAL. */
typedef struct {
    int32_t tile;
    int32_t blocks;
    int32_t root_lds;
    int32_t pad;
    uint64_t group_limit;
} tm_batch_opts;
int tm_batch_options(const tm_batch_opts* in, tm_batch_opts* prev);

/* Random instance listing (Sec. 4.3): samples j0 .. j0 + count - 1 of w's
 * motif with the given seed (the draws of tm_sample); every valid sample with
 * 0 < M_phi <= 2^20 lists its r-th completion, r = floor(X M_phi / 2^128)
 * with X the 128-bit Philox block of draw 15 of the sample, completions
 * ordered lexicographically by the eids of the motif edges in pi order (tree
 * edges fixed).  A motif instance H whose tree image is phi is thus listed by
 * a sample with probability (N_phi / W) / M_phi.  eids: device memory,
 * count x 16 int32, each row the eids of the motif's edges in pi order (-1
 * beyond l, and in rows that list nothing).  recs: NULL or device memory for
 * count records (the samples' tree images, N_phi and M_phi).  Synchronises
 * the stream.  Errors: TM_EINVAL, as tm_sample. */
int tm_list_instances(tm_weights* w, uint64_t seed, uint64_t j0, uint64_t count, void* stream, int32_t* eids,
                      tm_sample_rec* recs);

/* Motif families (Sec. 4.3; the paper counts its 4-vertex motifs "at once",
 * Tab. "4-vertex-runtime"): motifs whose spanning tree is w's -- the same
 * tree edges (the same source and destination vertices, each matching one
 * edge of the motif, in the same relative order), the same vertex count and
 * delta -- and that differ only in their non-tree edges.  One stream of k
 * tree samples (seed, ids 0 .. k-1) is drawn and validated once; every
 * sample is completed for each motif.  out[f] equals tm_sample of motif f's
 * own weights with that tree (the weights depend on the tree alone).
 * Errors: TM_EINVAL (a motif that does not share the tree), as tm_sample. */
int tm_sample_family(tm_weights* w, const tm_motif* motifs, int n_motifs, uint64_t seed, uint64_t k,
                     void* stream, tm_result* out);

/* Spanning-tree candidates (Sec. "Choosing the Spanning Tree", Alg. 8):
 * every (spanning tree, center) pair of the motif, ordered by constraint
 * looseness -- per motif vertex, over unordered pairs of tree edges incident
 * to it, |pi(e1) - pi(e2)| - 1 -- then by edge set (lexicographic), rooted
 * height and center; the first is tm_default_tree's choice.  Writes at most
 * max_out trees (and their looseness, when looseness is not NULL) and sets
 * *n_out to the number of pairs.  Errors: TM_EINVAL. */
int tm_tree_candidates(const tm_motif* mo, tm_tree* out, int64_t* looseness, int max_out, int* n_out);

/* Alg. 7: the first n_c candidates' total weight W on the graph (a full
 * weight build each, released afterwards); the smallest W wins, the earlier
 * candidate among equals.  W_out (may be NULL) receives the min(n_c, count)
 * values in candidate order and *n_eval (may be NULL) their number.
 * Synchronises the stream.  Errors: as tm_weights_create. */
int tm_choose_tree(tm_graph* g, const tm_motif* mo, int n_c, void* stream, tm_tree* best, tm_u128* W_out,
                   int* n_eval);

/* Device bytes the weight tables of (g, mo, tr) take in 64-bit (wide = 0)
 * or 128-bit (wide = 1) form: what tm_weights_info reports as device_bytes
 * after tm_weights_create builds them in that form (for a widened set, an
 * upper bound: see tm_weights_info), the kept child windows
 * included (kept when they total at most 32 GiB; a server builds its sets
 * without them).  tr may be NULL (the default tree).  Errors: TM_EINVAL. */
int tm_weights_footprint(const tm_graph* g, const tm_motif* mo, const tm_tree* tr, int32_t wide,
                         uint64_t* bytes);

/* ---- serving --------------------------------------------------------------
 * A server answers estimation queries on resident graphs from a worker
 * thread with a stream of its own (default priority).
 *
 * Weight sets are cached per (graph, motif, delta, time order, tree) and
 * shared by the queries that need them.  The budget bounds the server's
 * device memory: the resident weight sets, the one set being built with its
 * temporaries, and a reserve for one sampling pass (24 bytes per sample of
 * pass_samples).  Admission: a query whose weight set is resident is
 * admitted at once; otherwise, smallest set first, when the set's footprint
 * and its build's temporaries fit the budget after evicting idle sets, least
 * recently used first.  A set first reserves its 64-bit size; if it turns
 * out to need 128 bits, the 64-bit attempt stops, its memory goes back to
 * HIP and the query waits for the 128-bit reservation (every later build of
 * that set reserves 128 bits at once; TM_EADMIT if that can never fit).
 *
 * Continuous batching: each pass draws up to job_chunk samples of every
 * admitted query (fewest remaining samples first, at most max_jobs queries
 * and pass_samples samples in all) with one batched sampling pass, so a query
 * arriving during a long one joins at the next pass.  A query's result is
 * its exact integer sums over its passes, hence equal to tm_estimate's for
 * the same (graph, motif, tree, k, seed), whatever else is in the mix. */
typedef struct tm_server tm_server;

typedef struct {
    uint64_t pass_samples;  /* samples per pass over all queries (0: 2^24) */
    uint64_t job_chunk;     /* samples one query adds to a pass (0: 2^22) */
    int32_t max_jobs;       /* queries per pass (0: 256) */
    int32_t fifo;           /* 1: oldest query first in a pass instead of fewest remaining */
} tm_server_opts;

typedef struct {
    double queued_ms;      /* submit -> admitted (its weight set resident) */
    double latency_ms;     /* submit -> result ready */
    uint32_t weights_hit;  /* 1: the weight set was resident on admission */
    uint32_t passes;       /* sampling passes the query took part in */
} tm_query_info;

typedef struct {
    uint64_t submitted, completed, failed;
    uint64_t passes, samples;
    uint64_t weight_builds, weight_hits, evictions;
    uint64_t admission_waits;  /* queries that waited for memory to be admitted */
    uint64_t budget_bytes, resident_bytes, peak_bytes;
    uint64_t cached_sets;
    double build_ms;  /* worker time in weight builds */
    double pass_ms;   /* worker time in sampling passes */
    uint64_t pass_retries;  /* passes run again after the device ran out of memory */
} tm_server_stats;

/* Start a server on the current device.  opts may be NULL (defaults).
 * alloc: NULL (the library's block cache) or the allocator of the server's
 * weight sets and pass buffers (copied; see tm_allocator).
 * Errors: TM_EINVAL (budget below the pass reserve), TM_EDEVICE. */
int tm_server_create(uint64_t budget_bytes, const tm_server_opts* opts, const tm_allocator* alloc,
                     tm_server** out);
/* Register a built graph; it stays owned by the caller and must outlive the
 * server.  Its memory is not counted in the budget. */
int tm_server_add_graph(tm_server* srv, tm_graph* g, int32_t* gid);
/* Queue a query: k samples with the given seed of the motif on graph gid
 * (tr NULL: default tree).  Errors, at once: TM_EINVAL (bad graph id,
 * motif or tree), TM_EADMIT (its 64-bit weight set exceeds the budget). */
int tm_server_submit(tm_server* srv, int32_t gid, const tm_motif* mo, const tm_tree* tr, uint64_t k,
                     uint64_t seed, uint64_t* ticket);
/* Result of a finished query: returns its status (TM_OK or its error) and
 * forgets the ticket; TM_EAGAIN while it runs; TM_EINVAL for an unknown
 * ticket.  info may be NULL. */
int tm_server_poll(tm_server* srv, uint64_t ticket, tm_result* out, tm_query_info* info);
/* As tm_server_poll, blocking until the query finishes. */
int tm_server_wait(tm_server* srv, uint64_t ticket, tm_result* out, tm_query_info* info);
int tm_server_read_stats(tm_server* srv, tm_server_stats* out);
/* Stop the worker (queries not finished end with TM_ECANCELED) and free the
 * weight cache.  Waiting threads must have returned first. */
void tm_server_destroy(tm_server* srv);

/* ---- measurement --------------------------------------------------------
 * Device time of the library's stages, measured with HIP events recorded on
 * the caller's stream around each stage's kernels (no extra synchronisation:
 * the events are read when the call synchronises anyway). */
enum tm_stage {
    TM_STAGE_GRAPH = 0,    /* tm_graph_create: validation, sorts, lists */
    TM_STAGE_WEIGHTS = 1,  /* tm_weights_create: all levels, prefix tables, intervals */
    TM_STAGE_SAMPLE = 2,   /* the sampling kernel of tm_sample (draw, validate, complete) */
    TM_STAGE_REDUCE = 3,   /* the final reduction of tm_sample */
    TM_STAGE_ROOTS = 4,    /* tm_sample on large counts: root draws and their sort by root */
    TM_STAGE_LEVELS = 5,   /* each level kernel launch of a synchronous weight build (inside WEIGHTS) */
    TM_N_STAGES = 6
};
typedef struct {
    double ms[TM_N_STAGES];          /* accumulated device milliseconds */
    uint64_t launches[TM_N_STAGES];  /* timed stage executions */
} tm_profile;

/* Turn stage timing on (1) or off (0, the default); process-wide. */
void tm_profile_enable(int on);
/* Which stages are timed while timing is on: bit s for stage s (default all
 * of them; other bits are ignored).  Each timed stage records two events on
 * its stream; timing fewer stages leaves fewer of them between the kernels.
 * Process-wide. */
void tm_profile_stages(uint32_t mask);
/* Copy the accumulated times; reset = 1 clears them afterwards. */
int tm_profile_read(tm_profile* out, int reset);

/* Device memory.  Blocks the library releases are kept for its later
 * allocations on the current device (they go back to HIP by themselves only
 * when an allocation fails); this returns every such block to HIP now, after
 * a device synchronisation, so that other users of the device (a caching
 * allocator, a server budget taken from the free memory) see it.  Blocks
 * from a caller's tm_allocator are never kept.  Returns TM_OK. */
int tm_release_cached(void);

/* Bytes the sampling kernel's access model requests for samples j0 ..
 * j0 + count - 1 (a counting pass, not timed, same draws and the same kernel
 * variant as tm_sample with that count): every binary search over a range of
 * L entries is charged ceil(log2(L + 1)) reads of its element size, every
 * other read its element size; writes of records are not counted, nor is the
 * root-draw stage that large counts run first.  Used as the numerator of the
 * sampling kernel's roofline. */
int tm_sample_model_bytes(tm_weights* w, uint64_t seed, uint64_t j0, uint64_t count,
                          void* stream, uint64_t* bytes);

/* Bytes the level kernels of a weight build (Alg. 2: the s-weights of every
 * non-leaf tree edge, level by level) request under their access model: a
 * search over a list of L entries is charged ceil(log2 L) + 1 probes of
 * each of its six bounds (three over the T order, of the lists' time size:
 * 4 B when every shifted time is below 2^32 - 1, else 8 B; three 8 B keys
 * over the N order), every other read and write its element size (the edge, the
 * first pass's products, the children's prefix entries, the kept windows,
 * the products written).  The set is built as tm_weights_create_ex with
 * constraints TM_C_ALL builds it (a counting variant of the same kernels,
 * not timed) and then freed; a 64-bit build that overflows counts both
 * attempts, as the TM_STAGE_LEVELS timing does.  The numerator of the level
 * kernel's roofline.  Errors: as tm_weights_create. */
int tm_weights_model_bytes(tm_graph* g, const tm_motif* mo, const tm_tree* tr, void* stream,
                           uint64_t* bytes);

#ifdef __cplusplus
}
#endif
#endif
