/*
 * TIMEST reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU implementation of the temporal
 * spanning-tree sampling estimator (TIMEST, arXiv 2507.20441), plus the
 * brute-force enumerators that pin it.  It exists to check the GPU library:
 * only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code with the GPU library.
 *
 * All counts and weights are exact unsigned 128-bit integers; any value that
 * would reach 2^128 makes the call return OR_EOVERFLOW.
 *
 * Semantics (where the paper leaves a choice, the reading taken is stated
 * here with the passage it rests on):
 *   - timestamps are shifted so the smallest is 0 (Sec. 4, storage paragraph);
 *   - the canonical edge id (eid) is the rank under the key (t, u, v);
 *   - intervals I_i = [i*delta, (i+2)*delta), i = 0 .. q-1, q = floor(T/delta)+1
 *     (Alg. 1 "Preprocess", Constraint 3 of Sec. 2.1);
 *   - s-weights per Def. "s-weight" and Claim "overall-num-matches";
 *   - the sampler is Alg. 3 "SampleSubg" with one Philox4x32-10 block per
 *     draw; counter = (j_lo, j_hi, draw, 0), key = (seed_lo, seed_hi);
 *   - validation and derivation are Alg. 4 / Alg. 5;
 *   - the estimate is Alg. 6:  C^ = W * acc2 / (2k),  acc2 = sum 2*M_phi/N_phi.
 */
#ifndef TIMEST_ORACLE_H
#define TIMEST_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    OR_OK = 0,
    OR_EINVAL = -1,
    OR_ESELFLOOP = -2,
    OR_EDUP = -3,
    OR_EOVERFLOW = -4,
    OR_ERANGE = -5,
};

typedef struct { uint64_t lo, hi; } or_u128;

typedef struct or_graph or_graph;
typedef struct or_prep or_prep;

/* Motif M = (H, pi, delta): l directed edges on vertices 0..k-1, listed in
 * pi order (edge p is the p-th in time).  Def. "temporal motif".
 *
 * Partial-order motifs (Sec. 1.1 remark and Sec. 6, "a partial order of time
 * constraints"): with partial = 1 only the pairs of the relation `before`
 * constrain the times -- bit p of before[q] says edge p is strictly earlier
 * than edge q -- taken with its transitive closure; other pairs may occur in
 * any order or at equal times.  The listing order must be a linear extension
 * (bits p < q only), and parallel motif edges must be ordered (so that the
 * edge map stays 1-1).  partial = 0 is the total order of the list. */
typedef struct {
    int32_t k;
    int32_t l;
    int32_t src[16];
    int32_t dst[16];
    int64_t delta;
    uint32_t partial;
    uint16_t before[16];
} or_motif;

/* Spanning tree S: n_edges = k-1 motif edge indices, and the center edge. */
typedef struct {
    int32_t n_edges;
    int32_t edge[8];
    int32_t center;
} or_tree;

/* std_error: the standard error of the estimate (the estimator's sample
 * standard deviation over sqrt(k), Sec. 4.4, Lemma "unbiased-estimate"):
 * (W / 2) * sqrt(D / (k^2 (k - 1))) with D = k * acc2_sq - acc2^2 formed
 * exactly in 256-bit integers and rounded once to double; 0 when k < 2, when
 * W = 0 or when acc2_sq saturated (flags bit 1). */
typedef struct {
    double estimate;
    double std_error;
    or_u128 W;
    or_u128 acc2;      /* sum over samples of 2*M_phi/N_phi */
    or_u128 acc2_sq;   /* sum of squares of the same terms (saturates, see flags) */
    uint64_t k;
    uint64_t n_valid, n_bad_vertex, n_bad_delta, n_bad_order, n_nonzero;
    int64_t q;
    uint32_t flags;    /* bit 0: W == 0;  bit 1: acc2_sq saturated */
} or_result;

/* One record per sample.  eid[j] is the edge matched to the j-th tree edge
 * when the tree edges are listed in increasing pi index. */
typedef struct {
    uint32_t interval;
    uint32_t status;   /* 0 valid, 1 vertex map not 1-1, 2 outside delta, 3 order */
    uint32_t n_phi;    /* 0 unless valid */
    uint32_t pad;
    int32_t eid[8];
    or_u128 m_phi;     /* 0 unless valid */
} or_rec;

/* ---- graph ---------------------------------------------------------- */
int or_graph_create(const int32_t* src, const int32_t* dst, const int64_t* t,
                    int64_t m, int32_t n, or_graph** out);
void or_graph_destroy(or_graph* g);
/* canonical (eid-ordered, time-shifted) edge arrays; any pointer may be NULL */
void or_graph_edges(const or_graph* g, int32_t* src, int32_t* dst, int64_t* t);
int64_t or_graph_shift(const or_graph* g);
/* eids of a vertex's out-list (dir=+1) or in-list (dir=-1), increasing eid;
 * returns the list length, writes at most cap entries */
int64_t or_graph_list(const or_graph* g, int32_t vertex, int dir, int32_t* eids, int64_t cap);

/* ---- motif planning ------------------------------------------------- */
/* Default spanning tree and center of a motif. */
int or_default_tree(const or_motif* mo, or_tree* out);

/* ---- choosing the tree (Alg. 7 / Alg. 8) ---------------------------- */
/* Every (spanning tree, center) pair, by looseness, then edge set, height,
 * center; at most max_out written, *n_out = their number. */
int or_tree_candidates(const or_motif* mo, or_tree* out, int64_t* looseness, int max_out, int* n_out);
/* W of the first n_c candidates (or_prepare each); the smallest wins. */
int or_choose_tree(const or_graph* g, const or_motif* mo, int n_c, or_tree* best, or_u128* W_out,
                   int* n_eval);

/* ---- preprocessing (Alg. 1 / Alg. 2) -------------------------------- */
int or_prepare(const or_graph* g, const or_motif* mo, const or_tree* tr, or_prep** out);
/* Constraint flags (Sec. "A Closer Look at Preprocessing"; Tab. "constraints"):
 * constraint 1 (order and delta between a tree edge and its parent) always;
 * OR_C_EXCLUDE adds constraint 2 (a child's far endpoint differs from the
 * parent's other endpoint); OR_C_WINDOWS adds constraint 3 (overlapping
 * 2 delta intervals; without it one interval spans all times, N_phi = 1). */
#define OR_C_EXCLUDE 1u
#define OR_C_WINDOWS 2u
#define OR_C_ALL 3u
int or_prepare_ex(const or_graph* g, const or_motif* mo, const or_tree* tr, uint32_t flags, or_prep** out);
void or_prep_destroy(or_prep* p);
or_u128 or_prep_W(const or_prep* p);
int64_t or_prep_q(const or_prep* p);
/* W_i for i = 0..q-1 */
void or_prep_interval_weights(const or_prep* p, or_u128* wi);
/* w_i(s,e) for tree edge s (motif edge index), every eid, and slot 0
 * (i = floor(t/delta)) or slot 1 (i = floor(t/delta) - 1; 0 where i < 0).
 * Leaf edges return 1 in every existing slot. */
int or_prep_weights(const or_prep* p, int32_t s, int slot, or_u128* out);

/* A preparation without weight tables: the plan, delta and the interval
 * count only.  For graphs too large for or_prepare; serves or_edge_weight
 * and or_derive_cnt (the table functions and or_sample need or_prepare). */
int or_prepare_light(const or_graph* g, const or_motif* mo, const or_tree* tr, or_prep** out);
int or_prepare_light_ex(const or_graph* g, const or_motif* mo, const or_tree* tr, uint32_t flags,
                        or_prep** out);
/* w_i(s,e) for one edge, evaluated from Claim "overall-num-matches" by
 * recursion over the candidate lists (no tables).  eid must lie in I_i.
 * OR_ERANGE when more than work_limit candidates would be visited. */
int or_edge_weight(const or_prep* p, int64_t interval, int32_t s, int32_t eid, uint64_t work_limit,
                   or_u128* w);

/* ---- sampling, validation, derivation, estimate (Alg. 3-6) ---------- */
/* Samples ids j0 .. j0+count-1 with the given seed; k_total is the k used in
 * the estimate formula.  recs may be NULL. */
int or_sample(const or_prep* p, uint64_t seed, uint64_t j0, uint64_t count,
              uint64_t k_total, or_result* res, or_rec* recs);
/* The std_error of a result with these sums (or_result's definition). */
double or_std_error(or_u128 W, or_u128 acc2, or_u128 acc2_sq, uint64_t k, uint32_t flags);
/* M_phi for a given image of the tree edges (eids indexed like or_rec.eid);
 * returns OR_EINVAL if the edges do not form a valid sample. */
int or_derive_cnt(const or_prep* p, const int32_t* eids, or_u128* m_phi);

/* The rank-th (0-based) completion of a valid tree image (eids like
 * or_derive_cnt), completions in lexicographic order of the eids of the
 * motif edges in pi order; out: l eids.  OR_EINVAL if the image is not
 * valid or rank >= M_phi. */
int or_list_instance(const or_prep* p, const int32_t* eids, or_u128 rank, int32_t* out);

/* ---- Philox4x32-10 and the range mapping ---------------------------- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* floor(X * n / 2^128) with X the 128-bit block of draw d of sample j */
or_u128 or_draw(uint64_t seed, uint64_t j, uint32_t d, or_u128 n);

/* ---- brute force (Def. "temporal match", Def. "partial match") ------ */
int or_brute_count(const or_graph* g, const or_motif* mo, or_u128* C);
/* sum over intervals i of the number of delta-partial matches of S in G_i */
int or_brute_tree_weight(const or_graph* g, const or_motif* mo, const or_tree* tr, or_u128* W);
int or_brute_tree_weight_ex(const or_graph* g, const or_motif* mo, const or_tree* tr, uint32_t flags,
                            or_u128* W);
/* number of partial matches in G_i of the subtree below tree edge s, with s
 * matched to edge eid (eid must lie in I_i) */
int or_brute_edge_weight(const or_graph* g, const or_motif* mo, const or_tree* tr,
                         int64_t interval, int32_t s, int32_t eid, or_u128* w);
/* Enumerate every partial match of S in G (each once, no interval
 * restriction).  For each one, writes the tree eids (8 per match, indexed like
 * or_rec.eid), its N_phi, its validation status and M_phi computed by brute
 * enumeration of completions.  Returns the number of partial matches, writes
 * at most cap of them. */
int64_t or_brute_partial_matches(const or_graph* g, const or_motif* mo, const or_tree* tr,
                                 int64_t cap, int32_t* eids, uint32_t* n_phi,
                                 uint32_t* status, or_u128* m_phi_brute);
int64_t or_brute_partial_matches_ex(const or_graph* g, const or_motif* mo, const or_tree* tr, uint32_t flags,
                                    int64_t cap, int32_t* eids, uint32_t* n_phi, uint32_t* status,
                                    or_u128* m_phi_brute);

#ifdef __cplusplus
}
#endif
#endif
