/*
 * cm.h -- C ABI of the MI355X ClusterMerge hot-path library (libcm.so).
 *
 * The library scores batches of protein pairs with Smith-Waterman local
 * alignment (affine gaps, 20x20 integer substitution matrix; the similarity
 * function f of Section 4 of Byma et al., "Parallel and Scalable Precise
 * Clustering for Homologous Protein Discovery") and runs ClusterMerge
 * (Algorithms 1 and 2, Section 3) on top of it.
 *
 * Conventions shared by every entry point:
 *  - Residues are bytes 0..19 over ACDEFGHIKLMNPQRSTVWY, concatenated; sequence
 *    k is residues[offsets[k] .. offsets[k+1]) (int64 offsets, n_seqs+1 of them).
 *    A sequence is referred to by its int32 index.  Empty sequences are legal.
 *  - A pair row (a, b) aligns sequence a (rows, index i) with sequence b
 *    (columns, index j).  Cells are 0-based and inclusive.  One call of the
 *    Smith-Waterman batch entry points (score, span, columns, autotune) takes
 *    at most 2^31 - 1 pairs (CM_EINVAL beyond).
 *  - The matrix is 400 int32 values, row-major, M[x][y] = score of residue x
 *    (row sequence) against residue y (column sequence); |M| <= 127.
 *  - Gap arguments are negative as written: a run of k gap columns of one kind
 *    scores gap_open + (k-1)*gap_extend.  Required: gap_open <= gap_extend <= 0
 *    and gap_open < 0.
 *  - Score S = max(0, best local alignment score).  End cell = first cell in
 *    row-major order (smallest i, then smallest j) whose Gotoh H value is S;
 *    start cell = the lexicographically largest start among optimal alignments
 *    ending there.  Both are (-1,-1) when S == 0.
 *  - Pointers documented as "device" are caller-owned device memory; calls
 *    enqueue work on `stream` (a hipStream_t, NULL = the null stream) and return
 *    without waiting.  The caller keeps buffers alive until the stream reaches
 *    the work.  Host pointers are read before the call returns.  Part of a
 *    score pass may run on a stream of the context, forked from and joined
 *    back into `stream` by events, so the call stays ordered on `stream`.  A
 *    context's scratch serves one call at a time: calls on different streams
 *    with one context must be ordered by the caller (or use one context each).
 *  - Errors: no C++ exception crosses this ABI (a failed host allocation
 *    inside the library returns CM_ENOMEM, any other internal exception
 *    CM_EDEVICE; the context stays usable).  Argument errors found on the
 *    host are returned immediately and nothing is enqueued.  Data errors found
 *    on the device (residue code >= 20, sequence index out of range, sequence
 *    longer than CM_MAX_LEN, end cell outside its sequence) make the affected
 *    pairs score 0 with cells (-1,-1) and are reported by the next
 *    cm_context_sync() as CM_ERANGE.  cm_last_error() describes the last error
 *    of the calling thread.
 *  - A context is not thread-safe; use one per host thread.  Results never
 *    depend on the launch plan (bit-identical across plans and runs).
 *  - Test hook: with the environment variable CM_TEST_FAIL_ALLOC=device every
 *    growth of a context's device scratch fails (CM_ENOMEM); with
 *    CM_TEST_FAIL_ALLOC=host the ClusterMerge driver's final stage fails a
 *    host allocation while a batch is on the device (CM_ENOMEM).  The variable
 *    is read at each allocation, so unsetting it restores normal operation.
 */
#ifndef CM_H
#define CM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cm_status;
#define CM_OK            0
#define CM_EINVAL       -1   /* bad scalar argument, NULL pointer, gap signs */
#define CM_ERANGE       -2   /* residue >= 20, index >= n_seqs, length > CM_MAX_LEN */
#define CM_ENOMEM       -3   /* device or host allocation failed */
#define CM_EDEVICE      -4   /* HIP runtime error (see cm_last_error) */
#define CM_EUNSUPPORTED -5   /* e.g. |matrix entry| > 127 */

#define CM_MAX_LEN 65535     /* longest sequence the alignment kernels accept */

const char* cm_status_str(cm_status s);
const char* cm_last_error(void);

typedef struct cm_context cm_context;

/* Create a context on HIP device `device_ordinal`; owns device scratch
 * (sort buffers, boundary rows, work counters) grown on demand. */
cm_status cm_context_create(int device_ordinal, cm_context** out);
void      cm_context_destroy(cm_context* ctx);
/* Wait for all work the context enqueued; returns CM_ERANGE if a kernel
 * flagged bad input data since the previous sync (and clears the flag). */
cm_status cm_context_sync(cm_context* ctx);

/* Timing of the alignment kernels (not of plan/sort/copies): when on, every
 * launch is bracketed by HIP events on its stream; cm_context_kernel_time
 * waits for outstanding launches and returns the running totals for `pass`
 * (CM_PASS_*): number of launches and summed device seconds. */
#define CM_PASS_SCORE     0
#define CM_PASS_SCORE_END 1
#define CM_PASS_SPAN      2
cm_status cm_context_set_timing(cm_context* ctx, int on);
/* When on, cm_clustermerge_run replays each GPU wave as a captured hipGraph
 * (one per power-of-two capacity; the live pair count is read from device
 * memory); alignment-kernel timing is then not collected.  Off by default. */
cm_status cm_context_set_graphs(cm_context* ctx, int on);
cm_status cm_context_kernel_time(cm_context* ctx, int pass, int64_t* launches, double* seconds);
/* DP cells the alignment kernels of `pass` computed in the context's timed
 * launches so far (running total; waits for the device): every lane-row of
 * every column step of every strip, so ramps, padded rows and columns beyond
 * a shorter pair's end are included.  Divided by the pairs' m * n it is the
 * kernels' padding overhead. */
cm_status cm_context_cells_computed(cm_context* ctx, int pass, double* cells);

/* Measured peak rate of one VALU instruction of the cell update (the
 * denominators of the alignment kernels' roofline): every lane of 8
 * wavefronts per SIMD runs 32 independent chains of the instruction;
 * *ops_per_second counts 16-bit halves of packed instructions as two
 * operations; *clock_hz (nullable) is the shader clock over the run (cycle
 * counter against the real-time counter).  Synchronous, about 0.1 s. */
#define CM_PROBE_I32_ADD   0   /* v_add_u32 */
#define CM_PROBE_I32_MAX3  1   /* v_max3_i32 */
#define CM_PROBE_PK16_ADD  2   /* v_pk_add_u16 */
#define CM_PROBE_PK16_MAX3 3   /* v_pk_maximum3_f16 */
cm_status cm_probe_valu(cm_context* ctx, int kind, double* ops_per_second, double* clock_hz);

/* Launch plan of the alignment kernels, per pass: the kernel (packed = 2: the
 * score pass groups pairs by query and runs items of eight pairs sharing one
 * query on the shared-query packed 16-bit kernel (up to 32 rows per lane),
 * the rest on the two-profile packed kernel; packed = 1: the two-profile
 * packed 16-bit kernel for every pair (two pairs per register); packed = 0: the
 * int32 kernel.  Packed plans serve the score pass only, and pairs whose
 * packed score reaches 31616 are recomputed by the int32 kernel), the most
 * query rows a lane holds (int32: 8, 12 or 16; packed: 4 or 8; shared-query:
 * 32; strips are 16 x that many rows) and the persistent blocks per CU (1 ..
 * occupancy limit).  Results never depend on the plan.  A context starts from
 * (2, 32, occupancy limit) for the score pass and (0, 16, occupancy limit) for
 * the others and, when the environment variable CM_AUTOTUNE_CACHE names a plan
 * file written by cm_plan_save for the same GPU architecture and HIP runtime,
 * from the plans recorded there (a missing, foreign or corrupt file is
 * ignored).  cm_plan_set fails with CM_EINVAL on a plan that is not valid for
 * the pass. */
cm_status cm_plan_get(const cm_context* ctx, int pass, int32_t* packed, int32_t* rmax, int32_t* blocks_per_cu,
                      int32_t* max_blocks_per_cu);
cm_status cm_plan_set(cm_context* ctx, int pass, int32_t packed, int32_t rmax, int32_t blocks_per_cu);
cm_status cm_plan_save(const cm_context* ctx, const char* path);
cm_status cm_plan_load(cm_context* ctx, const char* path);
/* Autotuner: times every candidate plan of `pass` (CM_PASS_SCORE or
 * CM_PASS_SCORE_END) on the given pair sample (device pointers as in
 * cm_sw_score_batch), fails with CM_EDEVICE if two candidates disagree on any
 * output, and keeps the fastest.  table (host, nullable) receives up to 32 rows
 * of (packed, rmax, blocks_per_cu, milliseconds); *n_rows their count.
 * Synchronous. */
cm_status cm_autotune(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                      const int32_t* pairs, int64_t n_pairs, const int32_t* matrix, int32_t gap_open,
                      int32_t gap_extend, int pass, double* table, int32_t* n_rows);

/* Smith-Waterman scores of a batch of pairs (Section 4: f(i, j) is the local
 * alignment score; Section 6.1: the similar-pair test).
 *   seqs     device u8 [offsets[n_seqs]]          residue codes
 *   offsets  device i64 [n_seqs+1]
 *   pairs    device i32 [n_pairs][2]             (a, b) = (rows, columns)
 *   matrix   host   i32 [400]
 *   scores   device i32 [n_pairs]                output
 *   end_a, end_b  device i32 [n_pairs] or both NULL: end cell (output)
 * Score-only calls (end_a == end_b == NULL) run a cheaper kernel. */
cm_status cm_sw_score_batch(cm_context* ctx,
                            const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                            const int32_t* pairs, int64_t n_pairs,
                            const int32_t* matrix, int32_t gap_open, int32_t gap_extend,
                            int32_t* scores, int32_t* end_a, int32_t* end_b,
                            void* stream);

/* For callers that cannot allocate (code under HIP stream capture, tight
 * serving loops, harnesses that forbid allocation): cm_sw_score_batch with
 * the same arguments, outputs and errors, bit-identical results, and no
 * allocation of any kind in the call.  Its per-call scratch (plan keys and
 * values, sorted copies, saturated-pair list, sort temp, counters) is a
 * static device array of CM_NOALLOC_SCRATCH_MIB MiB that the library holds on
 * every GPU it runs on until the process ends (its address is taken when a
 * context is created on that GPU); the boundary rows between strips are the
 * context's, allocated when it is created.  At most CM_NOALLOC_MAX_PAIRS
 * pairs per call (CM_EINVAL beyond, nothing enqueued).  All calls on one GPU
 * share the array: calls that overlap on one GPU (two streams, two contexts,
 * two host threads) race and must be ordered by the caller.  Score-only calls
 * run the two-profile packed kernel, score+end calls the int32 kernel, each
 * at its occupancy limit; the context's plans and timing are not used. */
#define CM_NOALLOC_MAX_PAIRS   1048576
#define CM_NOALLOC_SCRATCH_MIB 48
cm_status cm_sw_score_batch_noalloc(cm_context* ctx,
                                    const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                                    const int32_t* pairs, int64_t n_pairs,
                                    const int32_t* matrix, int32_t gap_open, int32_t gap_extend,
                                    int32_t* scores, int32_t* end_a, int32_t* end_b,
                                    void* stream);

/* Start cells of the optimal local alignments (needed by the coverage test of
 * the protein transitivity function, Section 4): for every pair whose score
 * (input, from cm_sw_score_batch) exceeds min_score, the same recurrence is run
 * on the reversed prefixes ending at (end_a, end_b) (inputs); start_a/start_b
 * (device i32 [n_pairs], outputs) receive the start cell, or (-1,-1) for pairs
 * at or below min_score. */
cm_status cm_sw_span_batch(cm_context* ctx,
                           const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                           const int32_t* pairs, int64_t n_pairs,
                           const int32_t* matrix, int32_t gap_open, int32_t gap_extend,
                           const int32_t* scores, const int32_t* end_a, const int32_t* end_b,
                           int32_t min_score, int32_t* start_a, int32_t* start_b,
                           void* stream);

/* Alignment columns of found pairs (the final stage records scores; the
 * alignments themselves are left to later analysis, Section 6.1): for every
 * pair with score > 0 (inputs as written by cm_sw_score_batch and
 * cm_sw_span_batch: score, end cell, start cell; device i32 [n_pairs] each),
 * the optimal local alignment between its start and end cells, as the Gotoh
 * global alignment of a[start_a..end_a] with b[start_b..end_b] that begins
 * and ends with an aligned pair (it scores exactly the pair's score).  Where
 * several such alignments tie, the walk back from the end prefers an aligned
 * pair, then the gap kind it is in, then the other kind.  Columns are written
 * start to end to ops[op_offsets[p] ..] as bytes 'M' (aligned pair), 'I'
 * (a residue of a against a gap) and 'D' (a gap against a residue of b), and
 * their number to n_ops[p] (0 when the score is 0, -1 when the pair was
 * rejected).  op_offsets (device i64 [n_pairs + 1], caller-computed) must give
 * every pair with score > 0 at least (end_a - start_a + 1) + (end_b - start_b
 * + 1) bytes.  The call waits for its work on `stream` (scratch of one byte per
 * box cell, bounded per launch: boxes of up to 2^28 cells, e.g. 16384 x 16384;
 * pairs are grouped 64 to a wavefront by box shape, and a wavefront whose
 * largest rows x columns exceed 2^28 makes the call return CM_EUNSUPPORTED
 * before anything is launched).  Bad indices, cells or capacities make the
 * pair's n_ops -1 and are reported by cm_context_sync as CM_ERANGE. */
cm_status cm_sw_traceback_batch(cm_context* ctx,
                                const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                                const int32_t* pairs, int64_t n_pairs,
                                const int32_t* matrix, int32_t gap_open, int32_t gap_extend,
                                const int32_t* scores, const int32_t* end_a, const int32_t* end_b,
                                const int32_t* start_a, const int32_t* start_b,
                                const int64_t* op_offsets, uint8_t* ops, int32_t* n_ops, void* stream);


/* ---------------------------------------------------------------------------
 * ClusterMerge (Algorithm 2 "BottomUpMerge" over Algorithm 1 "Cluster Set
 * Merge", Section 3; protein similarity and transitivity of Section 4; final
 * in-cluster all-against-all of Section 6.1).
 *
 * The result equals the plain sequential algorithm: elements 0..n-1 start as
 * one-cluster sets in a FIFO queue; two sets are popped, merged, the result
 * pushed back, until one set remains.  Within a merge, clusters of the first
 * set are compared in order with the not-yet-merged clusters of the second:
 * representatives similar (score >= T) and transitive one way fully merge
 * (the absorbed members are appended in order, skipping duplicates; the
 * second set's cluster is tested as absorber first), otherwise the two
 * clusters exchange the members similar to the other representative.
 * Transitivity of representative r over representative q: score > mT and
 * fewer than mU residues of q lie outside the optimal local alignment (both
 * flanks).  Representative alignments are oriented (cluster of the first set
 * = rows, cluster of the second set = columns).  Merges of one tree level are
 * scored together on the GPU; the replay on the host is exactly sequential.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t matrix[400];
    int32_t gap_open, gap_extend;   /* e.g. -11, -1 */
    int32_t T;                      /* similar pair: score >= T (e.g. 120) */
    int32_t mT;                     /* full merge needs score > mT (e.g. 166) */
    int32_t mU;                     /* and uncovered residues < mU (e.g. 15) */
    uint32_t screen_stages;         /* CM_STAGE_* bits screened when a screen is given */
    float screen_tau;               /* keep a candidate pair iff logit >= screen_tau */
    int64_t max_result_pairs;       /* keep at most this many similar pairs in the result
                                       (counts and the set hash always cover all) */
    int64_t screen_min_product;     /* when > 0: representative pairs whose clusters' member
                                       counts (at the start of the merge) multiply to at least
                                       this are aligned without consulting the screen */
    int64_t rep_chunk_pairs;        /* representative pairs of a level are aligned in column
                                       chunks of about this many pairs (at most 8 chunks), a row
                                       leaving Algorithm 1's loop is not aligned against later
                                       chunks; 0 = about 2^25, < 0 = one batch per level.  Not
                                       used while a screen covers CM_STAGE_REP under graph
                                       capture.  Results do not depend on it. */
    int64_t record_candidates;      /* 1: the result keeps every pair scored during the merge stage
                                       (representative and exchange alignments, speculative ones
                                       included) with its score (cm_result_candidates); 0: not kept */
} cm_params;

#define CM_STAGE_REP       1u       /* representative vs representative */
#define CM_STAGE_EXCHANGE  2u       /* member vs other representative */
#define CM_STAGE_FINAL     4u       /* in-cluster all-against-all */

typedef struct {
    int64_t rep_comparisons;        /* f(rep1, rep2) evaluations of Algorithm 1 */
    int64_t exchange_alignments;    /* member-vs-representative tests required */
    int64_t full_merges, exchanges;
    int64_t rounds, waves;          /* tree levels; GPU batches */
    int64_t aligned_pairs;          /* pairs aligned on the GPU, all stages */
    double  aligned_cells;          /* sum of m*n over them */
    int64_t speculative_pairs;      /* aligned but not needed by the replay */
    int64_t cache_hits;
    int64_t screened_out;           /* candidate pairs dropped by the screen */
    int64_t n_clusters;
    int64_t final_candidates;       /* unique in-cluster pairs of the final stage */
    int64_t n_similar_pairs;        /* pairs reported (score >= T) */
    uint64_t pair_set_hash;         /* order-independent hash of the reported (x, y, score) */
    double  t_total_s, t_merge_s, t_final_s, t_gpu_s, t_host_s;
    int64_t sw_launches;            /* score-kernel launches (timed; every aligned pair) */
    double  sw_kernel_s;            /* their summed device time; aligned_cells / sw_kernel_s
                                       is the score kernel's cell rate */
    double  end_kernel_s;           /* device time of the end-cell and start-cell kernels, which
                                       realign the representative pairs scoring above mT */
    int64_t end_pairs;              /* pairs realigned for end and start cells */
    double  t_screen_s;             /* wall time of screen inference calls */
    int64_t screened_pairs;         /* candidate pairs the screen evaluated */
    double  required_cells;         /* sum of m*n over the comparisons Algorithm 1 makes (representative
                                       pairs it compares, member-vs-representative tests of its
                                       exchanges) and the final stage's pairs not already scored: the
                                       cells the method needs, without speculative or cached work */
} cm_stats;

typedef struct cm_result cm_result;
typedef struct cm_screen cm_screen;

/* Run ClusterMerge on a device-resident sequence store (seqs, offsets: device
 * pointers as in cm_sw_score_batch).  Synchronous.  `screen` may be NULL
 * (plain method).  *out is library-owned; free it with cm_result_free.
 * Similarity (score >= T) is a property of the unordered pair (Algorithm 1
 * compares clusters both ways), so the matrix must be symmetric (CM_EINVAL
 * otherwise); the driver keeps one score per pair and aligns each pair in the
 * orientation that batches best. */
cm_status cm_clustermerge_run(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets,
                              int32_t n_seqs, const cm_params* params, const cm_screen* screen,
                              cm_result** out);
/* Classify new proteins against an existing clustering (the paper's
 * Conclusion: new sequences classified against the clusters already formed;
 * the procedure is this library's reading).  Elements 0..n_prev-1 of the
 * store are clustered by the previous result, given as host arrays in the
 * layout of cm_result_clusters (n_clusters clusters; cluster c has
 * representative reps[c] and members members[member_offsets[c] ..
 * member_offsets[c+1]), each previous element in at least one cluster, the
 * representative among the members, no member twice in a cluster).  The new
 * elements n_prev..n_seqs-1 are clustered among themselves with Algorithm 2;
 * that set is merged into the previous set with one Algorithm 1 merge (the
 * previous set first); the final stage then runs over all resulting clusters.
 * known_pairs / known_scores (host, n_known rows, e.g. the previous result's
 * similar pairs) are scores already computed: they are reused, not realigned.
 * Same parameters, screen and result as cm_clustermerge_run; the statistics
 * count the new work.  CM_EINVAL for an inconsistent previous clustering. */
cm_status cm_clustermerge_extend(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets,
                                 int32_t n_seqs, const cm_params* params, const cm_screen* screen,
                                 int32_t n_prev, int32_t n_clusters, const int32_t* reps,
                                 const int64_t* member_offsets, const int32_t* members,
                                 int64_t n_known, const int32_t* known_pairs,
                                 const int32_t* known_scores, cm_result** out);
/* Final clusters in final-set order; members of cluster k are
 * members[member_offsets[k] .. member_offsets[k+1]) in cluster order. */
cm_status cm_result_clusters(const cm_result* r, int32_t* n_clusters, const int32_t** reps,
                             const int64_t** member_offsets, const int32_t** members);
/* Similar pairs (x < y, score >= T), sorted by (x, y); pairs/scores are
 * NULL-free arrays of *n_pairs rows (possibly truncated to max_result_pairs). */
cm_status cm_result_pairs(const cm_result* r, int64_t* n_pairs, const int32_t** pairs,
                          const int32_t** scores);
/* Pairs (x < y) scored during the merge stage, sorted, with their scores,
 * when the run was made with params.record_candidates = 1 (else none): the
 * candidates the screen decides on, e.g. for calibrating its threshold. */
cm_status cm_result_candidates(const cm_result* r, int64_t* n_pairs, const int32_t** pairs,
                               const int32_t** scores);
cm_status cm_result_stats(const cm_result* r, cm_stats* out);
void      cm_result_free(cm_result* r);

/* Number of pairs (x < y) of the whole store with score >= T: the all-vs-all
 * ground truth against which ClusterMerge recall is measured (Section 6.1).
 * Synchronous; pairs are generated on the device in triangle tiles. */
cm_status cm_allvsall_count(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets,
                            int32_t n_seqs, const int32_t* matrix, int32_t gap_open,
                            int32_t gap_extend, int32_t T, int64_t* count, double* cells);


/* ---------------------------------------------------------------------------
 * Learned pair screen (not in the paper: a pre-filter in front of the exact
 * similarity function of Section 4).  A candidate pair is aligned only if the
 * screen's logit is >= tau; the alignment score still decides similarity.
 *
 * Features: per protein, counts of its 3-mers (code = 400 a_p + 20 a_{p+1} +
 * a_{p+2}) hashed into 1024 buckets (top 10 bits of code * 2654435761 mod
 * 2^32), divided by 8, stored as bf16 bit patterns [n_seqs][1024].
 * Network: x = [|f_a - f_b|, f_a * f_b] (2048, bf16), z = W3 relu(W2 relu(W1 x
 * + b1) + b2) + b3 with W1 512x2048, W2 512x512, W3 1x512 in bf16 on MFMA,
 * fp32 accumulation, hidden activations rounded to bf16.  Training: mean
 * binary cross-entropy on logits, Adam (beta 0.9/0.999, eps 1e-8) on fp32
 * master weights.  The fp32 master vector is W1, b1, W2, b2, W3, b3
 * (cm_screen_num_params() values, row-major).
 * ------------------------------------------------------------------------- */
cm_status cm_kmer_features(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                           uint16_t* feat /* device [n_seqs][1024] */, void* stream);
int64_t   cm_screen_num_params(void);
/* New screen with Kaiming-uniform weights drawn from `seed`, zero biases. */
cm_status cm_screen_create(cm_context* ctx, uint64_t seed, cm_screen** out);
void      cm_screen_destroy(cm_screen* s);
cm_status cm_screen_set_weights(cm_screen* s, const float* host_fp32_master);   /* also resets Adam */
/* host_bf16 (nullable) receives the bf16 W1, W2, W3 the network uses, concatenated. */
cm_status cm_screen_get_weights(const cm_screen* s, float* host_fp32_master, uint16_t* host_bf16);
/* Logits of pair rows (device i32 [n][2]) into device fp32 [n]; enqueued on stream. */
cm_status cm_screen_infer(const cm_screen* s, const uint16_t* feat, const int32_t* pairs, int64_t n_pairs,
                          float* logits, void* stream);
/* Synchronous: gradients of the mean loss over the batch (labels device u8 [n],
 * 1 = similar) into host fp32 [num_params]; loss (host, nullable). n <= 2^20. */
cm_status cm_screen_grads(cm_screen* s, const uint16_t* feat, const int32_t* pairs, const uint8_t* labels,
                          int64_t n_pairs, float* host_grads, float* loss);
/* A training run (the learned screen's training on GPU-Smith-Waterman labels):
 * epochs passes over the n_pairs rows; each epoch visits them in an order
 * drawn from `seed` (Fisher-Yates over a splitmix64 stream seeded from the
 * seed and the epoch number) or, with shuffle = 0, in the given order; every
 * `batch` consecutive rows of that order make one Adam step (lr; beta 0.9 /
 * 0.999, eps 1e-8), and a last partial batch is a smaller step unless
 * drop_last = 1 skips it. */
typedef struct {
    int32_t epochs;       /* >= 1 */
    int32_t batch;        /* pairs per step, 1 .. 2^20 */
    float lr;             /* > 0 */
    int32_t shuffle;      /* 0 or 1 */
    uint64_t seed;
    int32_t drop_last;    /* 0 or 1 */
} cm_train_cfg;
/* Number of steps (= loss-log entries) a training run makes; -1 for a bad config. */
int64_t   cm_screen_train_steps(int64_t n_pairs, const cm_train_cfg* cfg);
/* Run the whole training on the device (features as from cm_kmer_features,
 * pairs device i32 [n_pairs][2], labels device u8 [n_pairs], 1 = similar):
 * every step's gather, forward, backward, loss and Adam update are enqueued
 * back to back on the screen's stream, with no host round trip between steps.
 * loss_log (host, nullable, cm_screen_train_steps() floats) receives every
 * step's mean loss before its update.  Synchronous: returns when the run is
 * done.  Equivalent, bit for bit, to cm_screen_train_step over the same
 * batches.  CM_EINVAL for a bad config or n_pairs outside [1, 2^31 - 1]. */
cm_status cm_screen_train(cm_screen* s, const uint16_t* feat, const int32_t* pairs, const uint8_t* labels,
                          int64_t n_pairs, const cm_train_cfg* cfg, float* loss_log);
/* Synchronous: one Adam step on the batch; loss (host, nullable) is the batch's
 * mean loss before the update. */
cm_status cm_screen_train_step(cm_screen* s, const uint16_t* feat, const int32_t* pairs, const uint8_t* labels,
                               int64_t n_pairs, float lr, float* loss);
cm_status cm_screen_save(const cm_screen* s, const char* path);       /* weights + Adam state */
cm_status cm_screen_load(cm_context* ctx, const char* path, cm_screen** out);

#ifdef __cplusplus
}
#endif
#endif /* CM_H */
