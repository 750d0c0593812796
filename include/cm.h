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
 *    (columns, index j).  Cells are 0-based and inclusive.
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
 *    the work.  Host pointers are read before the call returns.
 *  - Errors: no C++ exception crosses this ABI.  Argument errors found on the
 *    host are returned immediately and nothing is enqueued.  Data errors found
 *    on the device (residue code >= 20, sequence index out of range, sequence
 *    longer than CM_MAX_LEN, end cell outside its sequence) make the affected
 *    pairs score 0 with cells (-1,-1) and are reported by the next
 *    cm_context_sync() as CM_ERANGE.  cm_last_error() describes the last error
 *    of the calling thread.
 *  - A context is not thread-safe; use one per host thread.  Results never
 *    depend on the launch plan (bit-identical across plans and runs).
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
#define CM_ENOMEM       -3   /* device allocation failed */
#define CM_EDEVICE      -4   /* HIP runtime error (see cm_last_error) */
#define CM_EUNSUPPORTED -5   /* e.g. |matrix entry| > 127 */

#define CM_MAX_LEN 16384     /* longest sequence the alignment kernels accept */

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

#ifdef __cplusplus
}
#endif
#endif /* CM_H */
