// cm_internal.h -- structures shared by the HIP kernels and the host runtime
// of libcm.so.  Not part of the public ABI (that is include/cm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmk {

constexpr int kMaxLen = 65535;      // longest sequence (the plans' sort keys hold a column count in 16 bits)
constexpr int kGroup = 16;          // lanes that cooperate on one pair (one DPP row)
constexpr int kPairsPerWave = 4;    // 64-lane wavefront = 4 groups
constexpr int kRMax = 16;           // most query rows a lane can hold
constexpr int kNumRMax = 3;         // plan choices for the per-lane row limit
constexpr int kRMaxChoice[kNumRMax] = {8, 12, 16};
constexpr int kNRes = 21;           // 20 residues + sentinel
constexpr int kSent = 20;           // sentinel residue code (padding rows / columns)
// packed 16-bit score kernel: two pairs per group (one per 16-bit half of
// every register), eight pairs per wavefront
constexpr int kPairsPerWavePk = 8;
constexpr int kNumRMaxPk = 2;
constexpr int kRMaxChoicePk[kNumRMaxPk] = {4, 8};
// The packed kernels keep H, E, F and the best score plus kPkBias, so that
// H_diag + s is never negative and every value is a non-negative 16-bit
// integer that orders like a binary16 below 0x7C00 (maxima of three values are
// binary16 maximum3 operations).  A biased best of 0x7C00 or more (score of
// 0x7C00 - kPkBias = 31616 or more) may be inexact: the pair is rescored in int32.
constexpr int kPkBias = 128;        // covers the most negative profile byte, -128
constexpr int kPkSaturated = 0x7C00;
// shared-query packed kernel: the eight pairs of a wavefront share their query,
// so one LDS profile serves the wavefront and a lane can hold up to 32 rows
constexpr int kRMaxQ = 32;
constexpr int kMatStride = 24;      // bytes per row of the int8 matrix in LDS
// query-profile bytes per row slot: R rows padded to 4, 8 or 16 bytes
constexpr int prof_row_bytes(int r) { return r <= 4 ? 4 : (r <= 8 ? 8 : (r <= 16 ? 16 : 32)); }
// shared-query profile with 16-bit values (up to kR16Max rows per lane):
// 2 bytes per row, padded to 8
constexpr int kR16Max = 28;
constexpr int prof16_row_bytes(int r) { return 8 * ((2 * r + 7) / 8); }
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr uint32_t kSkipKey = 0xffffffffu;

// Error bits raised by kernels (reported by cm_context_sync).
constexpr uint32_t kErrResidue = 1u;     // residue code >= 20
constexpr uint32_t kErrIndex = 2u;       // pair index outside [0, n_seqs)
constexpr uint32_t kErrLength = 4u;      // sequence longer than CM_MAX_LEN
constexpr uint32_t kErrCell = 8u;        // span input end cell outside its sequence
constexpr uint32_t kErrPlan = 16u;       // internal: an item's pairs do not share the shape the plan promised
constexpr uint32_t kErrCapacity = 32u;   // traceback: a pair's share of the column buffer is too small
constexpr uint32_t kErrTrace = 64u;      // traceback: the box does not reproduce the pair's score

// Counters block in device memory.
struct Counters {
    int32_t n_work;      // pairs that need the DP (after the plan kernel)
    int32_t ticket;      // persistent-queue ticket
    int32_t n_over;      // pairs the packed kernel handed to the int32 kernel
    int32_t ticket_over; // ticket of the int32 re-run over those pairs
    int32_t n_sel[2];    // shared-query plan: pairs in full same-query items / the rest
    int32_t ticket_b;    // ticket of the second packed launch (the rest)
    int32_t pad[9];
};

struct SwArgs {
    const uint8_t* seqs;
    const int64_t* offsets;
    const int32_t* pairs;
    int64_t n_pairs;            // rows of the pair buffer
    const int64_t* n_live;      // nullable: rows at or past *n_live are padding (captured launches)
    int32_t n_seqs;
    int32_t go, ge;
    int32_t min_score;          // span pass: only pairs with score > min_score
    int32_t zero;               // always 0 (see the kernel's clamp)
    int32_t rmax;               // plan: most query rows per lane (8, 12 or 16; packed: 4 or 8)
    int32_t packed;             // score pass: run the packed 16-bit kernel
    int32_t end_filter;         // score+end pass: only pairs whose known score > min_score
    uint32_t go_pk, ge_pk;      // packed kernel: -gap_open, -gap_extend (capped at 65535) in both halves
    int32_t* over;              // packed kernel: indices of saturated pairs (capacity n_pairs)
    const int32_t* n_work_ptr;  // packed kernels: work count (null: ctr->n_work)
    int32_t* ticket;            // packed kernels: ticket counter (null: ctr->ticket)
    const uint32_t* keys;       // sorted plan keys (R, strips, columns)
    const int32_t* order;       // pair index per sorted position
    Counters* ctr;
    int32_t* scores;            // forward: output; span: input
    int32_t* end_a;             // forward: output (nullable); span: input
    int32_t* end_b;
    int32_t* start_a;           // span: output
    int32_t* start_b;
    int2* bnd;                  // boundary rows, one slot of bnd_stride per group
    int32_t bnd_stride;
    uint32_t* err;
    const uint8_t* dummy;       // >= 64 readable bytes (target of clamped prefetches)
    unsigned long long* cells_acc;   // nullable: running count of DP cells computed (padding and ramps included)
    int8_t mat[kNRes * kMatStride];   // M[row residue][column residue], sentinel -> -128
};

enum class Pass : int { Score = 0, ScoreEnd = 1, Span = 2 };

// Host launchers (sw_kernels.hip).
hipError_t launch_plan(const SwArgs& a, Pass pass, uint32_t* keys_out, int32_t* vals_out,
                       hipStream_t s);
hipError_t launch_sw(const SwArgs& a, Pass pass, int grid, hipStream_t s);   // uses a.rmax
int sw_blocks_per_cu(Pass pass, int rmax);
// packed score kernel followed by the int32 re-run of saturated pairs
hipError_t launch_sw_pk(const SwArgs& a, int grid, int grid_over, hipStream_t s);   // uses a.rmax
int sw_pk_blocks_per_cu(int rmax);
int sw_over_blocks_per_cu();
int sw_pkq_blocks_per_cu();

// Shared-query plan (score pass): 64-bit keys (rows-per-lane class, strips,
// query, columns), sorted; then every run of pairs with the same query is cut
// into full items of eight (list A, the shared-query kernel, when the item's
// subject lengths are close) and the rest (list B, the two-profile packed
// kernel, re-sorted by its own shape keys).
hipError_t launch_plan_q(const SwArgs& a, uint64_t* keys, int32_t* vals, hipStream_t s);
hipError_t launch_runs_q(const uint64_t* keys_sorted, int64_t n, const int32_t* n_work, int32_t* start_in,
                         hipStream_t s);
hipError_t launch_flags_q(const uint64_t* keys_sorted, const int32_t* start, int64_t n, const int32_t* n_work,
                          int32_t* run_len, uint8_t* flag_a, uint8_t* flag_b, hipStream_t s);
// two-profile shape keys (a.rmax) of the pairs of a list, skip keys past *count
hipError_t launch_keys_list(const SwArgs& a, const int32_t* list, const int32_t* count, int64_t n, uint32_t* keys,
                            hipStream_t s);
// list A on the shared-query kernel (stream s) and, concurrently, list B
// (sorted by its shape keys, boundary slots of its own) on the two-profile
// kernel (stream side, forked from and joined back into s by the two events),
// then the int32 re-run on s
hipError_t launch_sw_pkq(const SwArgs& a_list, const SwArgs& b_list, int grid, int grid_b, int grid_over,
                         hipStream_t s, hipStream_t side, hipEvent_t fork, hipEvent_t join);

}  // namespace cmk
