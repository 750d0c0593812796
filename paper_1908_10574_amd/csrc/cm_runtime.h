// cm_runtime.h -- the context object behind the C ABI (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cm.h"
#include "cm_internal.h"

#include <exception>
#include <new>
#include <utility>
#include <vector>

namespace cmrt {

// A growable device allocation owned by a context.
struct DeviceBuf {
    void* ptr = nullptr;
    size_t cap = 0;
    bool ensure(size_t bytes);
    void release();
};

cm_status fail(cm_status s, const char* fmt, ...);
cm_status hip_fail(hipError_t e, const char* what);

// Test hook: when the environment variable CM_TEST_FAIL_ALLOC equals `site`
// ("host": a large host allocation of the ClusterMerge driver; "device":
// every growth of a context's device scratch), the allocation fails.
bool test_fail_alloc(const char* site);
// throws std::bad_alloc when test_fail_alloc("host") holds
void test_host_alloc_point();
cm_status check_matrix(const int32_t* matrix, int8_t* mat8);
cm_status check_gaps(int32_t go, int32_t ge);

// Optional HIP-event timing of every alignment-kernel launch, per pass.
struct KernelTimer {
    bool on = false;
    std::vector<hipEvent_t> pool;           // begin/end pairs
    std::vector<std::pair<int, int>> pending;   // (pass, pair index), in stream order
    size_t next = 0;
    double secs[3] = {0, 0, 0};
    int64_t launches[3] = {0, 0, 0};
};

}  // namespace cmrt

// Every extern "C" body runs inside CM_TRY ... CM_CATCH so that no C++
// exception crosses the ABI: a failed host allocation becomes CM_ENOMEM,
// anything else CM_EDEVICE, with the detail in cm_last_error().
#define CM_TRY try {
#define CM_CATCH                                                                          \
    }                                                                                     \
    catch (const std::bad_alloc&) {                                                       \
        return cmrt::fail(CM_ENOMEM, "host memory exhausted");                            \
    }                                                                                     \
    catch (const std::exception& ex_) {                                                   \
        return cmrt::fail(CM_EDEVICE, "internal error: %s", ex_.what());                  \
    }                                                                                     \
    catch (...) {                                                                         \
        return cmrt::fail(CM_EDEVICE, "internal error");                                  \
    }
#define CM_CATCH_VOID                                                                     \
    }                                                                                     \
    catch (...) {                                                                         \
    }

struct cm_context {
    int device = 0;
    int n_cu = 0;
    // launch plan per pass (score, score+end, span): kernel (packed 16-bit,
    // score pass only, or int32), rows-per-lane limit and persistent blocks per
    // CU; occ = occupancy limit per (pass, rmax choice), occ_pk per packed rmax
    // choice, occ_over of the int32 re-run of saturated packed pairs
    // packed: 0 int32 kernel, 1 two-profile packed kernel, 2 shared-query packed
    // kernel (items of one query, up to 32 rows per lane) with the rest on kind 1
    struct Plan { int packed = 0; int rmax = 16; int blocks_per_cu = 1; } plan[3];
    int occ[3][cmk::kNumRMax] = {};
    int occ_pk[cmk::kNumRMaxPk] = {};
    int occ_over = 1;
    int occ_pkq = 1;                    // shared-query packed kernel (plan kind 2, rmax 32)
    char arch[64] = {0};
    int runtime_version = 0;
    void* small = nullptr;              // counters, error flag, dummy bytes
    cmk::Counters* counters = nullptr;
    uint32_t* err_flag = nullptr;
    const uint8_t* dummy = nullptr;
    unsigned long long* cells_acc = nullptr;   // per pass: DP cells the alignment kernels computed
    cmrt::DeviceBuf keys, keys_alt, vals, vals_alt, sort_tmp;
    cmrt::DeviceBuf bnd;                // boundary rows between strips
    cmrt::DeviceBuf over;               // saturated pairs of the packed kernel
    cmrt::DeviceBuf q_start, q_len, q_flags, q_lists;   // shared-query plan scratch
    cmrt::DeviceBuf tb_meta, tb_offs, tb_dir, tb_rows;  // traceback scratch
    int32_t bnd_stride = 0;
    // buffers of the ClusterMerge driver and the screen (released with the context)
    cmrt::DeviceBuf drv[12];
    cmrt::KernelTimer timer;
    bool graphs = false;                // capture per-wave launch sequences in hipGraphs
    // the score pass of plan kind 2 runs its second list on this stream,
    // forked from and joined back into the caller's stream by the two events
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    void extra_release() {
        for (auto& b : drv) b.release();
        tb_meta.release();
        tb_offs.release();
        tb_dir.release();
        tb_rows.release();
    }
};

namespace cmrt {
// Scratch of one plan -> sort -> sweep pass on the int32 or the two-profile
// packed kernel (plan kinds 0 and 1): plan keys and values and their sorted
// copies (n_pairs each), the saturated-pair list (packed), the radix-sort
// temp and the counters block.
struct PassScratch {
    int packed = 0, rmax = 16, grid = 0;
    uint32_t* keys = nullptr;
    uint32_t* keys_alt = nullptr;
    int32_t* vals = nullptr;
    int32_t* vals_alt = nullptr;
    int32_t* over = nullptr;
    void* sort_tmp = nullptr;
    size_t sort_bytes = 0;
    cmk::Counters* ctr = nullptr;
    bool timed = false;
};
cm_status run_pass_scratch(cm_context* ctx, cmk::SwArgs& a, cmk::Pass pass, const PassScratch& ps, hipStream_t st);
size_t sort_temp_bytes(int64_t n);
// argument checks and SwArgs of a score / score+end batch (nothing enqueued)
cm_status score_args(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                     const int32_t* pairs, int64_t n_pairs, const int64_t* n_live, const int32_t* matrix,
                     int32_t gap_open, int32_t gap_extend, int32_t* scores, int32_t* end_a, int32_t* end_b,
                     cmk::SwArgs& a);
// the allocation-free entry point's per-device scratch address (set up once
// per device by cm_context_create)
cm_status noalloc_setup(int device);
// accumulate the durations of timed launches that have completed
// (blocking = wait for all of them)
void drain_timers(cm_context* ctx, bool blocking);
cm_status run_pass(cm_context* ctx, cmk::SwArgs& a, cmk::Pass pass, hipStream_t st);
cm_status load_plans(cm_context* ctx, const char* path);
cm_status reserve(cm_context* ctx, int64_t n);
// batch entry points with an optional device-resident live count (rows at or
// past *n_live are padding); the public C functions pass nullptr
cm_status score_batch(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                      const int32_t* pairs, int64_t n_pairs, const int64_t* n_live, const int32_t* matrix,
                      int32_t gap_open, int32_t gap_extend, int32_t* scores, int32_t* end_a, int32_t* end_b,
                      hipStream_t stream);
cm_status span_batch(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                     const int32_t* pairs, int64_t n_pairs, const int64_t* n_live, const int32_t* matrix,
                     int32_t gap_open, int32_t gap_extend, const int32_t* scores, const int32_t* end_a,
                     const int32_t* end_b, int32_t min_score, int32_t* start_a, int32_t* start_b,
                     hipStream_t stream);
cm_status save_plans(const cm_context* ctx, const char* path);
// occupancy limit of a plan (0 if the plan is not valid for the pass)
int plan_limit(const cm_context* ctx, int pass, int packed, int rmax);
// score+end of the pairs whose known score (scores[], kept) exceeds min_score;
// the others get end cell (-1, -1)
cm_status end_batch(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                    const int32_t* pairs, int64_t n_pairs, const int64_t* n_live, const int32_t* matrix,
                    int32_t gap_open, int32_t gap_extend, int32_t* scores, int32_t* end_a, int32_t* end_b,
                    int32_t min_score, hipStream_t stream);
}
