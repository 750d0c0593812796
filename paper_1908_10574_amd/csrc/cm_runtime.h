// cm_runtime.h -- the context object behind the C ABI (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cm.h"
#include "cm_internal.h"

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

struct cm_context {
    int device = 0;
    int n_cu = 0;
    int grid[3] = {0, 0, 0};            // persistent grid per pass (score, score+end, span)
    void* small = nullptr;              // counters, error flag, dummy bytes
    cmk::Counters* counters = nullptr;
    uint32_t* err_flag = nullptr;
    const uint8_t* dummy = nullptr;
    cmrt::DeviceBuf keys, keys_alt, vals, vals_alt, sort_tmp;
    cmrt::DeviceBuf bnd;                // boundary rows between strips
    int32_t bnd_stride = 0;
    // buffers of the ClusterMerge driver and the screen (released with the context)
    cmrt::DeviceBuf drv[12];
    cmrt::KernelTimer timer;
    void extra_release() {
        for (auto& b : drv) b.release();
    }
};

namespace cmrt {
// accumulate the durations of timed launches that have completed
// (blocking = wait for all of them)
void drain_timers(cm_context* ctx, bool blocking);
cm_status run_pass(cm_context* ctx, cmk::SwArgs& a, cmk::Pass pass, hipStream_t st);
}
