// cm_noalloc.hip -- cm_sw_score_batch_noalloc: the Smith-Waterman score batch
// without any allocation in the call, for callers that cannot allocate
// (code under stream capture, tight serving loops).
//
// The per-call scratch of a score pass (plan keys and values, their sorted
// copies, the saturated-pair list, the radix-sort temp and the counters
// block) lives in the file-scope device array `scratch` below, one copy per
// GPU for the life of the process.  In host code the array's name is only a
// stand-in: its device address is taken once per device by noalloc_setup()
// (called by cm_context_create with that device current) and that address is
// what the kernels receive.  The boundary rows between strips come from the
// context (allocated once when it is created).  Every call on one GPU shares
// the array, so calls that overlap on one GPU race; the counters are cleared
// by a kernel at the start of each call.
#include <hipcub/hipcub.hpp>

#include <mutex>

#include "../../include/cm.h"
#include "cm_internal.h"
#include "cm_runtime.h"

namespace {

constexpr int kMaxDevices = 64;
constexpr size_t kAlign = 256;
constexpr size_t kScratchBytes = static_cast<size_t>(CM_NOALLOC_SCRATCH_MIB) << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
cm_status g_setup[kMaxDevices] = {};        // setup status per device (CM_OK until a setup fails)

size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// scratch layout for CM_NOALLOC_MAX_PAIRS pairs
struct Layout {
    size_t ctr, keys, keys_alt, vals, vals_alt, over, sort, sort_bytes, end;
};

Layout layout() {
    const size_t n = static_cast<size_t>(CM_NOALLOC_MAX_PAIRS);
    Layout L{};
    L.ctr = 0;
    L.keys = up(L.ctr + sizeof(cmk::Counters));
    L.keys_alt = up(L.keys + 4 * n);
    L.vals = up(L.keys_alt + 4 * n);
    L.vals_alt = up(L.vals + 4 * n);
    L.over = up(L.vals_alt + 4 * n);
    L.sort = up(L.over + 4 * n);
    L.sort_bytes = cmrt::sort_temp_bytes(CM_NOALLOC_MAX_PAIRS);
    L.end = L.sort + L.sort_bytes;
    return L;
}

}  // namespace

namespace cmrt {

cm_status noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(CM_EINVAL, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[device]) return CM_OK;
    const size_t need = layout().end;
    if (need > kScratchBytes) {
        g_setup[device] = CM_EUNSUPPORTED;
        return fail(CM_EUNSUPPORTED, "allocation-free scratch layout (%zu bytes) exceeds the %zu-byte array", need,
                    kScratchBytes);
    }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        g_setup[device] = CM_EDEVICE;
        return hip_fail(e, "address of the allocation-free scratch");
    }
    g_ptr[device] = p;
    g_setup[device] = CM_OK;
    return CM_OK;
}

}  // namespace cmrt

extern "C" cm_status cm_sw_score_batch_noalloc(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets,
                                               int32_t n_seqs, const int32_t* pairs, int64_t n_pairs,
                                               const int32_t* matrix, int32_t gap_open, int32_t gap_extend,
                                               int32_t* scores, int32_t* end_a, int32_t* end_b, void* stream) {
    CM_TRY
    if (n_pairs > CM_NOALLOC_MAX_PAIRS)
        return cmrt::fail(CM_EINVAL, "%lld pairs exceed the allocation-free limit of %d per call",
                          static_cast<long long>(n_pairs), CM_NOALLOC_MAX_PAIRS);
    cmk::SwArgs a{};
    cm_status s = cmrt::score_args(ctx, seqs, offsets, n_seqs, pairs, n_pairs, nullptr, matrix, gap_open, gap_extend,
                                   scores, end_a, end_b, a);
    if (s != CM_OK || n_pairs == 0) return s;
    void* base = nullptr;
    cm_status setup = CM_EDEVICE;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (ctx->device >= 0 && ctx->device < kMaxDevices) {
            base = g_ptr[ctx->device];
            setup = g_setup[ctx->device];
        }
    }
    if (!base)
        return cmrt::fail(setup == CM_OK ? CM_EDEVICE : setup,
                          "allocation-free scratch unavailable on device %d (its setup when the context was created "
                          "failed)", ctx->device);
    const Layout L = layout();
    char* b = static_cast<char*>(base);
    const cmk::Pass pass = end_a ? cmk::Pass::ScoreEnd : cmk::Pass::Score;
    cmrt::PassScratch ps;
    // score only: the two-profile packed kernel (8 rows per lane); with end
    // cells: the int32 kernel (16 rows per lane); each at its occupancy limit
    if (pass == cmk::Pass::Score) {
        ps.packed = 1;
        ps.rmax = cmk::kRMaxChoicePk[cmk::kNumRMaxPk - 1];
        ps.grid = ctx->n_cu * ctx->occ_pk[cmk::kNumRMaxPk - 1];
    } else {
        ps.packed = 0;
        ps.rmax = cmk::kRMaxChoice[cmk::kNumRMax - 1];
        ps.grid = ctx->n_cu * ctx->occ[static_cast<int>(pass)][cmk::kNumRMax - 1];
    }
    ps.ctr = reinterpret_cast<cmk::Counters*>(b + L.ctr);
    ps.keys = reinterpret_cast<uint32_t*>(b + L.keys);
    ps.keys_alt = reinterpret_cast<uint32_t*>(b + L.keys_alt);
    ps.vals = reinterpret_cast<int32_t*>(b + L.vals);
    ps.vals_alt = reinterpret_cast<int32_t*>(b + L.vals_alt);
    ps.over = reinterpret_cast<int32_t*>(b + L.over);
    ps.sort_tmp = b + L.sort;
    ps.sort_bytes = L.sort_bytes;
    ps.timed = false;
    return cmrt::run_pass_scratch(ctx, a, pass, ps, static_cast<hipStream_t>(stream));
    CM_CATCH
}
