// cm_tune.hip -- autotuner for the alignment launch plan.
//
// A plan is (kernel, rows-per-lane limit, persistent blocks per CU); the score
// pass can run the packed 16-bit kernel or the int32 kernel.  The limit trades
// LDS footprint and occupancy against strip count: 8 rows per lane keeps two
// times more wavefronts resident but splits queries longer than 128 residues
// into more strips (more ramp steps, more boundary traffic); 16 does the
// opposite.  The tuner times every candidate on a caller-supplied sample of
// the workload, checks that every candidate returns bit-identical results,
// and keeps the fastest for that pass.
#include <cstring>
#include <vector>

#include "../../include/cm.h"
#include "cm_internal.h"
#include "cm_runtime.h"

using cmrt::fail;
using cmrt::hip_fail;

extern "C" cm_status cm_autotune(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                                 const int32_t* pairs, int64_t n_pairs, const int32_t* matrix, int32_t gap_open,
                                 int32_t gap_extend, int pass, double* table, int32_t* n_rows) {
    CM_TRY
    if (!ctx || !pairs || n_pairs <= 0 || (pass != CM_PASS_SCORE && pass != CM_PASS_SCORE_END))
        return fail(CM_EINVAL, "bad argument");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(CM_EDEVICE, "hipSetDevice");
    const cm_context::Plan saved = ctx->plan[pass];
    const bool with_end = pass == CM_PASS_SCORE_END;
    constexpr int kMaxRows = 32;
    int32_t* d = nullptr;
    hipError_t e = hipMalloc(&d, static_cast<size_t>(n_pairs) * 12);
    if (e != hipSuccess) return hip_fail(e, "tuner buffers");
    int32_t* sc = d;
    int32_t* ea = d + n_pairs;
    int32_t* eb = d + 2 * n_pairs;
    hipEvent_t t0, t1;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    std::vector<int32_t> ref, cur;
    double best_ms = 1e300;
    cm_context::Plan best = saved;
    int rows = 0;
    cm_status st = CM_OK;
    // candidates: (kernel, rows-per-lane limit); the packed kernel serves the score pass only
    struct Cand { int packed, rmax; };
    std::vector<Cand> cands;
    if (pass == CM_PASS_SCORE) {
        cands.push_back({2, cmk::kRMaxQ});
        for (int k = 0; k < cmk::kNumRMaxPk; ++k) cands.push_back({1, cmk::kRMaxChoicePk[k]});
    }
    for (int k = 0; k < cmk::kNumRMax; ++k) cands.push_back({0, cmk::kRMaxChoice[k]});
    for (const Cand& cd : cands) {
        if (st != CM_OK) break;
        const int occ = cmrt::plan_limit(ctx, pass, cd.packed, cd.rmax);
        int bpcs[3] = {occ, (occ * 3) / 4, occ / 2};
        for (int c = 0; c < 3 && st == CM_OK; ++c) {
            const int bpc = bpcs[c];
            if (bpc < 1 || (c > 0 && bpc == bpcs[c - 1]) || (c > 1 && bpc == bpcs[c - 2])) continue;
            ctx->plan[pass].packed = cd.packed;
            ctx->plan[pass].rmax = cd.rmax;
            ctx->plan[pass].blocks_per_cu = bpc;
            double ms = 1e300;
            for (int rep = 0; rep < 3 && st == CM_OK; ++rep) {
                (void)hipEventRecord(t0, nullptr);
                st = cm_sw_score_batch(ctx, seqs, offsets, n_seqs, pairs, n_pairs, matrix, gap_open, gap_extend,
                                       sc, with_end ? ea : nullptr, with_end ? eb : nullptr, nullptr);
                (void)hipEventRecord(t1, nullptr);
                if (st != CM_OK) break;
                if ((e = hipEventSynchronize(t1)) != hipSuccess) { st = hip_fail(e, "tuner run"); break; }
                float f = 0.f;
                (void)hipEventElapsedTime(&f, t0, t1);
                if (rep > 0 && f < ms) ms = f;   // first run warms the plan
            }
            if (st != CM_OK) break;
            st = cm_context_sync(ctx);
            if (st != CM_OK) break;
            cur.resize(static_cast<size_t>(n_pairs) * (with_end ? 3 : 1));
            if ((e = hipMemcpy(cur.data(), d, cur.size() * 4, hipMemcpyDeviceToHost)) != hipSuccess) {
                st = hip_fail(e, "tuner results");
                break;
            }
            if (ref.empty()) ref = cur;
            else if (ref != cur) { st = fail(CM_EDEVICE, "launch plans disagree (kernel %d, rmax %d, %d blocks/CU)",
                                             cd.packed, cd.rmax, bpc); break; }
            if (table && rows < kMaxRows) {
                table[4 * rows] = cd.packed;
                table[4 * rows + 1] = cd.rmax;
                table[4 * rows + 2] = bpc;
                table[4 * rows + 3] = ms;
            }
            ++rows;
            if (ms < best_ms) { best_ms = ms; best = ctx->plan[pass]; }
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    (void)hipFree(d);
    ctx->plan[pass] = st == CM_OK ? best : saved;
    if (n_rows) *n_rows = rows < kMaxRows ? rows : kMaxRows;
    return st;
    CM_CATCH
}
