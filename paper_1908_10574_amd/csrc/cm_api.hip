// cm_api.hip -- host runtime behind include/cm.h: contexts, argument
// validation, device scratch, the plan/sort/sweep launch sequence.
#include <hipcub/hipcub.hpp>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "../../include/cm.h"
#include "cm_internal.h"
#include "cm_runtime.h"

static_assert(cmk::kMaxLen == CM_MAX_LEN, "kernel length limit and the ABI's CM_MAX_LEN differ");

namespace {
thread_local std::string g_last_error;
}

namespace cmrt {

cm_status fail(cm_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

cm_status hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? CM_ENOMEM : CM_EDEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

bool test_fail_alloc(const char* site) {
    const char* v = getenv("CM_TEST_FAIL_ALLOC");
    return v && std::strcmp(v, site) == 0;
}

void test_host_alloc_point() {
    if (test_fail_alloc("host")) throw std::bad_alloc();
}

bool DeviceBuf::ensure(size_t bytes) {
    if (bytes <= cap) return true;
    if (test_fail_alloc("device")) return false;
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    cap = 0;
    size_t want = bytes + bytes / 4 + 256;
    if (hipMalloc(&ptr, want) != hipSuccess) { ptr = nullptr; return false; }
    cap = want;
    return true;
}

void DeviceBuf::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    cap = 0;
}

cm_status check_matrix(const int32_t* matrix, int8_t* mat8 /* [21*24] */) {
    if (!matrix) return fail(CM_EINVAL, "matrix is NULL");
    std::memset(mat8, -128, cmk::kNRes * cmk::kMatStride);
    for (int x = 0; x < 20; ++x)
        for (int y = 0; y < 20; ++y) {
            const int32_t v = matrix[20 * x + y];
            if (v < -127 || v > 127)
                return fail(CM_EUNSUPPORTED, "matrix entry M[%d][%d]=%d outside [-127,127]", x, y, v);
            mat8[x * cmk::kMatStride + y] = static_cast<int8_t>(v);
        }
    return CM_OK;
}

cm_status check_gaps(int32_t go, int32_t ge) {
    if (!(go < 0 && go <= ge && ge <= 0))
        return fail(CM_EINVAL, "gaps must satisfy gap_open < 0 and gap_open <= gap_extend <= 0 (got %d, %d)",
                    go, ge);
    if (go < -1000000000 || ge < -1000000)
        return fail(CM_EINVAL, "gap penalties too large in magnitude (%d, %d)", go, ge);
    return CM_OK;
}

// temp bytes for the shared-query plan's sort, scan and selects over n pairs
static size_t plan_q_temp(int64_t n) {
    size_t t0 = 0, t1 = 0, t2 = 0;
    const int ni = static_cast<int>(n);
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, t0, static_cast<uint64_t*>(nullptr), static_cast<uint64_t*>(nullptr),
                                             static_cast<int32_t*>(nullptr), static_cast<int32_t*>(nullptr), ni, 0, 64);
    (void)hipcub::DeviceScan::InclusiveScan(nullptr, t1, static_cast<int32_t*>(nullptr), static_cast<int32_t*>(nullptr),
                                            hipcub::Max(), ni);
    (void)hipcub::DeviceSelect::Flagged(nullptr, t2, static_cast<int32_t*>(nullptr), static_cast<uint8_t*>(nullptr),
                                        static_cast<int32_t*>(nullptr), static_cast<int32_t*>(nullptr), ni);
    size_t t3 = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, t3, static_cast<uint32_t*>(nullptr), static_cast<uint32_t*>(nullptr),
                                             static_cast<int32_t*>(nullptr), static_cast<int32_t*>(nullptr), ni, 0, 32);
    return std::max(std::max(t0, t3), std::max(t1, t2));
}

static bool ensure_plan_q(cm_context* ctx, int64_t n) {
    const size_t m = static_cast<size_t>(n);
    return ctx->keys.ensure(m * 8) && ctx->keys_alt.ensure(m * 8) && ctx->vals.ensure(m * 4) &&
           ctx->vals_alt.ensure(m * 4) && ctx->q_start.ensure(m * 4) && ctx->q_len.ensure(m * 4) &&
           ctx->q_flags.ensure(m * 2) && ctx->q_lists.ensure(m * 12) && ctx->over.ensure(m * 4) &&
           ctx->sort_tmp.ensure(plan_q_temp(n));
}

// Shared-query plan and launches of the score pass (plan kind 2).
static cm_status run_pass_q(cm_context* ctx, cmk::SwArgs& a, hipStream_t st, int& timer_pair) {
    const int64_t n = a.n_pairs;
    if (!ensure_plan_q(ctx, n)) return fail(CM_ENOMEM, "cannot allocate the shared-query plan for %lld pairs",
                                            static_cast<long long>(n));
    a.over = static_cast<int32_t*>(ctx->over.ptr);
    const int ni = static_cast<int>(n);
    uint64_t* keys = static_cast<uint64_t*>(ctx->keys.ptr);
    uint64_t* keys_s = static_cast<uint64_t*>(ctx->keys_alt.ptr);
    int32_t* vals = static_cast<int32_t*>(ctx->vals.ptr);
    int32_t* vals_s = static_cast<int32_t*>(ctx->vals_alt.ptr);
    int32_t* start = static_cast<int32_t*>(ctx->q_start.ptr);
    int32_t* len = static_cast<int32_t*>(ctx->q_len.ptr);
    uint8_t* fa = static_cast<uint8_t*>(ctx->q_flags.ptr);
    uint8_t* fb = fa + n;
    int32_t* list_a = static_cast<int32_t*>(ctx->q_lists.ptr);
    int32_t* list_b = list_a + n;
    cmk::Counters* ctr = ctx->counters;
    size_t tmp = ctx->sort_tmp.cap;
    hipError_t e = cmk::launch_plan_q(a, keys, vals, st);
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairs(ctx->sort_tmp.ptr, tmp, keys, keys_s, vals, vals_s, ni, 0, 64, st);
    if (e == hipSuccess) e = cmk::launch_runs_q(keys_s, n, &ctr->n_work, len, st);
    tmp = ctx->sort_tmp.cap;
    if (e == hipSuccess) e = hipcub::DeviceScan::InclusiveScan(ctx->sort_tmp.ptr, tmp, len, start, hipcub::Max(), ni, st);
    if (e == hipSuccess) e = cmk::launch_flags_q(keys_s, start, n, &ctr->n_work, len, fa, fb, st);
    tmp = ctx->sort_tmp.cap;
    if (e == hipSuccess)
        e = hipcub::DeviceSelect::Flagged(ctx->sort_tmp.ptr, tmp, vals_s, fa, list_a, &ctr->n_sel[0], ni, st);
    tmp = ctx->sort_tmp.cap;
    if (e == hipSuccess)
        e = hipcub::DeviceSelect::Flagged(ctx->sort_tmp.ptr, tmp, vals_s, fb, list_b, &ctr->n_sel[1], ni, st);
    // the rest, sorted by the two-profile kernel's own shape keys so that the
    // pairs of an item have like shapes (start / len are free again)
    cmk::SwArgs bb = a;
    bb.rmax = cmk::kRMaxChoicePk[cmk::kNumRMaxPk - 1];
    uint32_t* kb = reinterpret_cast<uint32_t*>(start);
    uint32_t* kb_s = reinterpret_cast<uint32_t*>(len);
    int32_t* list_b_s = list_b + n;
    if (e == hipSuccess) e = cmk::launch_keys_list(bb, list_b, &ctr->n_sel[1], n, kb, st);
    tmp = ctx->sort_tmp.cap;
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairs(ctx->sort_tmp.ptr, tmp, kb, kb_s, list_b, list_b_s, ni, 0, 32, st);
    if (e != hipSuccess) return hip_fail(e, "shared-query plan");
    cmk::SwArgs aa = a;
    aa.keys = nullptr; aa.order = list_a; aa.n_work_ptr = &ctr->n_sel[0]; aa.ticket = &ctr->ticket;
    aa.rmax = cmk::kRMaxQ;
    bb.keys = kb_s; bb.order = list_b_s; bb.n_work_ptr = &ctr->n_sel[1]; bb.ticket = &ctr->ticket_b;
    // the two kernels run concurrently: list B's boundary slots follow list A's
    const int grid_a = ctx->n_cu * ctx->plan[CM_PASS_SCORE].blocks_per_cu;
    const int grid_b = ctx->n_cu * ctx->occ_pk[cmk::kNumRMaxPk - 1];
    bb.bnd = a.bnd + static_cast<int64_t>(grid_a) * cmk::kPairsPerWave * a.bnd_stride;
    if (static_cast<size_t>(grid_a + grid_b) * cmk::kPairsPerWave * a.bnd_stride * sizeof(int2) > ctx->bnd.cap)
        return fail(CM_EINVAL, "boundary rows too small for the shared-query launch");
    KernelTimer& kt = ctx->timer;
    if (timer_pair >= 0) (void)hipEventRecord(kt.pool[2 * timer_pair], st);
    e = cmk::launch_sw_pkq(aa, bb, grid_a, grid_b, ctx->n_cu * ctx->occ_over, st, ctx->side, ctx->ev_fork,
                           ctx->ev_join);
    if (e != hipSuccess) return hip_fail(e, "alignment launch");
    if (timer_pair >= 0) {
        (void)hipEventRecord(kt.pool[2 * timer_pair + 1], st);
        kt.pending.emplace_back(CM_PASS_SCORE, timer_pair);
    }
    return CM_OK;
}

// a timing event pair for the next launch (or -1 when timing is off)
static cm_status timer_slot(cm_context* ctx, int* pair) {
    KernelTimer& kt = ctx->timer;
    *pair = -1;
    if (!kt.on) return CM_OK;
    if (kt.next * 2 + 2 > kt.pool.size()) {
        hipEvent_t b, c;
        if (hipEventCreate(&b) != hipSuccess || hipEventCreate(&c) != hipSuccess)
            return fail(CM_EDEVICE, "timing events");
        kt.pool.push_back(b);
        kt.pool.push_back(c);
    }
    *pair = static_cast<int>(kt.next++);
    return CM_OK;
}

// plan -> sort -> persistent sweep of one pass (int32 or two-profile packed
// kernel) on scratch the caller provides; allocates nothing
cm_status run_pass_scratch(cm_context* ctx, cmk::SwArgs& a, cmk::Pass pass, const PassScratch& ps,
                           hipStream_t st) {
    const int n = static_cast<int>(a.n_pairs);
    const bool packed = pass == cmk::Pass::Score && ps.packed;
    if (packed) {
        a.packed = 1;
        a.over = ps.over;
        const uint32_t go = static_cast<uint32_t>(-static_cast<int64_t>(a.go) < 65535 ? -a.go : 65535);
        const uint32_t ge = static_cast<uint32_t>(-static_cast<int64_t>(a.ge) < 65535 ? -a.ge : 65535);
        a.go_pk = go * 0x10001u;
        a.ge_pk = ge * 0x10001u;
    }
    a.rmax = ps.rmax;
    a.ctr = ps.ctr;
    a.err = ctx->err_flag;
    a.dummy = ctx->dummy;
    a.bnd = static_cast<int2*>(ctx->bnd.ptr);
    a.bnd_stride = ctx->bnd_stride;
    a.zero = 0;
    a.cells_acc = ps.timed ? ctx->cells_acc + static_cast<int>(pass) : nullptr;
    hipError_t e = cmk::launch_plan(a, pass, ps.keys, ps.vals, st);
    if (e != hipSuccess) return hip_fail(e, "plan launch");
    size_t tmp = ps.sort_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(ps.sort_tmp, tmp, ps.keys, ps.keys_alt, ps.vals, ps.vals_alt, n, 0, 32, st);
    if (e != hipSuccess) return hip_fail(e, "sort");
    a.keys = ps.keys_alt;
    a.order = ps.vals_alt;
    int pair = -1;
    if (ps.timed) {
        cm_status r = timer_slot(ctx, &pair);
        if (r != CM_OK) return r;
    }
    KernelTimer& kt = ctx->timer;
    if (pair >= 0) (void)hipEventRecord(kt.pool[2 * pair], st);
    e = packed ? cmk::launch_sw_pk(a, ps.grid, ctx->n_cu * ctx->occ_over, st) : cmk::launch_sw(a, pass, ps.grid, st);
    if (e != hipSuccess) return hip_fail(e, "alignment launch");
    if (pair >= 0) {
        (void)hipEventRecord(kt.pool[2 * pair + 1], st);
        kt.pending.emplace_back(static_cast<int>(pass), pair);
    }
    return CM_OK;
}

size_t sort_temp_bytes(int64_t n) {
    size_t tmp = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, static_cast<uint32_t*>(nullptr),
                                             static_cast<uint32_t*>(nullptr), static_cast<int32_t*>(nullptr),
                                             static_cast<int32_t*>(nullptr), static_cast<int>(n), 0, 32);
    return tmp;
}

// plan -> sort -> persistent sweep for one pass
cm_status run_pass(cm_context* ctx, cmk::SwArgs& a, cmk::Pass pass, hipStream_t st) {
    if (a.n_pairs <= 0) return CM_OK;
    if (a.n_pairs > (int64_t)0x7fffffff) return fail(CM_EINVAL, "n_pairs too large");
    const size_t n = static_cast<size_t>(a.n_pairs);
    const cm_context::Plan& plan = ctx->plan[static_cast<int>(pass)];
    const bool packed = pass == cmk::Pass::Score && plan.packed;
    if (packed && plan.packed == 2) {
        a.rmax = plan.rmax;
        a.ctr = ctx->counters;
        a.err = ctx->err_flag;
        a.dummy = ctx->dummy;
        a.bnd = static_cast<int2*>(ctx->bnd.ptr);
        a.bnd_stride = ctx->bnd_stride;
        a.zero = 0;
        a.cells_acc = ctx->cells_acc + CM_PASS_SCORE;
        a.packed = 1;
        const uint32_t go = static_cast<uint32_t>(-static_cast<int64_t>(a.go) < 65535 ? -a.go : 65535);
        const uint32_t ge = static_cast<uint32_t>(-static_cast<int64_t>(a.ge) < 65535 ? -a.ge : 65535);
        a.go_pk = go * 0x10001u;
        a.ge_pk = ge * 0x10001u;
        int timer_pair = -1;
        cm_status r = timer_slot(ctx, &timer_pair);
        if (r != CM_OK) return r;
        return run_pass_q(ctx, a, st, timer_pair);
    }
    if (!ctx->keys.ensure(n * 4) || !ctx->keys_alt.ensure(n * 4) || !ctx->vals.ensure(n * 4) ||
        !ctx->vals_alt.ensure(n * 4))
        return fail(CM_ENOMEM, "cannot allocate %zu plan entries", n);
    const size_t tmp = sort_temp_bytes(a.n_pairs);
    if (!ctx->sort_tmp.ensure(tmp)) return fail(CM_ENOMEM, "cannot allocate sort scratch");
    if (packed && !ctx->over.ensure(n * 4)) return fail(CM_ENOMEM, "cannot allocate %zu saturation slots", n);
    PassScratch ps;
    ps.packed = packed ? 1 : 0;
    ps.rmax = plan.rmax;
    ps.grid = ctx->n_cu * plan.blocks_per_cu;
    ps.keys = static_cast<uint32_t*>(ctx->keys.ptr);
    ps.keys_alt = static_cast<uint32_t*>(ctx->keys_alt.ptr);
    ps.vals = static_cast<int32_t*>(ctx->vals.ptr);
    ps.vals_alt = static_cast<int32_t*>(ctx->vals_alt.ptr);
    ps.over = packed ? static_cast<int32_t*>(ctx->over.ptr) : nullptr;
    ps.sort_tmp = ctx->sort_tmp.ptr;
    ps.sort_bytes = ctx->sort_tmp.cap;
    ps.ctr = ctx->counters;
    ps.timed = true;
    return run_pass_scratch(ctx, a, pass, ps, st);
}

void drain_timers(cm_context* ctx, bool blocking) {
    KernelTimer& kt = ctx->timer;
    size_t k = 0;
    for (; k < kt.pending.size(); ++k) {
        const int pass = kt.pending[k].first, pair = kt.pending[k].second;
        hipEvent_t end = kt.pool[2 * pair + 1];
        if (blocking) (void)hipEventSynchronize(end);
        else if (hipEventQuery(end) != hipSuccess) break;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, kt.pool[2 * pair], end) == hipSuccess) {
            kt.secs[pass] += ms * 1e-3;
            kt.launches[pass] += 1;
        }
    }
    kt.pending.erase(kt.pending.begin(), kt.pending.begin() + static_cast<long>(k));
    if (kt.pending.empty()) kt.next = 0;
}

int plan_limit(const cm_context* ctx, int pass, int packed, int rmax) {
    if (pass < 0 || pass > 2) return 0;
    if (packed == 2) return (pass == CM_PASS_SCORE && rmax == cmk::kRMaxQ) ? ctx->occ_pkq : 0;
    if (packed) {
        if (pass != CM_PASS_SCORE) return 0;
        for (int q = 0; q < cmk::kNumRMaxPk; ++q)
            if (cmk::kRMaxChoicePk[q] == rmax) return ctx->occ_pk[q];
        return 0;
    }
    for (int q = 0; q < cmk::kNumRMax; ++q)
        if (cmk::kRMaxChoice[q] == rmax) return ctx->occ[pass][q];
    return 0;
}

// Plan cache: text lines "<arch> <runtime> <pass> <packed> <rmax> <blocks_per_cu>".
// Entries for another architecture or runtime, or out of range, are ignored.
cm_status load_plans(cm_context* ctx, const char* path) {
    FILE* f = fopen(path, "r");
    if (!f) return fail(CM_EINVAL, "cannot open %s", path);
    char arch[64];
    int rt, pass, packed, rmax, bpc, used = 0;
    while (fscanf(f, "%63s %d %d %d %d %d", arch, &rt, &pass, &packed, &rmax, &bpc) == 6) {
        if (std::strcmp(arch, ctx->arch) != 0 || rt != ctx->runtime_version) continue;
        const int lim = plan_limit(ctx, pass, packed, rmax);
        if (lim < 1 || bpc < 1 || bpc > lim) continue;
        ctx->plan[pass].packed = packed;
        ctx->plan[pass].rmax = rmax;
        ctx->plan[pass].blocks_per_cu = bpc;
        ++used;
    }
    fclose(f);
    return used ? CM_OK : fail(CM_EINVAL, "no usable plan in %s", path);
}

cm_status save_plans(const cm_context* ctx, const char* path) {
    FILE* f = fopen(path, "w");
    if (!f) return fail(CM_EINVAL, "cannot write %s", path);
    for (int p = 0; p < 3; ++p)
        fprintf(f, "%s %d %d %d %d %d\n", ctx->arch, ctx->runtime_version, p, ctx->plan[p].packed,
                ctx->plan[p].rmax, ctx->plan[p].blocks_per_cu);
    return fclose(f) == 0 ? CM_OK : fail(CM_EINVAL, "cannot write %s", path);
}

// make plan/sort scratch large enough for n pairs (no allocation later)
cm_status reserve(cm_context* ctx, int64_t n) {
    const size_t m = static_cast<size_t>(n);
    if (!ctx->keys.ensure(m * 4) || !ctx->keys_alt.ensure(m * 4) || !ctx->vals.ensure(m * 4) ||
        !ctx->vals_alt.ensure(m * 4) || !ctx->over.ensure(m * 4))
        return fail(CM_ENOMEM, "cannot allocate %zu plan entries", m);
    size_t tmp = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(
        nullptr, tmp, static_cast<uint32_t*>(ctx->keys.ptr), static_cast<uint32_t*>(ctx->keys_alt.ptr),
        static_cast<int32_t*>(ctx->vals.ptr), static_cast<int32_t*>(ctx->vals_alt.ptr), static_cast<int>(m), 0, 32,
        nullptr);
    if (e != hipSuccess) return hip_fail(e, "sort size query");
    if (!ctx->sort_tmp.ensure(tmp)) return fail(CM_ENOMEM, "cannot allocate sort scratch");
    if (ctx->plan[CM_PASS_SCORE].packed == 2 && !ensure_plan_q(ctx, n))
        return fail(CM_ENOMEM, "cannot allocate the shared-query plan");
    return CM_OK;
}

cm_status score_args(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                     const int32_t* pairs, int64_t n_pairs, const int64_t* n_live, const int32_t* matrix,
                     int32_t gap_open, int32_t gap_extend, int32_t* scores, int32_t* end_a, int32_t* end_b,
                     cmk::SwArgs& a) {
    if (!ctx) return fail(CM_EINVAL, "ctx is NULL");
    if (n_pairs < 0 || n_seqs < 0) return fail(CM_EINVAL, "negative count");
    if (n_pairs == 0) return CM_OK;
    if (!offsets || !pairs || !scores) return fail(CM_EINVAL, "NULL required pointer");
    if ((end_a == nullptr) != (end_b == nullptr)) return fail(CM_EINVAL, "end_a and end_b must both be set or both NULL");
    cm_status s = check_gaps(gap_open, gap_extend);
    if (s != CM_OK) return s;
    a = cmk::SwArgs{};
    s = check_matrix(matrix, a.mat);
    if (s != CM_OK) return s;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    a.seqs = seqs ? seqs : ctx->dummy;
    a.offsets = offsets;
    a.pairs = pairs;
    a.n_pairs = n_pairs;
    a.n_live = n_live;
    a.n_seqs = n_seqs;
    a.go = gap_open;
    a.ge = gap_extend;
    a.scores = scores;
    a.end_a = end_a;
    a.end_b = end_b;
    return CM_OK;
}

cm_status score_batch(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                      const int32_t* pairs, int64_t n_pairs, const int64_t* n_live, const int32_t* matrix,
                      int32_t gap_open, int32_t gap_extend, int32_t* scores, int32_t* end_a, int32_t* end_b,
                      hipStream_t stream) {
    cmk::SwArgs a{};
    cm_status s = score_args(ctx, seqs, offsets, n_seqs, pairs, n_pairs, n_live, matrix, gap_open, gap_extend, scores,
                             end_a, end_b, a);
    if (s != CM_OK || n_pairs == 0) return s;
    return run_pass(ctx, a, end_a ? cmk::Pass::ScoreEnd : cmk::Pass::Score, stream);
}

cm_status end_batch(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                    const int32_t* pairs, int64_t n_pairs, const int64_t* n_live, const int32_t* matrix,
                    int32_t gap_open, int32_t gap_extend, int32_t* scores, int32_t* end_a, int32_t* end_b,
                    int32_t min_score, hipStream_t stream) {
    if (!ctx) return fail(CM_EINVAL, "ctx is NULL");
    if (n_pairs < 0 || n_seqs < 0) return fail(CM_EINVAL, "negative count");
    if (n_pairs == 0) return CM_OK;
    if (!offsets || !pairs || !scores || !end_a || !end_b) return fail(CM_EINVAL, "NULL required pointer");
    if (min_score < 0) return fail(CM_EINVAL, "min_score must be >= 0");
    cm_status s = check_gaps(gap_open, gap_extend);
    if (s != CM_OK) return s;
    cmk::SwArgs a{};
    s = check_matrix(matrix, a.mat);
    if (s != CM_OK) return s;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    a.seqs = seqs ? seqs : ctx->dummy;
    a.offsets = offsets;
    a.pairs = pairs;
    a.n_pairs = n_pairs;
    a.n_live = n_live;
    a.n_seqs = n_seqs;
    a.go = gap_open;
    a.ge = gap_extend;
    a.min_score = min_score;
    a.end_filter = 1;
    a.scores = scores;
    a.end_a = end_a;
    a.end_b = end_b;
    return run_pass(ctx, a, cmk::Pass::ScoreEnd, stream);
}

cm_status span_batch(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                     const int32_t* pairs, int64_t n_pairs, const int64_t* n_live, const int32_t* matrix,
                     int32_t gap_open, int32_t gap_extend, const int32_t* scores, const int32_t* end_a,
                     const int32_t* end_b, int32_t min_score, int32_t* start_a, int32_t* start_b,
                     hipStream_t stream) {
    if (!ctx) return fail(CM_EINVAL, "ctx is NULL");
    if (n_pairs < 0 || n_seqs < 0) return fail(CM_EINVAL, "negative count");
    if (n_pairs == 0) return CM_OK;
    if (!offsets || !pairs || !scores || !end_a || !end_b || !start_a || !start_b)
        return fail(CM_EINVAL, "NULL required pointer");
    if (min_score < 0) return fail(CM_EINVAL, "min_score must be >= 0");
    cm_status s = check_gaps(gap_open, gap_extend);
    if (s != CM_OK) return s;
    cmk::SwArgs a{};
    s = check_matrix(matrix, a.mat);
    if (s != CM_OK) return s;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    a.seqs = seqs ? seqs : ctx->dummy;
    a.offsets = offsets;
    a.pairs = pairs;
    a.n_pairs = n_pairs;
    a.n_live = n_live;
    a.n_seqs = n_seqs;
    a.go = gap_open;
    a.ge = gap_extend;
    a.min_score = min_score;
    a.scores = const_cast<int32_t*>(scores);
    a.end_a = const_cast<int32_t*>(end_a);
    a.end_b = const_cast<int32_t*>(end_b);
    a.start_a = start_a;
    a.start_b = start_b;
    return run_pass(ctx, a, cmk::Pass::Span, stream);
}

}  // namespace cmrt

using namespace cmrt;

extern "C" {

const char* cm_status_str(cm_status s) {
    switch (s) {
        case CM_OK: return "ok";
        case CM_EINVAL: return "invalid argument";
        case CM_ERANGE: return "input data out of range";
        case CM_ENOMEM: return "out of device memory";
        case CM_EDEVICE: return "device error";
        case CM_EUNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

const char* cm_last_error(void) { return g_last_error.c_str(); }

cm_status cm_context_create(int device_ordinal, cm_context** out) {
    CM_TRY
    if (!out) return fail(CM_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device_ordinal < 0 || device_ordinal >= ndev)
        return fail(CM_EINVAL, "device %d out of range (%d devices)", device_ordinal, ndev);
    e = hipSetDevice(device_ordinal);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    cm_context* ctx = new cm_context();
    ctx->device = device_ordinal;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device_ordinal);
    if (e != hipSuccess) { delete ctx; return hip_fail(e, "hipGetDeviceProperties"); }
    ctx->n_cu = prop.multiProcessorCount;
    std::snprintf(ctx->arch, sizeof(ctx->arch), "%s", prop.gcnArchName);
    (void)hipRuntimeGetVersion(&ctx->runtime_version);
    int gmax = 1;
    for (int p = 0; p < 3; ++p) {
        for (int k = 0; k < cmk::kNumRMax; ++k) {
            ctx->occ[p][k] = cmk::sw_blocks_per_cu(static_cast<cmk::Pass>(p), cmk::kRMaxChoice[k]);
            gmax = ctx->occ[p][k] > gmax ? ctx->occ[p][k] : gmax;
        }
        ctx->plan[p].rmax = 16;
        ctx->plan[p].blocks_per_cu = ctx->occ[p][cmk::kNumRMax - 1];
    }
    for (int k = 0; k < cmk::kNumRMaxPk; ++k) {
        ctx->occ_pk[k] = cmk::sw_pk_blocks_per_cu(cmk::kRMaxChoicePk[k]);
        gmax = ctx->occ_pk[k] > gmax ? ctx->occ_pk[k] : gmax;
    }
    ctx->occ_over = cmk::sw_over_blocks_per_cu();
    gmax = ctx->occ_over > gmax ? ctx->occ_over : gmax;
    ctx->occ_pkq = cmk::sw_pkq_blocks_per_cu();
    // the shared-query kernel and the two-profile kernel of its second list run
    // concurrently, each with boundary-row slots of its own
    const int g_q = ctx->occ_pkq + ctx->occ_pk[cmk::kNumRMaxPk - 1];
    gmax = g_q > gmax ? g_q : gmax;
    // the score pass defaults to the shared-query packed kernel (items of one
    // query, up to 32 rows per lane; the rest on the two-profile packed kernel)
    ctx->plan[CM_PASS_SCORE].packed = 2;
    ctx->plan[CM_PASS_SCORE].rmax = cmk::kRMaxQ;
    ctx->plan[CM_PASS_SCORE].blocks_per_cu = ctx->occ_pkq;
    gmax *= ctx->n_cu;
    void* small = nullptr;
    e = hipMalloc(&small, 4096);
    if (e != hipSuccess) { delete ctx; return hip_fail(e, "context scratch"); }
    (void)hipMemset(small, 0, 4096);
    ctx->small = small;
    ctx->counters = reinterpret_cast<cmk::Counters*>(static_cast<char*>(small));
    ctx->err_flag = reinterpret_cast<uint32_t*>(static_cast<char*>(small) + 1024);
    ctx->dummy = reinterpret_cast<const uint8_t*>(static_cast<char*>(small) + 2048);
    ctx->cells_acc = reinterpret_cast<unsigned long long*>(static_cast<char*>(small) + 3072);
    // boundary rows: one slot per group of the largest persistent grid
    ctx->bnd_stride = CM_MAX_LEN + 64;
    const size_t bnd_bytes = static_cast<size_t>(gmax) * cmk::kPairsPerWave * ctx->bnd_stride * sizeof(int2);
    if (!ctx->bnd.ensure(bnd_bytes)) {
        (void)hipFree(small);
        delete ctx;
        return fail(CM_ENOMEM, "cannot allocate %zu bytes of boundary rows", bnd_bytes);
    }
    e = hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) { cm_context_destroy(ctx); return hip_fail(e, "context init"); }
    // device address of the allocation-free entry point's scratch array (once
    // per device; a failure only disables that entry point, which reports it)
    (void)noalloc_setup(device_ordinal);
    const char* cache = getenv("CM_AUTOTUNE_CACHE");
    if (cache && *cache) (void)load_plans(ctx, cache);   // a missing or corrupt cache keeps the defaults
    *out = ctx;
    return CM_OK;
    CM_CATCH
}

void cm_context_destroy(cm_context* ctx) {
    CM_TRY
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->keys.release();
    ctx->keys_alt.release();
    ctx->vals.release();
    ctx->vals_alt.release();
    ctx->sort_tmp.release();
    ctx->bnd.release();
    ctx->over.release();
    ctx->q_start.release();
    ctx->q_len.release();
    ctx->q_flags.release();
    ctx->q_lists.release();
    ctx->extra_release();
    for (hipEvent_t ev : ctx->timer.pool) (void)hipEventDestroy(ev);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->small) (void)hipFree(ctx->small);
    delete ctx;
    CM_CATCH_VOID
}

cm_status cm_context_sync(cm_context* ctx) {
    CM_TRY
    if (!ctx) return fail(CM_EINVAL, "ctx is NULL");
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "synchronize");
    drain_timers(ctx, true);
    uint32_t flag = 0;
    e = hipMemcpy(&flag, ctx->err_flag, sizeof(flag), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read error flag");
    if (flag) {
        const uint32_t zero = 0;
        (void)hipMemcpy(ctx->err_flag, &zero, sizeof(zero), hipMemcpyHostToDevice);
        if (flag & cmk::kErrPlan) return fail(CM_EDEVICE, "internal error: an item's pairs do not share its query");
        if (flag & cmk::kErrTrace)
            return fail(CM_EDEVICE, "traceback: a box does not reproduce its pair's score (inconsistent cells)");
        return fail(CM_ERANGE, "device flagged bad input:%s%s%s%s%s",
                    (flag & cmk::kErrResidue) ? " residue>=20" : "",
                    (flag & cmk::kErrIndex) ? " index out of range" : "",
                    (flag & cmk::kErrLength) ? " sequence longer than CM_MAX_LEN" : "",
                    (flag & cmk::kErrCell) ? " end cell outside its sequence" : "",
                    (flag & cmk::kErrCapacity) ? " column buffer too small" : "");
    }
    return CM_OK;
    CM_CATCH
}

cm_status cm_context_set_timing(cm_context* ctx, int on) {
    CM_TRY
    if (!ctx) return fail(CM_EINVAL, "ctx is NULL");
    drain_timers(ctx, true);
    ctx->timer.on = on != 0;
    return CM_OK;
    CM_CATCH
}

cm_status cm_context_set_graphs(cm_context* ctx, int on) {
    CM_TRY
    if (!ctx) return fail(CM_EINVAL, "ctx is NULL");
    ctx->graphs = on != 0;
    return CM_OK;
    CM_CATCH
}

cm_status cm_context_kernel_time(cm_context* ctx, int pass, int64_t* launches, double* seconds) {
    CM_TRY
    if (!ctx || pass < 0 || pass > 2) return fail(CM_EINVAL, "bad argument");
    drain_timers(ctx, true);
    if (launches) *launches = ctx->timer.launches[pass];
    if (seconds) *seconds = ctx->timer.secs[pass];
    return CM_OK;
    CM_CATCH
}

cm_status cm_context_cells_computed(cm_context* ctx, int pass, double* cells) {
    CM_TRY
    if (!ctx || !cells || pass < 0 || pass > 2) return fail(CM_EINVAL, "bad argument");
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    unsigned long long v = 0;
    if (e == hipSuccess) e = hipMemcpy(&v, ctx->cells_acc + pass, sizeof(v), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "cells computed");
    *cells = static_cast<double>(v);
    return CM_OK;
    CM_CATCH
}

cm_status cm_plan_get(const cm_context* ctx, int pass, int32_t* packed, int32_t* rmax, int32_t* blocks_per_cu,
                      int32_t* max_blocks_per_cu) {
    CM_TRY
    if (!ctx || pass < 0 || pass > 2) return fail(CM_EINVAL, "bad argument");
    const cm_context::Plan& pl = ctx->plan[pass];
    if (packed) *packed = pl.packed;
    if (rmax) *rmax = pl.rmax;
    if (blocks_per_cu) *blocks_per_cu = pl.blocks_per_cu;
    if (max_blocks_per_cu) *max_blocks_per_cu = plan_limit(ctx, pass, pl.packed, pl.rmax);
    return CM_OK;
    CM_CATCH
}

cm_status cm_plan_set(cm_context* ctx, int pass, int32_t packed, int32_t rmax, int32_t blocks_per_cu) {
    CM_TRY
    if (!ctx || pass < 0 || pass > 2) return fail(CM_EINVAL, "bad argument");
    if (packed < 0 || packed > 2) return fail(CM_EINVAL, "packed must be 0, 1 or 2");
    if (packed && pass != CM_PASS_SCORE) return fail(CM_EINVAL, "the packed kernels serve the score pass only");
    const int lim = plan_limit(ctx, pass, packed, rmax);
    if (lim < 1)
        return fail(CM_EINVAL, packed == 2 ? "shared-query rmax must be 32"
                                           : (packed ? "packed rmax must be 4 or 8" : "rmax must be 8, 12 or 16"));
    if (blocks_per_cu < 1 || blocks_per_cu > lim)
        return fail(CM_EINVAL, "blocks_per_cu must be in [1, %d]", lim);
    drain_timers(ctx, true);
    ctx->plan[pass].packed = packed;
    ctx->plan[pass].rmax = rmax;
    ctx->plan[pass].blocks_per_cu = blocks_per_cu;
    return CM_OK;
    CM_CATCH
}

cm_status cm_plan_save(const cm_context* ctx, const char* path) {
    CM_TRY
    if (!ctx || !path) return fail(CM_EINVAL, "bad argument");
    return save_plans(ctx, path);
    CM_CATCH
}

cm_status cm_plan_load(cm_context* ctx, const char* path) {
    CM_TRY
    if (!ctx || !path) return fail(CM_EINVAL, "bad argument");
    return load_plans(ctx, path);
    CM_CATCH
}

cm_status cm_sw_score_batch(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                            const int32_t* pairs, int64_t n_pairs, const int32_t* matrix, int32_t gap_open,
                            int32_t gap_extend, int32_t* scores, int32_t* end_a, int32_t* end_b, void* stream) {
    CM_TRY
    return score_batch(ctx, seqs, offsets, n_seqs, pairs, n_pairs, nullptr, matrix, gap_open, gap_extend, scores,
                       end_a, end_b, static_cast<hipStream_t>(stream));
    CM_CATCH
}

cm_status cm_sw_span_batch(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                           const int32_t* pairs, int64_t n_pairs, const int32_t* matrix, int32_t gap_open,
                           int32_t gap_extend, const int32_t* scores, const int32_t* end_a, const int32_t* end_b,
                           int32_t min_score, int32_t* start_a, int32_t* start_b, void* stream) {
    CM_TRY
    return span_batch(ctx, seqs, offsets, n_seqs, pairs, n_pairs, nullptr, matrix, gap_open, gap_extend, scores,
                      end_a, end_b, min_score, start_a, start_b, static_cast<hipStream_t>(stream));
    CM_CATCH
}

}  // extern "C"
