// cm_driver.hip -- ClusterMerge on top of the batched Smith-Waterman kernels.
//
// Algorithm 2 (BottomUpMerge, Section 3.2) fixes the merge tree from n alone:
// the FIFO pops sets in pairs and pushes each result to the back.  Merges whose
// inputs exist after the same number of rounds (the tree level) are independent
// and are scored together.  Algorithm 1 (Cluster Set Merge, Section 3.1) is
// replayed on the host exactly in its sequential order; every alignment score
// it needs comes from the GPU in batches ("waves"):
//   wave A  every representative pair of every merge of the level, with end
//           cells, and the start cells of pairs scoring above mT (the protein
//           transitivity test of Section 4 needs the covered span);
//   waves   the replay of each merge runs until an ExchangeSimilar event lacks
//           member-vs-representative scores; that event's pairs are requested
//           exactly, and a dry walk over the rest of the merge (whose full-merge
//           and break decisions depend on representative scores only) requests
//           the later exchange events' pairs speculatively.  All merges' requests
//           form one GPU batch; the replays resume until every merge is done.
// The final stage aligns the unique within-cluster pairs (Section 6.1),
// generated per element in sorted order, reusing scores already computed.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <vector>

#include "../../include/cm.h"
#include "cm_internal.h"
#include "cm_runtime.h"

namespace cmdrv {
// Device-side compaction of the end/start cells: every row (< live count)
// whose score exceeds min_score appends (row, end_a, end_b, start_a,
// start_b); rows arrive in any order (the host sorts them).
__global__ void k_zero_u32(uint32_t* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}
__global__ void k_end_compact(const int32_t* planes, int64_t stride, const int64_t* n_live, int64_t n,
                              int32_t min_score, uint32_t* count, int32_t* entries) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int64_t live = n_live ? *n_live : n;
    if (i >= live || i >= n) return;
    if (planes[i] > min_score) {
        const uint32_t k = atomicAdd(count, 1u);
        int32_t* e = entries + 5 * static_cast<int64_t>(k);
        e[0] = static_cast<int32_t>(i);
        e[1] = planes[stride + i];
        e[2] = planes[2 * stride + i];
        e[3] = planes[3 * stride + i];
        e[4] = planes[4 * stride + i];
    }
}
// The representative pairs of a level, merge by merge: merge m's block of
// pairs starts at desc[5m] and holds its n1 x n2 product, row-major
// (desc[5m + 1], desc[5m + 2]: offset and count of the first set's
// representatives in reps; desc[5m + 3], desc[5m + 4]: the second set's).
// Offsets ascend; every merge has n2 >= 1.
__global__ void k_rep_product(const int64_t* desc, int n_merges, const int32_t* reps, int64_t n, int32_t* pairs) {
    const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (t >= n) return;
    int lo = 0, hi = n_merges - 1;   // the last merge whose block starts at or before t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[5 * mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    const int64_t* d = desc + 5 * static_cast<int64_t>(lo);
    const int64_t local = t - d[0];
    const int64_t i = local / d[4], j = local - i * d[4];
    pairs[2 * t] = reps[d[1] + i];
    pairs[2 * t + 1] = reps[d[3] + j];
}
// The same product with the screen's size guard: guard[t] = 1 when the two
// clusters' member counts (counts, parallel to reps) multiply to at least
// min_product (> 0).
__global__ void k_rep_product_guard(const int64_t* desc, int n_merges, const int32_t* reps, const int32_t* counts,
                                    int64_t min_product, int64_t n, int32_t* pairs, uint8_t* guard) {
    const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (t >= n) return;
    int lo = 0, hi = n_merges - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[5 * mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    const int64_t* d = desc + 5 * static_cast<int64_t>(lo);
    const int64_t local = t - d[0];
    const int64_t i = local / d[4], j = local - i * d[4];
    pairs[2 * t] = reps[d[1] + i];
    pairs[2 * t + 1] = reps[d[3] + j];
    guard[t] = (min_product > 0 &&
                static_cast<int64_t>(counts[d[1] + i]) * static_cast<int64_t>(counts[d[3] + j]) >= min_product) ? 1 : 0;
}
// keep[i] = guard[i] (bypasses the screen) or logit >= tau
__global__ void k_keep(const float* z, const uint8_t* guard, float tau, int64_t n, uint8_t* keep) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i < n) keep[i] = (guard[i] != 0 || z[i] >= tau) ? 1 : 0;
}
}  // namespace cmdrv

// End and start cells of one pair whose score exceeds mT.
struct EndRec { int32_t idx, ea, eb, sa, sb; };

struct cm_result {
    std::vector<int32_t> reps;
    std::vector<int64_t> member_offsets;
    std::vector<int32_t> members;
    std::vector<int32_t> pairs;
    std::vector<int32_t> pair_scores;
    // pairs scored during the merge stage (representative and exchange
    // alignments, speculative ones included), when params.record_candidates
    std::vector<int32_t> cand_pairs;
    std::vector<int32_t> cand_scores;
    cm_stats stats{};
};

namespace cmdrv {

using cmrt::fail;
using cmrt::hip_fail;
using Clock = std::chrono::steady_clock;

static double secs(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double>(b - a).count();
}

// ---------------------------------------------------------------------------
// open-addressing map: unordered pair key -> int32 value
// ---------------------------------------------------------------------------
class PairMap {
public:
    static uint64_t key(int32_t x, int32_t y) {
        return (static_cast<uint64_t>(static_cast<uint32_t>(x)) << 32) | static_cast<uint32_t>(y);
    }
    PairMap() { rehash(1 << 16); }
    void clear() { rehash(1 << 16); }
    bool find(uint64_t k, int32_t* v) const {
        size_t i = mix(k) & mask_;
        while (true) {
            const uint64_t kk = keys_[i];
            if (kk == kEmpty) return false;
            if (kk == k) { *v = vals_[i]; return true; }
            i = (i + 1) & mask_;
        }
    }
    void put(uint64_t k, int32_t v) {
        if (2 * (size_ + 1) > keys_.size()) rehash(keys_.size() * 2);
        size_t i = mix(k) & mask_;
        while (keys_[i] != kEmpty && keys_[i] != k) i = (i + 1) & mask_;
        if (keys_[i] == kEmpty) ++size_;
        keys_[i] = k;
        vals_[i] = v;
    }
    size_t size() const { return size_; }
    // entries as (key, value) sorted by key: for keys made with key(x, y),
    // grouped by x with y ascending.  With every x below n_x: a counting
    // sort by x, then each x's (short) run sorted by y; otherwise one sort.
    void sorted_entries(std::vector<std::pair<uint64_t, int32_t>>* out, int32_t n_x) const {
        out->clear();
        bool bounded = n_x > 0;
        std::vector<size_t> start;
        if (bounded) {
            start.assign(static_cast<size_t>(n_x) + 1, 0);
            for (size_t i = 0; i < keys_.size() && bounded; ++i) {
                if (keys_[i] == kEmpty) continue;
                const uint64_t x = keys_[i] >> 32;
                if (x >= static_cast<uint64_t>(n_x)) bounded = false;
                else ++start[x + 1];
            }
        }
        if (!bounded) {
            out->reserve(size_);
            for (size_t i = 0; i < keys_.size(); ++i)
                if (keys_[i] != kEmpty) out->emplace_back(keys_[i], vals_[i]);
            std::sort(out->begin(), out->end());
            return;
        }
        for (size_t x = 0; x < static_cast<size_t>(n_x); ++x) start[x + 1] += start[x];
        out->resize(size_);
        std::vector<size_t> pos(start.begin(), start.end() - 1);
        for (size_t i = 0; i < keys_.size(); ++i)
            if (keys_[i] != kEmpty) (*out)[pos[keys_[i] >> 32]++] = std::make_pair(keys_[i], vals_[i]);
        for (size_t x = 0; x < static_cast<size_t>(n_x); ++x)
            if (start[x + 1] - start[x] > 1) std::sort(out->begin() + start[x], out->begin() + start[x + 1]);
    }

private:
    static constexpr uint64_t kEmpty = ~0ull;
    static uint64_t mix(uint64_t z) {
        z += 0x9e3779b97f4a7c15ull;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    }
    void rehash(size_t cap) {
        std::vector<uint64_t> ok;
        std::vector<int32_t> ov;
        ok.swap(keys_);
        ov.swap(vals_);
        keys_.assign(cap, kEmpty);
        vals_.assign(cap, 0);
        mask_ = cap - 1;
        size_ = 0;
        for (size_t i = 0; i < ok.size(); ++i)
            if (ok[i] != kEmpty) put(ok[i], ov[i]);
    }
    std::vector<uint64_t> keys_;
    std::vector<int32_t> vals_;
    size_t mask_ = 0, size_ = 0;
};

static uint64_t unordered_key(int32_t x, int32_t y) {
    return x < y ? PairMap::key(x, y) : PairMap::key(y, x);
}

// ---------------------------------------------------------------------------
// pinned host staging
// ---------------------------------------------------------------------------
struct Pinned {
    void* ptr = nullptr;
    size_t cap = 0;
    bool ensure(size_t bytes) {
        if (bytes <= cap) return true;
        if (ptr) (void)hipHostFree(ptr);
        ptr = nullptr;
        cap = 0;
        size_t want = bytes + bytes / 4 + 4096;
        if (hipHostMalloc(&ptr, want, hipHostMallocDefault) != hipSuccess) { ptr = nullptr; return false; }
        cap = want;
        return true;
    }
    ~Pinned() { if (ptr) (void)hipHostFree(ptr); }
};

// ---------------------------------------------------------------------------
// GPU batch aligner over the device-resident store
// ---------------------------------------------------------------------------
struct Aligner {
    cm_context* ctx = nullptr;
    const uint8_t* seqs = nullptr;
    const int64_t* offsets = nullptr;
    int32_t n_seqs = 0;
    const cm_params* p = nullptr;
    const std::vector<int32_t>* len = nullptr;
    hipStream_t st = nullptr;
    cm_stats* stats = nullptr;
    // two staging slots so that the host can prepare one batch while the
    // device aligns the other (batches still run in order on one stream)
    struct Slot {
        Pinned h_pairs, h_out, h_err;
        hipEvent_t e0 = nullptr, e1 = nullptr, done = nullptr;
        hipEvent_t scored = nullptr;   // score plane on the host (spans, outside graphs)
        bool have_scores = false;
        bool screened = false;         // screened batch: np candidates, the kept ones aligned
        int64_t kept = 0;
        int64_t np = 0;
        int64_t stride = 0;     // distance between output planes (np, or the capacity)
        int64_t prefix = 0;     // end records copied back with the scores
        bool spans = false;
        double cells = 0;
    } slot[2];
    // captured launch sequences, per (slot, capacity, spans); valid while the
    // buffers they reference stay where they were at capture
    struct Graph {
        int k;
        int64_t cap;
        bool spans;
        hipGraphExec_t exec;
        std::vector<void*> ptrs;
    };
    std::vector<Graph> graphs;
    Pinned sh_pairs, sh_out;   // screen staging (separate from the in-flight slots)
    // end and start cells for the first span_pairs pairs of the next submit
    // only (-1: all); the rest of the batch is scored only
    int64_t span_pairs = -1;
    hipEvent_t scr0 = nullptr, scr1 = nullptr;   // around the device-side screen of a batch

    cm_status init() {
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return fail(CM_EDEVICE, "stream");
        if (hipEventCreate(&scr0) != hipSuccess || hipEventCreate(&scr1) != hipSuccess)
            return fail(CM_EDEVICE, "events");
        for (Slot& sl : slot)
            if (hipEventCreate(&sl.e0) != hipSuccess || hipEventCreate(&sl.e1) != hipSuccess ||
                hipEventCreate(&sl.done) != hipSuccess || hipEventCreate(&sl.scored) != hipSuccess)
                return fail(CM_EDEVICE, "events");
        return CM_OK;
    }
    ~Aligner() {
        // work still in flight (an error return or an exception between a
        // submit and its wait) may write into the pinned staging: let it land
        if (st) (void)hipStreamSynchronize(st);
        for (Graph& g : graphs) (void)hipGraphExecDestroy(g.exec);
        for (Slot& sl : slot) {
            if (sl.e0) (void)hipEventDestroy(sl.e0);
            if (sl.e1) (void)hipEventDestroy(sl.e1);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.scored) (void)hipEventDestroy(sl.scored);
        }
        if (scr0) (void)hipEventDestroy(scr0);
        if (scr1) (void)hipEventDestroy(scr1);
        if (st) (void)hipStreamDestroy(st);
    }

    // Device output of a slot with capacity cap: 5 int32 planes (score,
    // end_a, end_b, start_a, start_b), the live count (graphs), the end-record
    // counter and cap end records of 5 int32.  The host copy holds the score
    // plane, the counter and the first `prefix` records.
    static size_t dev_ints(int64_t cap) { return static_cast<size_t>(cap) * 10 + 8; }
    static int64_t prefix_of(int64_t cap) { return std::min<int64_t>(cap, cap / 64 + 4096); }
    static size_t host_ints(int64_t cap, bool spans) {
        return spans ? static_cast<size_t>(cap) + 4 + 5 * static_cast<size_t>(prefix_of(cap)) : static_cast<size_t>(cap);
    }

    // scores of every pair; end and start cells only where the coverage test
    // can use them (score above mT), compacted on the device
    cm_status enqueue(int32_t* d_pairs, int64_t n, int64_t cap, const int64_t* d_live, int32_t* dsc, bool spans,
                      void* h_out, hipEvent_t scored, int64_t n_span) {
        cm_status s = cmrt::score_batch(ctx, seqs, offsets, n_seqs, d_pairs, n, d_live, p->matrix, p->gap_open,
                                        p->gap_extend, dsc, nullptr, nullptr, st);
        if (s != CM_OK) return s;
        int32_t* h = static_cast<int32_t*>(h_out);
        hipError_t e = hipMemcpyAsync(h, dsc, static_cast<size_t>(cap) * 4, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return hip_fail(e, "scores download");
        if (!spans) return CM_OK;
        // the host can process the scores while the end and start passes run
        if (scored) (void)hipEventRecord(scored, st);
        s = cmrt::end_batch(ctx, seqs, offsets, n_seqs, d_pairs, n_span, d_live, p->matrix, p->gap_open, p->gap_extend,
                            dsc, dsc + cap, dsc + 2 * cap, p->mT, st);
        if (s != CM_OK) return s;
        s = cmrt::span_batch(ctx, seqs, offsets, n_seqs, d_pairs, n_span, d_live, p->matrix, p->gap_open, p->gap_extend,
                             dsc, dsc + cap, dsc + 2 * cap, p->mT, dsc + 3 * cap, dsc + 4 * cap, st);
        if (s != CM_OK) return s;
        uint32_t* d_count = reinterpret_cast<uint32_t*>(dsc + 5 * cap + 4);
        int32_t* d_ent = dsc + 5 * cap + 8;
        hipLaunchKernelGGL(cmdrv::k_zero_u32, dim3(1), dim3(64), 0, st, d_count);
        hipLaunchKernelGGL(cmdrv::k_end_compact, dim3(static_cast<unsigned>((cap + 255) / 256)), dim3(256), 0, st,
                           dsc, cap, d_live, n_span, p->mT, d_count, d_ent);
        e = hipMemcpyAsync(h + cap, d_count, 16, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h + cap + 4, d_ent, static_cast<size_t>(prefix_of(cap)) * 20, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipGetLastError();
        return e == hipSuccess ? CM_OK : hip_fail(e, "results download");
    }

    // Grow slot k's staging for batches up to np pairs now, so that later
    // submits do not reallocate (a device free would wait for in-flight work).
    cm_status reserve(int k, int64_t np, bool spans) {
        Slot& sl = slot[k];
        const size_t pb = static_cast<size_t>(np) * 8;
        if (!ctx->drv[2 * k].ensure(pb) || !ctx->drv[2 * k + 1].ensure(dev_ints(np) * 4) || !sl.h_pairs.ensure(pb) ||
            !sl.h_out.ensure(host_ints(np, spans) * 4) || !sl.h_err.ensure(16))
            return fail(CM_ENOMEM, "cannot stage %lld pairs", static_cast<long long>(np));
        return ctx->graphs ? CM_OK : cmrt::reserve(ctx, np);
    }

    // Enqueue the alignment of np pairs (flat a,b) in slot k.  With spans,
    // the pairs scoring above mT also get end and start cells (EndRec).
    cm_status submit(int k, const int32_t* pairs, int64_t np, bool spans) {
        Slot& sl = slot[k];
        const int64_t n_span = span_pairs >= 0 ? std::min(span_pairs, np) : np;
        span_pairs = -1;
        sl.screened = false;
        sl.np = np;
        sl.stride = np;
        sl.spans = spans;
        sl.cells = 0;
        if (np == 0) return CM_OK;
        double cells = 0;
        for (int64_t q = 0; q < np; ++q)
            cells += static_cast<double>((*len)[pairs[2 * q]]) * (*len)[pairs[2 * q + 1]];
        sl.cells = cells;
        if (ctx->graphs) return submit_graph(k, pairs, np, spans);
        const size_t pb = static_cast<size_t>(np) * 8;
        cmrt::DeviceBuf& d_pairs = ctx->drv[2 * k];
        cmrt::DeviceBuf& d_out = ctx->drv[2 * k + 1];
        if (!d_pairs.ensure(pb) || !d_out.ensure(dev_ints(np) * 4) || !sl.h_pairs.ensure(pb) ||
            !sl.h_out.ensure(host_ints(np, spans) * 4) || !sl.h_err.ensure(16))
            return fail(CM_ENOMEM, "cannot stage %lld pairs", static_cast<long long>(np));
        sl.prefix = prefix_of(np);
        std::memcpy(sl.h_pairs.ptr, pairs, pb);
        hipError_t e = hipMemcpyAsync(d_pairs.ptr, sl.h_pairs.ptr, pb, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "pairs upload");
        (void)hipEventRecord(sl.e0, st);
        return align_staged(k, n_span);
    }

    // The device pair list of slot k is in place (or will be, in stream
    // order): align it and queue the copies back and the slot's events.
    cm_status align_staged(int k, int64_t n_span) {
        Slot& sl = slot[k];
        sl.have_scores = false;
        cm_status s = enqueue(static_cast<int32_t*>(ctx->drv[2 * k].ptr), sl.np, sl.np, nullptr,
                              static_cast<int32_t*>(ctx->drv[2 * k + 1].ptr), sl.spans, sl.h_out.ptr,
                              sl.spans ? sl.scored : nullptr, n_span);
        if (s != CM_OK) return s;
        (void)hipEventRecord(sl.e1, st);
        hipError_t e = hipMemcpyAsync(sl.h_err.ptr, ctx->err_flag, 4, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return hip_fail(e, "flag download");
        (void)hipEventRecord(sl.done, st);
        return CM_OK;
    }

    // Enqueue, in slot k, the representative pairs of a level's merges,
    // generated on the device from one descriptor per merge (see
    // k_rep_product; n_prod pairs in all), followed by n_extra host pairs.
    // cells: the batch's cells (for the statistics).  Not under graphs.
    cm_status submit_product(int k, const std::vector<int64_t>& desc, const std::vector<int32_t>& reps,
                             int64_t n_prod, const int32_t* extra, int64_t n_extra, bool spans, double cells) {
        Slot& sl = slot[k];
        const int64_t np = n_prod + n_extra;
        const int64_t n_span = span_pairs >= 0 ? std::min(span_pairs, np) : np;
        span_pairs = -1;
        sl.screened = false;
        sl.np = np;
        sl.stride = np;
        sl.spans = spans;
        sl.cells = cells;
        if (np == 0) return CM_OK;
        const int n_merges = static_cast<int>(desc.size() / 5);
        if (ctx->graphs || (n_prod > 0 && n_merges < 1)) return fail(CM_EINVAL, "product batch");
        // device: [pairs of the product | extra pairs | descriptors | reps]
        const size_t pb = static_cast<size_t>(np) * 8;
        const size_t xb = static_cast<size_t>(n_extra) * 8, db = desc.size() * 8, rb = reps.size() * 4;
        cmrt::DeviceBuf& d_pairs = ctx->drv[2 * k];
        cmrt::DeviceBuf& d_out = ctx->drv[2 * k + 1];
        if (!d_pairs.ensure(pb + db + rb) || !d_out.ensure(dev_ints(np) * 4) || !sl.h_pairs.ensure(xb + db + rb) ||
            !sl.h_out.ensure(host_ints(np, spans) * 4) || !sl.h_err.ensure(16))
            return fail(CM_ENOMEM, "cannot stage %lld pairs", static_cast<long long>(np));
        sl.prefix = prefix_of(np);
        char* h = static_cast<char*>(sl.h_pairs.ptr);
        if (xb) std::memcpy(h, extra, xb);
        if (db) std::memcpy(h + xb, desc.data(), db);
        if (rb) std::memcpy(h + xb + db, reps.data(), rb);
        char* dp = static_cast<char*>(d_pairs.ptr);
        hipError_t e = hipMemcpyAsync(dp + static_cast<size_t>(n_prod) * 8, h, xb + db + rb, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "pairs upload");
        (void)hipEventRecord(sl.e0, st);
        if (n_prod > 0)
            hipLaunchKernelGGL(cmdrv::k_rep_product, dim3(static_cast<unsigned>((n_prod + 255) / 256)), dim3(256), 0,
                               st, reinterpret_cast<const int64_t*>(dp + pb), n_merges,
                               reinterpret_cast<const int32_t*>(dp + pb + db), n_prod, reinterpret_cast<int32_t*>(dp));
        return align_staged(k, n_span);
    }

    // Same sequence as a replayed hipGraph: fixed capacity (a power of two),
    // live pair count read from device memory by the plan kernel.
    cm_status submit_graph(int k, const int32_t* pairs, int64_t np, bool spans) {
        Slot& sl = slot[k];
        int64_t cap = 1024;
        while (cap < np) cap *= 2;
        sl.stride = cap;
        sl.prefix = prefix_of(cap);
        const size_t pb = static_cast<size_t>(cap) * 8;
        cmrt::DeviceBuf& d_pairs = ctx->drv[2 * k];
        cmrt::DeviceBuf& d_out = ctx->drv[2 * k + 1];
        if (!d_pairs.ensure(pb) || !d_out.ensure(dev_ints(cap) * 4) || !sl.h_pairs.ensure(pb) ||
            !sl.h_out.ensure(host_ints(cap, true) * 4) || !sl.h_err.ensure(16))
            return fail(CM_ENOMEM, "cannot stage %lld pairs", static_cast<long long>(cap));
        cm_status s = cmrt::reserve(ctx, cap);
        if (s != CM_OK) return s;
        int32_t* dsc = static_cast<int32_t*>(d_out.ptr);
        int64_t* d_live = reinterpret_cast<int64_t*>(dsc + 5 * cap);
        int64_t* h_live = reinterpret_cast<int64_t*>(static_cast<char*>(sl.h_err.ptr) + 8);
        const std::vector<void*> ptrs = {d_pairs.ptr, d_out.ptr, ctx->keys.ptr, ctx->keys_alt.ptr, ctx->vals.ptr,
                                         ctx->vals_alt.ptr, ctx->sort_tmp.ptr, sl.h_pairs.ptr, sl.h_out.ptr,
                                         sl.h_err.ptr, ctx->bnd.ptr, ctx->over.ptr};
        Graph* g = nullptr;
        for (size_t q = 0; q < graphs.size(); ++q) {
            if (graphs[q].ptrs != ptrs) {        // stale: a referenced buffer moved
                (void)hipGraphExecDestroy(graphs[q].exec);
                graphs.erase(graphs.begin() + static_cast<long>(q));
                --q;
                continue;
            }
            if (graphs[q].k == k && graphs[q].cap == cap && graphs[q].spans == spans) g = &graphs[q];
        }
        if (!g) {
            const bool timed = ctx->timer.on;
            ctx->timer.on = false;               // no timing events inside a captured sequence
            hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) { ctx->timer.on = timed; return hip_fail(e, "begin capture"); }
            (void)hipMemcpyAsync(d_live, h_live, 8, hipMemcpyHostToDevice, st);
            (void)hipMemcpyAsync(d_pairs.ptr, sl.h_pairs.ptr, pb, hipMemcpyHostToDevice, st);
            s = enqueue(static_cast<int32_t*>(d_pairs.ptr), cap, cap, d_live, dsc, spans, sl.h_out.ptr, nullptr, cap);
            (void)hipMemcpyAsync(sl.h_err.ptr, ctx->err_flag, 4, hipMemcpyDeviceToHost, st);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(st, &graph);
            ctx->timer.on = timed;
            if (s != CM_OK) { if (graph) (void)hipGraphDestroy(graph); return s; }
            if (e != hipSuccess) return hip_fail(e, "end capture");
            hipGraphExec_t exec = nullptr;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return hip_fail(e, "instantiate");
            graphs.push_back(Graph{k, cap, spans, exec, ptrs});
            g = &graphs.back();
        }
        *h_live = np;
        std::memcpy(sl.h_pairs.ptr, pairs, static_cast<size_t>(np) * 8);
        (void)hipEventRecord(sl.e0, st);
        hipError_t e = hipGraphLaunch(g->exec, st);
        if (e != hipSuccess) return hip_fail(e, "graph launch");
        (void)hipEventRecord(sl.e1, st);
        (void)hipEventRecord(sl.done, st);
        (void)hipEventRecord(sl.scored, st);
        sl.have_scores = false;
        return CM_OK;
    }

    // Screened batch in slot 0 (not under graph capture): the device screens
    // the np candidates (guard[i] != 0 bypasses the screen), compacts the kept
    // pairs in order and aligns them with end and start cells.  wait_scores()
    // then returns the kept pairs' scores in order and keep_flags() the
    // decision for every candidate.
    // The representative pairs of a screened wave as merge descriptors (see
    // k_rep_product_guard): counts holds each representative's cluster size.
    struct Product {
        const std::vector<int64_t>* desc;
        const std::vector<int32_t>* reps;
        const std::vector<int32_t>* counts;
        int64_t min_product;
    };
    // pairs and guard from the host, or (prod) generated on the device
    cm_status submit_screened(const int32_t* pairs, const uint8_t* guard, int64_t np, const cm_screen* scr,
                              const uint16_t* feat, float tau, const Product* prod = nullptr) {
        Slot& sl = slot[0];
        sl.np = np;
        sl.stride = np;
        sl.spans = true;
        sl.cells = 0;
        sl.screened = true;
        sl.kept = 0;
        sl.have_scores = false;
        sl.prefix = prefix_of(np);
        if (np == 0) return CM_OK;
        const size_t pb = static_cast<size_t>(np) * 8;
        size_t tmp = 0;
        hipError_t e = hipcub::DeviceSelect::Flagged(nullptr, tmp, static_cast<uint64_t*>(nullptr),
                                                     static_cast<uint8_t*>(nullptr), static_cast<uint64_t*>(nullptr),
                                                     static_cast<int64_t*>(nullptr), static_cast<int>(np));
        if (e != hipSuccess) return hip_fail(e, "select size query");
        // screen scratch: logits, guard flags, keep flags, kept count, select temp
        const size_t o_guard = static_cast<size_t>(np) * 4, o_keep = o_guard + np;
        const size_t o_count = (o_keep + np + 15) & ~static_cast<size_t>(15), o_tmp = o_count + 16;
        cmrt::DeviceBuf& d_pairs = ctx->drv[0];
        cmrt::DeviceBuf& d_out = ctx->drv[1];
        cmrt::DeviceBuf& d_kept = ctx->drv[4];
        cmrt::DeviceBuf& d_scr = ctx->drv[11];
        const size_t hb = host_ints(np, true) * 4;
        // with a product: [pairs | descriptors | reps | counts] on the device
        const size_t db = prod ? prod->desc->size() * 8 : 0, rb = prod ? prod->reps->size() * 4 : 0;
        const size_t up = prod ? db + 2 * rb : pb + np;   // bytes staged on the host
        if (prod && (prod->counts->size() != prod->reps->size() || prod->desc->size() < 5))
            return fail(CM_EINVAL, "screened product batch");
        if (!d_pairs.ensure(pb + db + 2 * rb) || !d_out.ensure(dev_ints(np) * 4) || !d_kept.ensure(pb) ||
            !d_scr.ensure(o_tmp + tmp) || !sl.h_pairs.ensure(up) || !sl.h_out.ensure(hb + np) ||
            !sl.h_err.ensure(16))
            return fail(CM_ENOMEM, "cannot stage %lld screened pairs", static_cast<long long>(np));
        char* scr_base = static_cast<char*>(d_scr.ptr);
        float* z = reinterpret_cast<float*>(scr_base);
        uint8_t* d_guard = reinterpret_cast<uint8_t*>(scr_base + o_guard);
        uint8_t* d_keep = reinterpret_cast<uint8_t*>(scr_base + o_keep);
        int64_t* d_count = reinterpret_cast<int64_t*>(scr_base + o_count);
        char* h = static_cast<char*>(sl.h_pairs.ptr);
        char* dp = static_cast<char*>(d_pairs.ptr);
        if (prod) {
            std::memcpy(h, prod->desc->data(), db);
            std::memcpy(h + db, prod->reps->data(), rb);
            std::memcpy(h + db + rb, prod->counts->data(), rb);
            e = hipMemcpyAsync(dp + pb, h, up, hipMemcpyHostToDevice, st);
        } else {
            std::memcpy(h, pairs, pb);
            std::memcpy(h + pb, guard, static_cast<size_t>(np));
            e = hipMemcpyAsync(dp, h, pb, hipMemcpyHostToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(d_guard, h + pb, static_cast<size_t>(np), hipMemcpyHostToDevice, st);
        }
        if (e != hipSuccess) return hip_fail(e, "pairs upload");
        (void)hipEventRecord(sl.e0, st);
        if (prod)
            hipLaunchKernelGGL(cmdrv::k_rep_product_guard, dim3(static_cast<unsigned>((np + 255) / 256)), dim3(256),
                               0, st, reinterpret_cast<const int64_t*>(dp + pb),
                               static_cast<int>(prod->desc->size() / 5), reinterpret_cast<const int32_t*>(dp + pb + db),
                               reinterpret_cast<const int32_t*>(dp + pb + db + rb), prod->min_product, np,
                               reinterpret_cast<int32_t*>(dp), d_guard);
        (void)hipEventRecord(scr0, st);
        cm_status s = cm_screen_infer(scr, feat, static_cast<const int32_t*>(d_pairs.ptr), np, z, st);
        if (s != CM_OK) return s;
        hipLaunchKernelGGL(cmdrv::k_keep, dim3(static_cast<unsigned>((np + 255) / 256)), dim3(256), 0, st, z, d_guard,
                           tau, np, d_keep);
        e = hipcub::DeviceSelect::Flagged(scr_base + o_tmp, tmp, static_cast<const uint64_t*>(d_pairs.ptr), d_keep,
                                          static_cast<uint64_t*>(d_kept.ptr), d_count, static_cast<int>(np), st);
        if (e != hipSuccess) return hip_fail(e, "screen select");
        (void)hipEventRecord(scr1, st);
        e = hipMemcpyAsync(static_cast<char*>(sl.h_out.ptr) + hb, d_keep, static_cast<size_t>(np),
                           hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return hip_fail(e, "keep flags download");
        s = enqueue(static_cast<int32_t*>(d_kept.ptr), np, np, d_count, static_cast<int32_t*>(d_out.ptr), true,
                    sl.h_out.ptr, sl.scored, np);
        if (s != CM_OK) return s;
        (void)hipEventRecord(sl.e1, st);
        e = hipMemcpyAsync(sl.h_err.ptr, ctx->err_flag, 4, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return hip_fail(e, "flag download");
        (void)hipEventRecord(sl.done, st);
        return CM_OK;
    }
    // keep decisions of the screened batch in slot 0 (valid after wait_scores)
    const uint8_t* keep_flags() const {
        return static_cast<const uint8_t*>(slot[0].h_out.ptr) + host_ints(slot[0].np, true) * 4;
    }
    // device seconds of the last batch's screen (after wait_scores)
    double screen_seconds() {
        float ms = 0.f;
        return hipEventElapsedTime(&ms, scr0, scr1) == hipSuccess ? ms * 1e-3 : 0.0;
    }
    // the screened batch aligned `kept` pairs of `cells` cells (for the statistics)
    void set_kept(int64_t kept, double cells) {
        slot[0].kept = kept;
        slot[0].cells = cells;
    }

    // Scores of slot k (submitted with spans) into out, as soon as the score
    // pass is back; wait() later adds the end records.
    cm_status wait_scores(int k, std::vector<int32_t>& out) {
        Slot& sl = slot[k];
        out.resize(static_cast<size_t>(sl.np));
        if (sl.np == 0) return CM_OK;
        hipError_t e = hipEventSynchronize(sl.scored);
        if (e != hipSuccess) return hip_fail(e, "score pass");
        std::memcpy(out.data(), sl.h_out.ptr, static_cast<size_t>(sl.np) * 4);
        sl.have_scores = true;
        return CM_OK;
    }

    // Wait for slot k: scores into out, and (with spans) the end records of
    // the pairs scoring above mT, sorted by pair index, into ends.
    cm_status wait(int k, std::vector<int32_t>& out, std::vector<EndRec>* ends = nullptr) {
        Slot& sl = slot[k];
        if (!sl.have_scores) out.resize(static_cast<size_t>(sl.np));
        if (ends) ends->clear();
        if (sl.np == 0) return CM_OK;
        hipError_t e = hipEventSynchronize(sl.done);
        if (e != hipSuccess) return hip_fail(e, "alignment batch");
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, sl.e0, sl.e1);
        if (*static_cast<const uint32_t*>(sl.h_err.ptr) != 0) {
            cm_status s = cm_context_sync(ctx);   // clears the flag and describes it
            return s != CM_OK ? s : fail(CM_ERANGE, "device flagged bad input");
        }
        const int32_t* h = static_cast<const int32_t*>(sl.h_out.ptr);
        if (!sl.have_scores) std::memcpy(out.data(), h, static_cast<size_t>(sl.np) * 4);
        sl.have_scores = false;
        if (sl.spans && ends) {
            const int64_t cnt = static_cast<uint32_t>(h[sl.stride]);
            ends->resize(static_cast<size_t>(cnt));
            const int64_t head = std::min(cnt, sl.prefix);
            std::memcpy(ends->data(), h + sl.stride + 4, static_cast<size_t>(head) * 20);
            if (cnt > head) {   // more records than the prefix copy held
                const int32_t* d_ent = static_cast<const int32_t*>(ctx->drv[2 * k + 1].ptr) + 5 * sl.stride + 8;
                e = hipMemcpy(ends->data() + head, d_ent + 5 * head, static_cast<size_t>(cnt - head) * 20,
                              hipMemcpyDeviceToHost);
                if (e != hipSuccess) return hip_fail(e, "end records download");
            }
            std::sort(ends->begin(), ends->end(), [](const EndRec& a, const EndRec& b) { return a.idx < b.idx; });
        }
        cmrt::drain_timers(ctx, false);
        stats->t_gpu_s += ms * 1e-3;
        stats->waves += 1;
        stats->aligned_pairs += sl.screened ? sl.kept : sl.np;
        stats->aligned_cells += sl.cells;
        sl.np = 0;
        sl.screened = false;
        return CM_OK;
    }

    // Screen logits for np pairs (flat a,b) -> keep[k] = logit >= tau.  Synchronous.
    cm_status screen(const cm_screen* scr, const uint16_t* feat, float tau, const int32_t* pairs, int64_t np,
                     std::vector<uint8_t>& keep) {
        keep.assign(static_cast<size_t>(np), 1);
        if (np == 0) return CM_OK;
        cmrt::DeviceBuf& d_pairs = ctx->drv[8];
        cmrt::DeviceBuf& d_z = ctx->drv[9];
        if (!d_pairs.ensure(np * 8) || !d_z.ensure(np * 4) || !sh_pairs.ensure(np * 8) || !sh_out.ensure(np * 4))
            return fail(CM_ENOMEM, "screen staging");
        std::memcpy(sh_pairs.ptr, pairs, np * 8);
        hipError_t e = hipMemcpyAsync(d_pairs.ptr, sh_pairs.ptr, np * 8, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "screen upload");
        cm_status s = cm_screen_infer(scr, feat, static_cast<const int32_t*>(d_pairs.ptr), np,
                                      static_cast<float*>(d_z.ptr), st);
        if (s != CM_OK) return s;
        e = hipMemcpyAsync(sh_out.ptr, d_z.ptr, np * 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "screen inference");
        const float* z = static_cast<const float*>(sh_out.ptr);
        for (int64_t k = 0; k < np; ++k) keep[k] = z[k] >= tau;
        return CM_OK;
    }

    cm_status run(const int32_t* pairs, int64_t np, bool spans, std::vector<int32_t>& out) {
        cm_status s = submit(0, pairs, np, spans);
        if (s != CM_OK) return s;
        return wait(0, out);
    }
};

// ---------------------------------------------------------------------------
// clusters and the Algorithm 1 replay
// ---------------------------------------------------------------------------
// open-addressing set of non-negative int32 (element indices)
class IdSet {
public:
    bool has(int32_t x) const {
        if (slots_.empty()) return false;
        for (size_t i = slot(x);; i = (i + 1) & mask_) {
            const int32_t v = slots_[i];
            if (v == x) return true;
            if (v < 0) return false;
        }
    }
    // true when x was not in the set
    bool insert(int32_t x) {
        if (2 * (size_ + 1) > slots_.size()) grow();
        size_t i = slot(x);
        while (slots_[i] >= 0) {
            if (slots_[i] == x) return false;
            i = (i + 1) & mask_;
        }
        slots_[i] = x;
        ++size_;
        return true;
    }
    void clear() {
        if (size_) std::fill(slots_.begin(), slots_.end(), -1);
        size_ = 0;
    }

private:
    size_t slot(int32_t x) const {
        return static_cast<size_t>((static_cast<uint32_t>(x) * 2654435761u) >> 7) & mask_;
    }
    void grow() {
        std::vector<int32_t> old;
        old.swap(slots_);
        slots_.assign(old.empty() ? 16 : 2 * old.size(), -1);
        mask_ = slots_.size() - 1;
        size_ = 0;
        for (int32_t v : old)
            if (v >= 0) insert(v);
    }
    std::vector<int32_t> slots_;
    size_t mask_ = 0, size_ = 0;
};

struct Cluster {
    int32_t rep;
    std::vector<int32_t> objs;
    IdSet mem;
    void add(int32_t x) {
        if (mem.insert(x)) objs.push_back(x);
    }
    bool has(int32_t x) const { return mem.has(x); }
};

// representative-pair outcome bits
constexpr uint8_t kSim = 1, kT21 = 2, kT12 = 4;

// One step of Algorithm 1 that changes memberships.  The order of these
// events and the clusters that survive depend only on representative scores:
// ExchangeSimilar changes member lists, never the merged flags or the loop.
enum EventType : uint8_t { kAbsorb21 = 0, kAbsorb12 = 1, kExchange = 2 };
struct Event {
    uint8_t type;
    int32_t i, j;             // cluster positions in the first / second set
};

struct MergeJob {
    int32_t set1, set2, out;
    size_t rep_off = 0;           // offset of this merge's rep pairs in the level batch
    std::vector<Event> events;
    size_t next = 0;              // next event to apply
    bool done = false;
    std::vector<int32_t> result;  // clusters of the new set, in Algorithm 1 order
};

// A previous clustering of elements 0..n_prev-1 (host arrays, validated by the
// caller) and the scores it already knows.
struct PrevClustering {
    int32_t n_prev = 0, n_clusters = 0;
    const int32_t* reps = nullptr;
    const int64_t* member_offsets = nullptr;
    const int32_t* members = nullptr;
    int64_t n_known = 0;
    const int32_t* known_pairs = nullptr;
    const int32_t* known_scores = nullptr;
};

class Driver {
public:
    // classify elements prev.n_prev..n-1 against `prev` instead of clustering from singletons
    void set_prev(const PrevClustering* prev) { prev_ = prev; }
    Driver(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n, const cm_params* p,
           const cm_screen* scr)
        : ctx_(ctx), n_(n), p_(*p), scr_(scr) {
        al_.ctx = ctx;
        al_.seqs = seqs;
        al_.offsets = offsets;
        al_.n_seqs = n;
        al_.p = &p_;
        al_.len = &len_;
        al_.stats = &st_;
        const char* lg = getenv("CM_LOG");
        log_ = lg && *lg && *lg != '0';
    }

    cm_status run(cm_result** out);

private:
    cm_status load_lengths();
    // A level is its representative stage (one wave, events simulated) and
    // its exchange stage (replay passes, each blocked pass followed by the
    // alignment of the pairs it requested).  Exchanges move members between
    // clusters and never change which clusters survive or their
    // representatives, so the next level's representative pairs are fixed
    // before a level's exchanges end: a level's first requests can ride in
    // the next level's representative batch (carry_), and its exchange stage
    // then finishes after that wave, before the next level's replay.
    int rep_chunks(std::vector<MergeJob>& jobs, size_t* total);   // sets rep_off
    bool can_carry(std::vector<MergeJob>& next);
    cm_status rep_stage(std::vector<MergeJob>& jobs, int level);
    bool replay_pass(std::vector<MergeJob>& jobs, std::vector<int32_t>& req);
    // requests in req (may be empty) aligned, then replay until no merge is blocked
    cm_status exchange_stage(std::vector<MergeJob>& jobs, std::vector<int32_t>& req, int level);
    // the representative wave of a level: every pair in one batch (with the
    // screen when it covers this stage), or the columns in chunks
    cm_status wave_a(std::vector<MergeJob>& jobs, size_t total);
    cm_status wave_a_chunked(std::vector<MergeJob>& jobs, int chunks);
    // a representative pair of clusters this large is aligned without the screen
    bool rep_guarded(int32_t a, int32_t b) const {
        const int64_t prod = static_cast<int64_t>(cl_[a].objs.size()) * cl_[b].objs.size();
        return p_.screen_min_product > 0 && prod >= p_.screen_min_product;
    }
    void simulate(MergeJob& job, const uint8_t* bits);
    // apply events until done or blocked on missing scores; true when blocked
    bool replay(MergeJob& job, std::vector<int32_t>& req);
    void request_exchange(const Cluster& c1, const Cluster& c2, std::vector<int32_t>& req);
    void speculate(MergeJob& job, std::vector<int32_t>& req);
    cm_status align_requests(std::vector<int32_t>& req);
    cm_status final_stage(cm_result* res);

    // Screen decision for an exchange pair: 1 keep, 0 dropped, -1 not yet
    // screened (always 1 when the exchange stage is not screened)
    int decision(uint64_t k) const {
        if (!screened(CM_STAGE_EXCHANGE)) return 1;
        int32_t d;
        return decisions_.find(k, &d) ? d : -1;
    }
    // Score of a member-vs-representative pair as the replay sees it: -1 for
    // a pair the screen dropped (never aligned, not similar)
    bool score_of(int32_t x, int32_t y, int32_t* s) const {
        const uint64_t k = unordered_key(x, y);
        const int d = decision(k);
        if (d < 0) return false;
        if (d == 0) { *s = -1; return true; }
        return cache_.find(k, s);
    }
    bool screened(uint32_t stage) const { return scr_ && (p_.screen_stages & stage); }
    // split a request list into screen-kept pairs (returned in place) and
    // dropped pairs (recorded); no-op when the stage is not screened
    cm_status apply_screen(uint32_t stage, std::vector<int32_t>& pairs, std::vector<uint8_t>* keep_out);

    cm_context* ctx_;
    int32_t n_;
    cm_params p_;
    const cm_screen* scr_ = nullptr;
    cmrt::DeviceBuf* feat_ = nullptr;  // store features when screening
    PairMap decisions_;                // exchange-stage screen decisions
    Aligner al_;
    cm_stats st_{};
    bool log_ = false;
    const PrevClustering* prev_ = nullptr;
    // speculate's scratch: slot per touched cluster (-1: none), lists and sets
    std::vector<int32_t> spec_slot_;
    std::vector<std::vector<int32_t>> spec_list_;
    std::vector<IdSet> spec_set_;
    double t_spec_ = 0;   // host seconds in speculate (logging)
    // representative pairs aligned but not compared by Algorithm 1 (logging):
    // past a row's break, and against already-absorbed columns
    int64_t spec_after_break_ = 0, spec_merged_col_ = 0;
    double t_prep_ = 0, t_submit_ = 0, t_wait_ = 0, t_bits_ = 0;   // wave A phases (logging)
    std::vector<int32_t> len_;
    std::vector<Cluster> cl_;
    std::vector<std::vector<int32_t>> sets_;
    PairMap cache_;    // unordered pair -> score
    std::vector<std::pair<uint64_t, int32_t>> cand_;   // merge-stage scores (params.record_candidates)
    PairMap pending_;  // pairs requested in the current wave
    std::vector<int32_t> carry_;   // a level's first exchange requests, aligned with the next representative wave
};

cm_status Driver::load_lengths() {
    std::vector<int64_t> off(static_cast<size_t>(n_) + 1);
    hipError_t e = hipMemcpy(off.data(), al_.offsets, off.size() * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "offsets download");
    len_.resize(n_);
    for (int32_t k = 0; k < n_; ++k) {
        const int64_t L = off[k + 1] - off[k];
        if (L < 0 || L > CM_MAX_LEN) return fail(CM_ERANGE, "sequence %d has length %lld", k, static_cast<long long>(L));
        len_[k] = static_cast<int32_t>(L);
    }
    return CM_OK;
}

void Driver::request_exchange(const Cluster& c1, const Cluster& c2, std::vector<int32_t>& req) {
    auto want = [&](int32_t m, int32_t rep) {
        int32_t s;
        const uint64_t k = unordered_key(m, rep);
        const int d = decision(k);
        if (d == 0 || (d == 1 && cache_.find(k, &s)) || pending_.find(k, &s)) return;
        pending_.put(k, 0);
        req.push_back(rep);   // the representative is the query: one query per exchange
        req.push_back(m);
    };
    for (int32_t m : c2.objs)
        if (!c1.has(m)) want(m, c1.rep);
    for (int32_t m : c1.objs)
        if (!c2.has(m)) want(m, c2.rep);
}

// Algorithm 1's events from the outcome matrix of a merge (rows: clusters of
// the first set, columns: clusters of the second; bits[i * n2 + j] holds
// similarity and the two transitivity directions).  Row i meets the columns
// still live when it starts, up to its first absorber: the first live column
// that is similar and whose cluster absorbs row i's (Section 4's test); there
// its cluster is absorbed and its comparisons end.  Before that, a similar
// column either is absorbed by row i (it leaves the live mask) or exchanges
// members with it.  A row only retires columns behind its own scan, so the
// first-absorber scan over the mask at the row's start is exact.
void Driver::simulate(MergeJob& job, const uint8_t* bits) {
    const std::vector<int32_t>& cs1 = sets_[job.set1];
    const std::vector<int32_t>& cs2 = sets_[job.set2];
    const size_t n2 = cs2.size();
    std::vector<uint8_t> retired(n2, 0);     // second-set clusters absorbed so far
    for (size_t i = 0; i < cs1.size(); ++i) {
        const uint8_t* row = bits + i * n2;
        size_t stop = n2;                    // first absorber of row i (n2: none)
        for (size_t j = 0; j < n2; ++j)
            if (!retired[j] && (row[j] & kSim) && (row[j] & kT21)) { stop = j; break; }
        const size_t end = stop < n2 ? stop + 1 : n2;
        const int32_t rep1 = cl_[cs1[i]].rep;
        for (size_t j = 0; j < end; ++j) {
            if (retired[j]) { ++spec_merged_col_; continue; }
            ++st_.rep_comparisons;
            st_.required_cells += static_cast<double>(len_[rep1]) * len_[cl_[cs2[j]].rep];
            if (!(row[j] & kSim)) continue;
            const int32_t ii = static_cast<int32_t>(i), jj = static_cast<int32_t>(j);
            if (j == stop) {
                job.events.push_back({kAbsorb21, ii, jj});
            } else if (row[j] & kT12) {
                job.events.push_back({kAbsorb12, ii, jj});
                retired[j] = 1;
            } else {
                job.events.push_back({kExchange, ii, jj});
            }
        }
        if (stop < n2) spec_after_break_ += static_cast<int64_t>(n2 - stop - 1);   // aligned, never compared
        else job.result.push_back(cs1[i]);
    }
    for (size_t j = 0; j < n2; ++j)
        if (!retired[j]) job.result.push_back(cs2[j]);
}

// The replay is blocked at event job.next (its own pairs are requested).
// Walk the remaining events with simulated member lists: full merges add the
// absorbed members exactly; an exchange adds every member whose score is
// known similar or not yet known (a superset of what it will add).  Pairs of
// every later exchange are requested against these lists, so that most of the
// merge completes after one more wave.
void Driver::speculate(MergeJob& job, std::vector<int32_t>& req) {
    const std::vector<int32_t>& cs1 = sets_[job.set1];
    const std::vector<int32_t>& cs2 = sets_[job.set2];
    // simulated additions per cluster of the two sets: a slot per cluster
    // touched, its list in insertion order and its set (reused across calls)
    const size_t n_slots = cs1.size() + cs2.size();
    if (spec_list_.size() < n_slots) { spec_list_.resize(n_slots); spec_set_.resize(n_slots); }
    if (spec_slot_.size() < cl_.size()) spec_slot_.resize(cl_.size(), -1);
    std::vector<int32_t> touched;
    auto slot_of = [&](int32_t cid) {
        if (spec_slot_[cid] < 0) {
            spec_slot_[cid] = static_cast<int32_t>(touched.size());
            touched.push_back(cid);
        }
        return spec_slot_[cid];
    };
    auto has = [&](int32_t cid, int32_t m) {
        if (cl_[cid].has(m)) return true;
        const int32_t sl = spec_slot_[cid];
        return sl >= 0 && spec_set_[sl].has(m);
    };
    auto add = [&](int32_t cid, int32_t m) {
        if (cl_[cid].has(m)) return;
        const int32_t sl = slot_of(cid);
        if (spec_set_[sl].insert(m)) spec_list_[sl].push_back(m);
    };
    // members of a cluster with its simulated additions, visited in order
    auto for_members = [&](int32_t cid, auto&& f) {
        for (int32_t x : cl_[cid].objs) f(x);
        const int32_t sl = spec_slot_[cid];
        if (sl >= 0)
            for (int32_t x : spec_list_[sl]) f(x);
    };
    auto want = [&](int32_t m, int32_t rep) {
        int32_t sc;
        const uint64_t k = unordered_key(m, rep);
        const int d = decision(k);
        if (d == 0) return false;
        if (d == 1 && cache_.find(k, &sc)) return sc >= p_.T;
        if (!pending_.find(k, &sc)) {
            pending_.put(k, 0);
            req.push_back(rep);
            req.push_back(m);
        }
        return true;   // unknown: assume similar
    };
    std::vector<int32_t> to_a, to_b;
    for (size_t k = job.next; k < job.events.size(); ++k) {
        const Event& ev = job.events[k];
        const int32_t a = cs1[ev.i], b = cs2[ev.j];
        // a and b are distinct clusters and the slot lists are sized before
        // the loop, so one cluster's members can be read while adding to the other
        if (ev.type == kAbsorb21) {
            for_members(a, [&](int32_t x) { add(b, x); });
        } else if (ev.type == kAbsorb12) {
            for_members(b, [&](int32_t x) { add(a, x); });
        } else {
            const int32_t ra = cl_[a].rep, rb = cl_[b].rep;
            to_a.clear();
            to_b.clear();
            for_members(b, [&](int32_t x) {
                if (!has(a, x) && want(x, ra)) to_a.push_back(x);
            });
            for_members(a, [&](int32_t x) {
                if (!has(b, x) && want(x, rb)) to_b.push_back(x);
            });
            for (int32_t x : to_a) add(a, x);
            for (int32_t x : to_b) add(b, x);
        }
    }
    for (size_t q = 0; q < touched.size(); ++q) {
        spec_list_[q].clear();
        spec_set_[q].clear();
        spec_slot_[touched[q]] = -1;
    }
}

bool Driver::replay(MergeJob& job, std::vector<int32_t>& req) {
    const std::vector<int32_t>& cs1 = sets_[job.set1];
    const std::vector<int32_t>& cs2 = sets_[job.set2];
    std::vector<int32_t> add1, add2;
    while (job.next < job.events.size()) {
        Event& ev = job.events[job.next];
        Cluster& c1 = cl_[cs1[ev.i]];
        Cluster& c2 = cl_[cs2[ev.j]];
        if (ev.type == kAbsorb21) {
            for (int32_t x : c1.objs) c2.add(x);
            ++st_.full_merges;
            ++job.next;
            continue;
        }
        if (ev.type == kAbsorb12) {
            for (int32_t x : c2.objs) c1.add(x);
            ++st_.full_merges;
            ++job.next;
            continue;
        }
        // ExchangeSimilar: every member-vs-representative score must be known
        add1.clear();
        add2.clear();
        bool missing = false;
        int64_t tests = 0;
        double test_cells = 0;
        for (int32_t m : c2.objs) {
            if (c1.has(m)) continue;
            ++tests;
            test_cells += static_cast<double>(len_[m]) * len_[c1.rep];
            int32_t s;
            if (!score_of(m, c1.rep, &s)) { missing = true; continue; }
            if (s >= p_.T) add1.push_back(m);
        }
        for (int32_t m : c1.objs) {
            if (c2.has(m)) continue;
            ++tests;
            test_cells += static_cast<double>(len_[m]) * len_[c2.rep];
            int32_t s;
            if (!score_of(m, c2.rep, &s)) { missing = true; continue; }
            if (s >= p_.T) add2.push_back(m);
        }
        if (missing) {
            const auto sp0 = Clock::now();
            speculate(job, req);
            t_spec_ += secs(sp0, Clock::now());
            return true;
        }
        st_.exchange_alignments += tests;
        st_.required_cells += test_cells;
        ++st_.exchanges;
        for (int32_t m : add1) c1.add(m);
        for (int32_t m : add2) c2.add(m);
        ++job.next;
    }
    job.done = true;
    return false;
}

cm_status Driver::apply_screen(uint32_t stage, std::vector<int32_t>& pairs, std::vector<uint8_t>* keep_out) {
    if (!screened(stage)) {
        if (keep_out) keep_out->assign(pairs.size() / 2, 1);
        return CM_OK;
    }
    std::vector<uint8_t> keep;
    const auto t0 = Clock::now();
    cm_status s = al_.screen(scr_, static_cast<const uint16_t*>(feat_->ptr), p_.screen_tau, pairs.data(),
                             static_cast<int64_t>(pairs.size() / 2), keep);
    if (s != CM_OK) return s;
    st_.t_screen_s += secs(t0, Clock::now());
    st_.screened_pairs += static_cast<int64_t>(pairs.size() / 2);
    size_t w = 0;
    for (size_t k = 0; k < keep.size(); ++k) {
        if (stage == CM_STAGE_EXCHANGE)
            decisions_.put(unordered_key(pairs[2 * k], pairs[2 * k + 1]), keep[k] ? 1 : 0);
        if (keep[k]) {
            pairs[2 * w] = pairs[2 * k];
            pairs[2 * w + 1] = pairs[2 * k + 1];
            ++w;
        } else {
            ++st_.screened_out;
        }
    }
    pairs.resize(2 * w);
    if (keep_out) keep_out->swap(keep);
    return CM_OK;
}

cm_status Driver::align_requests(std::vector<int32_t>& req) {
    cm_status s0 = apply_screen(CM_STAGE_EXCHANGE, req, nullptr);
    if (s0 != CM_OK) return s0;
    {   // kept pairs whose score is already known need no alignment
        size_t w = 0;
        int32_t sc;
        for (size_t k = 0; k < req.size() / 2; ++k)
            if (!cache_.find(unordered_key(req[2 * k], req[2 * k + 1]), &sc)) {
                req[2 * w] = req[2 * k];
                req[2 * w + 1] = req[2 * k + 1];
                ++w;
            }
        req.resize(2 * w);
    }
    std::vector<int32_t> out;
    cm_status s = al_.run(req.data(), static_cast<int64_t>(req.size() / 2), false, out);
    if (s != CM_OK) return s;
    for (size_t k = 0; k < out.size(); ++k) cache_.put(unordered_key(req[2 * k], req[2 * k + 1]), out[k]);
    if (p_.record_candidates)
        for (size_t k = 0; k < out.size(); ++k) cand_.emplace_back(unordered_key(req[2 * k], req[2 * k + 1]), out[k]);
    pending_.clear();
    req.clear();
    return CM_OK;
}

int Driver::rep_chunks(std::vector<MergeJob>& jobs, size_t* total_out) {
    size_t total = 0;
    for (MergeJob& job : jobs) {
        job.rep_off = total;
        total += sets_[job.set1].size() * sets_[job.set2].size();
    }
    if (total_out) *total_out = total;
    // a large representative product goes in column chunks (not under a
    // screen of this stage): default about 2^25 pairs per chunk, at most 8
    // (each chunk pays the latency of its end-cell and start-cell launches,
    // so only waves of tens of millions of pairs gain)
    int chunks = 1;
    if ((!screened(CM_STAGE_REP) || !ctx_->graphs) && p_.rep_chunk_pairs >= 0) {
        const int64_t per = p_.rep_chunk_pairs > 0 ? p_.rep_chunk_pairs : (int64_t(1) << 25);
        chunks = static_cast<int>(std::min<int64_t>(8, (static_cast<int64_t>(total) + per - 1) / per));
        if (chunks < 1) chunks = 1;
    }
    return chunks;
}

bool Driver::can_carry(std::vector<MergeJob>& next) {
    return !screened(CM_STAGE_REP) && !screened(CM_STAGE_EXCHANGE) && !ctx_->graphs && rep_chunks(next, nullptr) == 1;
}

cm_status Driver::rep_stage(std::vector<MergeJob>& jobs, int level) {
    const auto t0 = Clock::now();
    size_t total = 0;
    const int chunks = rep_chunks(jobs, &total);
    t_prep_ = t_submit_ = t_wait_ = t_bits_ = 0;
    cm_status s = CM_OK;
    if (chunks > 1 && !carry_.empty()) s = align_requests(carry_);   // chunked waves carry nothing
    if (s == CM_OK) s = chunks > 1 ? wave_a_chunked(jobs, chunks) : wave_a(jobs, total);
    if (s != CM_OK) return s;
    if (log_)
        fprintf(stderr, "[cm] level %d merges=%zu rep_pairs=%zu waveA=%.3fs in %d chunk(s) (prep %.3f submit %.3f "
                "wait %.3f bits+simulate %.3f) not compared: %lld past a break, %lld absorbed columns\n",
                level, jobs.size(), total, secs(t0, Clock::now()), chunks, t_prep_, t_submit_, t_wait_, t_bits_,
                static_cast<long long>(spec_after_break_), static_cast<long long>(spec_merged_col_));
    spec_after_break_ = 0;
    spec_merged_col_ = 0;
    return CM_OK;
}

bool Driver::replay_pass(std::vector<MergeJob>& jobs, std::vector<int32_t>& req) {
    bool blocked = false;
    for (MergeJob& job : jobs)
        if (!job.done && replay(job, req)) blocked = true;
    return blocked;
}

cm_status Driver::exchange_stage(std::vector<MergeJob>& jobs, std::vector<int32_t>& req, int level) {
    const auto t0 = Clock::now();
    int waves = 0;
    double t_rep = 0, t_al = 0;
    size_t n_req = 0;
    while (true) {
        if (!req.empty()) {
            const auto a0 = Clock::now();
            n_req += req.size() / 2;
            cm_status s = align_requests(req);
            if (s != CM_OK) return s;
            t_al += secs(a0, Clock::now());
            ++waves;
        }
        const auto q0 = Clock::now();
        const bool blocked = replay_pass(jobs, req);
        t_rep += secs(q0, Clock::now());
        if (!blocked) break;
    }
    if (log_)
        fprintf(stderr, "[cm] level %d exchange=%.3fs (%d more waves, %zu pairs, replay %.3f [speculate %.3f] align %.3f)\n",
                level, secs(t0, Clock::now()), waves, n_req, t_rep, t_spec_, t_al);
    t_spec_ = 0;
    return CM_OK;
}

// Columns in chunks: chunk c aligns, for every merge of the level, the rows
// (first-set clusters) still inside Algorithm 1's inner loop against the c-th
// slice of the second set's columns.  Algorithm 1 advances slice by slice: in
// a slice, a row's comparisons depend only on the absorbed flags of the
// slice's columns, which only earlier rows of the same slice set, and on
// whether the row left the loop in an earlier slice; a row that leaves (its
// cluster is absorbed) is not aligned against later slices.  The events are
// put back in row-major order at the end, so the replay is Algorithm 1's.
cm_status Driver::wave_a_chunked(std::vector<MergeJob>& jobs, int chunks) {
    struct JobState {
        std::vector<uint8_t> broken, merged2;
        std::vector<int32_t> rows;          // rows aligned in the current slice
    };
    std::vector<JobState> js(jobs.size());
    for (size_t b = 0; b < jobs.size(); ++b) {
        js[b].broken.assign(sets_[jobs[b].set1].size(), 0);
        js[b].merged2.assign(sets_[jobs[b].set2].size(), 0);
        jobs[b].events.clear();
        jobs[b].result.clear();
    }
    // under the screen (graphs off), the device screens each chunk's pairs
    // (the size guard as for one batch) and aligns the kept ones
    const bool dev_screen = screened(CM_STAGE_REP);
    // plain eager chunks: the device generates each chunk's pairs from one
    // descriptor per merge (its live rows' and the chunk's columns'
    // representatives), in the order the host walks them below
    const bool dev_pairs = !dev_screen && !ctx_->graphs;
    std::vector<int32_t> pairs, out, reps;
    std::vector<int64_t> desc;
    std::vector<EndRec> ends;
    std::vector<uint8_t> bits, guard, keep;
    std::vector<size_t> deferred;
    std::vector<std::pair<int32_t, int32_t>> deferred_reps;
    for (int c = 0; c < chunks; ++c) {
        const auto q0 = Clock::now();
        pairs.clear();
        guard.clear();
        desc.clear();
        reps.clear();
        size_t n = 0;
        double cells = 0;
        for (size_t b = 0; b < jobs.size(); ++b) {
            const std::vector<int32_t>& cs1 = sets_[jobs[b].set1];
            const std::vector<int32_t>& cs2 = sets_[jobs[b].set2];
            const size_t n2 = cs2.size();
            const size_t c0 = n2 * c / chunks, c1 = n2 * (c + 1) / chunks;
            js[b].rows.clear();
            for (size_t i = 0; i < cs1.size(); ++i)
                if (!js[b].broken[i]) js[b].rows.push_back(static_cast<int32_t>(i));
            if (dev_pairs) {
                if (js[b].rows.empty() || c1 == c0) continue;
                desc.push_back(static_cast<int64_t>(n));
                desc.push_back(static_cast<int64_t>(reps.size()));
                desc.push_back(static_cast<int64_t>(js[b].rows.size()));
                double l1 = 0, l2 = 0;
                for (int32_t i : js[b].rows) { reps.push_back(cl_[cs1[i]].rep); l1 += len_[cl_[cs1[i]].rep]; }
                desc.push_back(static_cast<int64_t>(reps.size()));
                desc.push_back(static_cast<int64_t>(c1 - c0));
                for (size_t j = c0; j < c1; ++j) { reps.push_back(cl_[cs2[j]].rep); l2 += len_[cl_[cs2[j]].rep]; }
                cells += l1 * l2;
                n += js[b].rows.size() * (c1 - c0);
                continue;
            }
            for (int32_t i : js[b].rows) {
                const int32_t ra = cl_[cs1[i]].rep;
                for (size_t j = c0; j < c1; ++j) {
                    pairs.push_back(ra);
                    pairs.push_back(cl_[cs2[j]].rep);
                    if (dev_screen) guard.push_back(rep_guarded(cs1[i], cs2[j]) ? 1 : 0);
                }
            }
        }
        if (!dev_pairs) n = pairs.size() / 2;
        if (n == 0) continue;
        const auto q1 = Clock::now();
        cm_status s = dev_screen ? al_.submit_screened(pairs.data(), guard.data(), static_cast<int64_t>(n), scr_,
                                                       static_cast<const uint16_t*>(feat_->ptr), p_.screen_tau)
                      : dev_pairs ? al_.submit_product(0, desc, reps, static_cast<int64_t>(n), nullptr, 0, true, cells)
                                  : al_.submit(0, pairs.data(), static_cast<int64_t>(n), true);
        if (s != CM_OK) return s;
        const auto q2 = Clock::now();
        s = al_.wait_scores(0, out);
        if (s != CM_OK) return s;
        keep.assign(n, 1);
        if (dev_screen) {
            const uint8_t* kf = al_.keep_flags();
            int64_t n_kept = 0, n_guard = 0;
            double cells = 0;
            for (size_t k = 0; k < n; ++k) {
                keep[k] = kf[k];
                n_guard += guard[k];
                if (keep[k]) {
                    ++n_kept;
                    cells += static_cast<double>(len_[pairs[2 * k]]) * len_[pairs[2 * k + 1]];
                } else {
                    ++st_.screened_out;
                }
            }
            st_.screened_pairs += static_cast<int64_t>(n) - n_guard;
            st_.t_screen_s += al_.screen_seconds();
            al_.set_kept(n_kept, cells);
        }
        // scores of the kept pairs come in order; end records are indexed by
        // the kept pair's rank (pairs walked in generation order: merge,
        // live row, column of the chunk)
        bits.assign(n, 0);
        deferred.clear();
        deferred_reps.clear();
        std::vector<int32_t> rank;
        size_t q = 0, k = 0;
        for (size_t b = 0; b < jobs.size(); ++b) {
            const std::vector<int32_t>& cs1 = sets_[jobs[b].set1];
            const std::vector<int32_t>& cs2 = sets_[jobs[b].set2];
            const size_t n2 = cs2.size();
            const size_t c0 = n2 * c / chunks, c1 = n2 * (c + 1) / chunks;
            for (int32_t i : js[b].rows) {
                const int32_t ra = cl_[cs1[i]].rep;
                for (size_t j = c0; j < c1; ++j, ++k) {
                    if (!keep[k]) continue;     // (a pair the screen dropped is not similar)
                    const int32_t rb = cl_[cs2[j]].rep;
                    const int32_t sc = out[q];
                    if (p_.record_candidates) cand_.emplace_back(unordered_key(ra, rb), sc);
                    if (sc >= p_.T) {
                        bits[k] = kSim;
                        cache_.put(unordered_key(ra, rb), sc);
                    }
                    if (sc > p_.mT) {
                        deferred.push_back(k);
                        deferred_reps.emplace_back(ra, rb);
                        rank.push_back(static_cast<int32_t>(q));
                    }
                    ++q;
                }
            }
        }
        if (k != n) return fail(CM_EDEVICE, "chunk walk: %zu of %zu pairs", k, n);
        s = al_.wait(0, out, &ends);
        if (s != CM_OK) return s;
        const auto q3 = Clock::now();
        if (deferred.size() != ends.size())
            return fail(CM_EDEVICE, "end records: %zu of %zu", ends.size(), deferred.size());
        for (size_t qe = 0; qe < deferred.size(); ++qe) {
            const size_t k = deferred[qe];
            if (ends[qe].idx != rank[qe]) return fail(CM_EDEVICE, "missing end record for pair %zu", k);
            const int32_t u1 = len_[deferred_reps[qe].first] - (ends[qe].ea - ends[qe].sa + 1);
            const int32_t u2 = len_[deferred_reps[qe].second] - (ends[qe].eb - ends[qe].sb + 1);
            if (u1 < p_.mU) bits[k] |= kT21;
            if (u2 < p_.mU) bits[k] |= kT12;
            ++st_.end_pairs;
        }
        // Algorithm 1 over this slice, rows in order
        q = 0;
        for (size_t b = 0; b < jobs.size(); ++b) {
            const size_t n2 = sets_[jobs[b].set2].size();
            const size_t c0 = n2 * c / chunks, c1 = n2 * (c + 1) / chunks;
            JobState& st = js[b];
            for (int32_t i : st.rows) {
                for (size_t j = c0; j < c1; ++j) {
                    if (st.merged2[j]) { ++spec_merged_col_; continue; }
                    ++st_.rep_comparisons;
                    st_.required_cells += static_cast<double>(len_[cl_[sets_[jobs[b].set1][i]].rep]) *
                                          len_[cl_[sets_[jobs[b].set2][j]].rep];
                    const uint8_t bb = bits[q + (j - c0)];
                    if (!(bb & kSim)) continue;
                    if (bb & kT21) {            // cluster2 absorbs cluster1; the row leaves the loop
                        jobs[b].events.push_back({kAbsorb21, i, static_cast<int32_t>(j)});
                        st.broken[i] = 1;
                        spec_after_break_ += static_cast<int64_t>(c1 - j - 1);
                        break;
                    }
                    if (bb & kT12) {            // cluster1 absorbs cluster2
                        jobs[b].events.push_back({kAbsorb12, i, static_cast<int32_t>(j)});
                        st.merged2[j] = 1;
                        continue;
                    }
                    jobs[b].events.push_back({kExchange, i, static_cast<int32_t>(j)});
                }
                q += c1 - c0;
            }
        }
        const auto q4 = Clock::now();
        t_prep_ += secs(q0, q1);
        t_submit_ += secs(q1, q2);
        t_wait_ += secs(q2, q3);
        t_bits_ += secs(q3, q4);
    }
    for (size_t b = 0; b < jobs.size(); ++b) {
        MergeJob& job = jobs[b];
        std::stable_sort(job.events.begin(), job.events.end(),
                         [](const Event& x, const Event& y) { return x.i != y.i ? x.i < y.i : x.j < y.j; });
        const std::vector<int32_t>& cs1 = sets_[job.set1];
        const std::vector<int32_t>& cs2 = sets_[job.set2];
        for (size_t i = 0; i < cs1.size(); ++i)
            if (!js[b].broken[i]) job.result.push_back(cs1[i]);
        for (size_t j = 0; j < cs2.size(); ++j)
            if (!js[b].merged2[j]) job.result.push_back(cs2[j]);
    }
    return CM_OK;
}

// All representative pairs of the level in one batch, oriented (cs1 rep, cs2
// rep), with end and start cells for those above mT.
cm_status Driver::wave_a(std::vector<MergeJob>& jobs, size_t total) {
    const auto t0 = Clock::now();
    // the device screens, compacts and aligns in one stream (host-side
    // screening under graph capture)
    const bool dev_screen = screened(CM_STAGE_REP) && !ctx_->graphs && total > 0;
    // plain eager waves: the device generates the pairs from each merge's
    // representative lists (device-screened waves generate them with the
    // size guard; only host-screened waves build them here)
    const bool dev_pairs = !screened(CM_STAGE_REP) && !ctx_->graphs;
    std::vector<int32_t> pairs;
    // one descriptor per merge (block offset, first set's representatives,
    // second set's), the representatives' cluster sizes (screened waves) and
    // the batch's cells, (sum of lengths) x (sum of lengths) per merge
    std::vector<int64_t> desc;
    std::vector<int32_t> reps, counts;
    double desc_cells = 0;
    auto build_desc = [&](bool with_counts) {
        desc.reserve(5 * jobs.size());
        for (const MergeJob& job : jobs) {
            const std::vector<int32_t>& cs1 = sets_[job.set1];
            const std::vector<int32_t>& cs2 = sets_[job.set2];
            if (cs1.empty() || cs2.empty()) continue;
            desc.push_back(static_cast<int64_t>(job.rep_off));
            desc.push_back(static_cast<int64_t>(reps.size()));
            desc.push_back(static_cast<int64_t>(cs1.size()));
            double l1 = 0, l2 = 0;
            for (int32_t a : cs1) { reps.push_back(cl_[a].rep); l1 += len_[cl_[a].rep]; }
            desc.push_back(static_cast<int64_t>(reps.size()));
            desc.push_back(static_cast<int64_t>(cs2.size()));
            for (int32_t b : cs2) { reps.push_back(cl_[b].rep); l2 += len_[cl_[b].rep]; }
            if (with_counts) {
                for (int32_t a : cs1) counts.push_back(static_cast<int32_t>(cl_[a].objs.size()));
                for (int32_t b : cs2) counts.push_back(static_cast<int32_t>(cl_[b].objs.size()));
            }
            desc_cells += l1 * l2;
        }
    };
    if (!dev_pairs && !dev_screen) {
        pairs.resize(2 * total);
        for (const MergeJob& job : jobs) {
            size_t k = job.rep_off;
            for (int32_t a : sets_[job.set1]) {
                const int32_t ra = cl_[a].rep;
                for (int32_t b : sets_[job.set2]) {
                    pairs[2 * k] = ra;
                    pairs[2 * k + 1] = cl_[b].rep;
                    ++k;
                }
            }
        }
    }
    // the screen (when it covers this stage) decides which pairs are aligned;
    // pairs of large clusters (member-count product >= screen_min_product)
    // are always aligned
    std::vector<uint8_t> keep(total, 1);
    std::vector<int32_t> kept;
    const std::vector<int32_t>* src = &pairs;
    cm_status s = CM_OK;
    auto guarded = [&](int32_t a, int32_t b) { return rep_guarded(a, b); };
    int64_t n_guard = 0;
    if (dev_screen) {
        // the guard is set on the device; its count here, per merge from the
        // second set's sorted cluster sizes
        build_desc(true);
        const int64_t minp = p_.screen_min_product;
        if (minp > 0) {
            std::vector<int64_t> c2;
            for (const MergeJob& job : jobs) {
                c2.clear();
                for (int32_t b : sets_[job.set2]) c2.push_back(static_cast<int64_t>(cl_[b].objs.size()));
                std::sort(c2.begin(), c2.end());
                for (int32_t a : sets_[job.set1]) {
                    const int64_t c1 = static_cast<int64_t>(cl_[a].objs.size());
                    if (c1 <= 0) continue;
                    const int64_t need = (minp + c1 - 1) / c1;   // c1 * c2 >= minp  <=>  c2 >= need
                    n_guard += static_cast<int64_t>(c2.end() - std::lower_bound(c2.begin(), c2.end(), need));
                }
            }
        }
    } else if (screened(CM_STAGE_REP)) {
        std::vector<int32_t> cand;
        std::vector<size_t> cand_idx;
        for (const MergeJob& job : jobs) {
            size_t k = job.rep_off;
            for (int32_t a : sets_[job.set1])
                for (int32_t b : sets_[job.set2]) {
                    if (!guarded(a, b)) {
                        cand.push_back(pairs[2 * k]);
                        cand.push_back(pairs[2 * k + 1]);
                        cand_idx.push_back(k);
                    }
                    ++k;
                }
        }
        std::vector<uint8_t> ck;
        s = apply_screen(CM_STAGE_REP, cand, &ck);
        if (s != CM_OK) return s;
        for (size_t q = 0; q < cand_idx.size(); ++q) keep[cand_idx[q]] = ck[q];
        kept.reserve(pairs.size());
        for (size_t k = 0; k < total; ++k)
            if (keep[k]) { kept.push_back(pairs[2 * k]); kept.push_back(pairs[2 * k + 1]); }
        src = &kept;
    }
    // The previous level's first exchange requests (carry_, only on the plain
    // path) ride in this batch after the representative pairs: scores only,
    // the end and start passes cover the representative prefix.
    size_t n_carry = 0;
    const bool carried = !carry_.empty();
    if (carried) {
        if (!dev_pairs) return fail(CM_EDEVICE, "deferred exchange requests on a screened or captured wave");
        size_t w = 0;
        int32_t known;
        for (size_t k = 0; k < carry_.size() / 2; ++k)
            if (!cache_.find(unordered_key(carry_[2 * k], carry_[2 * k + 1]), &known)) {
                carry_[2 * w] = carry_[2 * k];
                carry_[2 * w + 1] = carry_[2 * k + 1];
                ++w;
            }
        carry_.resize(2 * w);
        n_carry = w;
    }
    std::vector<int32_t> out;
    std::vector<EndRec> ends;
    const auto ta = Clock::now();
    if (dev_screen) {
        const Aligner::Product prod{&desc, &reps, &counts, p_.screen_min_product};
        s = al_.submit_screened(nullptr, nullptr, static_cast<int64_t>(total), scr_,
                                static_cast<const uint16_t*>(feat_->ptr), p_.screen_tau, &prod);
    } else if (dev_pairs) {
        build_desc(false);
        double cells = desc_cells;
        for (size_t k = 0; k < n_carry; ++k)
            cells += static_cast<double>(len_[carry_[2 * k]]) * len_[carry_[2 * k + 1]];
        al_.span_pairs = static_cast<int64_t>(total);
        s = al_.submit_product(0, desc, reps, static_cast<int64_t>(total), carry_.data(), static_cast<int64_t>(n_carry),
                               true, cells);
    } else {
        s = al_.submit(0, src->data(), static_cast<int64_t>(src->size() / 2), true);
    }
    if (s != CM_OK) return s;
    const auto tb = Clock::now();
    // scores first (the end and start passes are still running), then the
    // coverage bits of the pairs scoring above mT
    s = al_.wait_scores(0, out);
    if (s != CM_OK) return s;
    if (carried) {
        for (size_t k = 0; k < n_carry; ++k) {
            const uint64_t key = unordered_key(carry_[2 * k], carry_[2 * k + 1]);
            cache_.put(key, out[total + k]);
            if (p_.record_candidates) cand_.emplace_back(key, out[total + k]);
        }
        carry_.clear();
        pending_.clear();
    }
    if (dev_screen) {
        const uint8_t* kf = al_.keep_flags();
        int64_t n_kept = 0;
        double cells = 0;
        for (const MergeJob& job : jobs) {
            size_t k = job.rep_off;
            for (int32_t a : sets_[job.set1]) {
                const double la = len_[cl_[a].rep];
                for (int32_t b : sets_[job.set2]) {
                    keep[k] = kf[k];
                    if (keep[k]) {
                        ++n_kept;
                        cells += la * len_[cl_[b].rep];
                    } else {
                        ++st_.screened_out;
                    }
                    ++k;
                }
            }
        }
        st_.screened_pairs += static_cast<int64_t>(total) - n_guard;
        st_.t_screen_s += al_.screen_seconds();
        al_.set_kept(n_kept, cells);
    }
    // outcome bits per pair in merge order (batch index k = rep_off + i n2 + j);
    // the pairs above mT keep their representatives for the end records
    std::vector<uint8_t> bits(total, 0);
    std::vector<size_t> deferred;                  // batch index k of the pairs above mT
    std::vector<std::pair<int32_t, int32_t>> deferred_reps;
    size_t q = 0;
    for (const MergeJob& job : jobs) {
        size_t k = job.rep_off;
        for (int32_t a : sets_[job.set1]) {
            const int32_t ra = cl_[a].rep;
            for (int32_t b : sets_[job.set2]) {
                if (keep[k]) {                     // (a pair the screen dropped is not similar)
                    const int32_t rb = cl_[b].rep;
                    const int32_t sc = out[q++];
                    if (p_.record_candidates) cand_.emplace_back(unordered_key(ra, rb), sc);
                    if (sc >= p_.T) {
                        bits[k] = kSim;
                        // similar representative scores may be needed again (exchanges, final stage)
                        cache_.put(unordered_key(ra, rb), sc);
                    }
                    if (sc > p_.mT) {
                        deferred.push_back(k);
                        deferred_reps.emplace_back(ra, rb);
                    }
                }
                ++k;
            }
        }
    }
    s = al_.wait(0, out, &ends);
    if (s != CM_OK) return s;
    const auto t1 = Clock::now();
    if (deferred.size() != ends.size()) return fail(CM_EDEVICE, "end records: %zu of %zu", ends.size(), deferred.size());
    q = 0;
    size_t qe = 0;
    for (size_t k = 0; k < total && qe < deferred.size(); ++k) {
        if (!keep[k]) continue;
        if (k == deferred[qe]) {
            if (ends[qe].idx != static_cast<int32_t>(q)) return fail(CM_EDEVICE, "missing end record for pair %zu", q);
            const int32_t r1 = deferred_reps[qe].first, r2 = deferred_reps[qe].second;
            const int32_t u1 = len_[r1] - (ends[qe].ea - ends[qe].sa + 1);
            const int32_t u2 = len_[r2] - (ends[qe].eb - ends[qe].sb + 1);
            if (u1 < p_.mU) bits[k] |= kT21;   // cluster2's rep covers nearly all of rep1
            if (u2 < p_.mU) bits[k] |= kT12;
            ++st_.end_pairs;
            ++qe;
        }
        ++q;
    }
    for (MergeJob& job : jobs) simulate(job, bits.data() + job.rep_off);
    const auto t2 = Clock::now();
    t_prep_ = secs(t0, ta);
    t_submit_ = secs(ta, tb);
    t_wait_ = secs(tb, t1);
    t_bits_ = secs(t1, t2);
    return CM_OK;
}

// Final stage: unique (x, y), x < y, sharing a cluster, generated per x in
// sorted order; scores reused from the cache when known.  Candidate
// generation for the next chunk overlaps the alignment of the current one.
cm_status Driver::final_stage(cm_result* res) {
    const auto t0 = Clock::now();
    const std::vector<int32_t>& fin = sets_.back();
    std::vector<std::vector<int32_t>> sorted(fin.size());
    std::vector<std::vector<int32_t>> of(n_);   // clusters containing each element
    for (size_t k = 0; k < fin.size(); ++k) {
        sorted[k] = cl_[fin[k]].objs;
        std::sort(sorted[k].begin(), sorted[k].end());
        for (int32_t x : sorted[k]) of[x].push_back(static_cast<int32_t>(k));
    }
    // chunks start small so the device starts early, then double up to 2M pairs
    const int64_t kChunk = 1 << 21;
    int64_t chunk = 1 << 15;
    for (int k = 0; k < 2; ++k) {
        cm_status s0 = al_.reserve(k, kChunk + (1 << 16), false);
        if (s0 != CM_OK) return s0;
    }
    struct Chunk {
        std::vector<int32_t> gpu;            // pairs sent to the device
        std::vector<int32_t> cx, cy, cs;     // candidates; cs = known score or -1
    } ch[2];
    uint64_t hash = 0;
    auto mixp = [](uint64_t z) {
        z += 0x9e3779b97f4a7c15ull;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    };
    auto consume = [&](Chunk& c, const std::vector<int32_t>& out) {
        size_t g = 0;
        for (size_t k = 0; k < c.cx.size(); ++k) {
            const int32_t sc = c.cs[k] >= 0 ? c.cs[k] : (c.cs[k] == -1 ? out[g++] : -1);
            if (sc >= p_.T) {
                ++st_.n_similar_pairs;
                hash += mixp((static_cast<uint64_t>(c.cx[k]) << 32 | static_cast<uint32_t>(c.cy[k])) ^
                             (static_cast<uint64_t>(sc) << 17));
                if (static_cast<int64_t>(res->pair_scores.size()) < p_.max_result_pairs) {
                    res->pairs.push_back(c.cx[k]);
                    res->pairs.push_back(c.cy[k]);
                    res->pair_scores.push_back(sc);
                }
            }
        }
        c.gpu.clear(); c.cx.clear(); c.cy.clear(); c.cs.clear();
    };
    int cur = 0;
    bool inflight = false;      // chunk 1-cur is on the device
    double t_submit = 0, t_wait = 0, t_consume = 0;
    std::vector<int32_t> out, ys;
    auto ship = [&]() -> cm_status {
        // submit the current chunk, then finish the previous one
        Chunk& c = ch[cur];
        auto q0 = Clock::now();
        if (screened(CM_STAGE_FINAL)) {
            // every candidate of the chunk is screened, known scores included
            std::vector<int32_t> all(2 * c.cx.size());
            for (size_t k = 0; k < c.cx.size(); ++k) { all[2 * k] = c.cx[k]; all[2 * k + 1] = c.cy[k]; }
            std::vector<uint8_t> keep;
            cm_status s0 = apply_screen(CM_STAGE_FINAL, all, &keep);
            if (s0 != CM_OK) return s0;
            c.gpu.clear();
            for (size_t k = 0; k < c.cs.size(); ++k) {
                if (!keep[k]) { c.cs[k] = -2; continue; }            // -2: dropped, not similar
                if (c.cs[k] == -1) { c.gpu.push_back(c.cx[k]); c.gpu.push_back(c.cy[k]); }
            }
        }
        cm_status s = al_.submit(cur, c.gpu.data(), static_cast<int64_t>(c.gpu.size() / 2), false);
        if (s != CM_OK) return s;
        // test hook: a host allocation failing while a chunk is on the device
        cmrt::test_host_alloc_point();
        auto q1 = Clock::now();
        t_submit += secs(q0, q1);
        if (inflight) {
            s = al_.wait(1 - cur, out);
            if (s != CM_OK) return s;
            auto q2 = Clock::now();
            t_wait += secs(q1, q2);
            consume(ch[1 - cur], out);
            t_consume += secs(q2, Clock::now());
        }
        inflight = true;
        cur = 1 - cur;
        return CM_OK;
    };
    // cached scores as per-element runs sorted by partner: candidates of x
    // come sorted by y, so one forward walk finds the cached ones (a probe of
    // the hash map per candidate costs a cache miss each)
    const auto t_members = Clock::now();
    std::vector<std::pair<uint64_t, int32_t>> known;
    cache_.sorted_entries(&known, n_);
    const auto t_known = Clock::now();
    size_t kp = 0;
    std::vector<int32_t> tmp;
    for (int32_t x = 0; x < n_; ++x) {
        // y > x sharing a cluster with x: the union of the sorted member
        // suffixes of x's clusters, merged linearly
        const int32_t* yb;
        const int32_t* ye;
        if (of[x].size() == 1) {
            const std::vector<int32_t>& v = sorted[of[x][0]];
            ye = v.data() + v.size();
            yb = std::upper_bound(v.data(), ye, x);
        } else {
            ys.clear();
            for (int32_t k : of[x]) {
                const std::vector<int32_t>& v = sorted[k];
                const int32_t* b = std::upper_bound(v.data(), v.data() + v.size(), x);
                tmp.resize(ys.size() + static_cast<size_t>(v.data() + v.size() - b));
                auto e = std::set_union(ys.begin(), ys.end(), b, v.data() + v.size(), tmp.begin());
                tmp.resize(static_cast<size_t>(e - tmp.begin()));
                ys.swap(tmp);
            }
            yb = ys.data();
            ye = ys.data() + ys.size();
        }
        Chunk& c = ch[cur];
        while (kp < known.size() && static_cast<int32_t>(known[kp].first >> 32) < x) ++kp;
        for (const int32_t* py = yb; py != ye; ++py) {
            const int32_t y = *py;
            ++st_.final_candidates;
            c.cx.push_back(x);
            c.cy.push_back(y);
            const uint64_t k = PairMap::key(x, y);
            while (kp < known.size() && known[kp].first < k) ++kp;
            if (kp < known.size() && known[kp].first == k) {
                ++st_.cache_hits;
                c.cs.push_back(known[kp].second);
            } else {
                c.cs.push_back(-1);
                c.gpu.push_back(x);
                c.gpu.push_back(y);
                st_.required_cells += static_cast<double>(len_[x]) * len_[y];
            }
        }
        if (static_cast<int64_t>(c.gpu.size() / 2) >= chunk || static_cast<int64_t>(c.cx.size()) >= 4 * kChunk) {
            cm_status s = ship();
            if (s != CM_OK) return s;
            chunk = std::min<int64_t>(2 * chunk, kChunk);
            if (log_ && (st_.waves & 15) == 0)
                fprintf(stderr, "[cm] final: element %d of %d, %lld candidates\n", x, n_,
                        static_cast<long long>(st_.final_candidates));
        }
    }
    cm_status s = ship();
    if (s != CM_OK) return s;
    s = al_.wait(1 - cur, out);
    if (s != CM_OK) return s;
    consume(ch[1 - cur], out);
    st_.pair_set_hash = hash;
    // clusters in final-set order
    res->member_offsets.push_back(0);
    for (int32_t c : fin) {
        res->reps.push_back(cl_[c].rep);
        res->members.insert(res->members.end(), cl_[c].objs.begin(), cl_[c].objs.end());
        res->member_offsets.push_back(static_cast<int64_t>(res->members.size()));
    }
    st_.n_clusters = static_cast<int64_t>(fin.size());
    if (log_)
        fprintf(stderr, "[cm] final candidates=%lld cache_hits=%lld similar=%lld %.3fs (members %.3f, sorted cache of "
                "%zu scores %.3f, submit %.3f wait %.3f consume %.3f)\n",
                static_cast<long long>(st_.final_candidates), static_cast<long long>(st_.cache_hits),
                static_cast<long long>(st_.n_similar_pairs), secs(t0, Clock::now()), secs(t0, t_members), known.size(),
                secs(t_members, t_known), t_submit, t_wait, t_consume);
    return CM_OK;
}

cm_status Driver::run(cm_result** out) {
    const auto t0 = Clock::now();
    cmrt::drain_timers(ctx_, true);
    // every launch of the run is timed; the caller's setting comes back on
    // every return, including errors
    struct TimerRestore {
        cm_context* ctx;
        bool was_on;
        ~TimerRestore() { ctx->timer.on = was_on; }
    } restore{ctx_, ctx_->timer.on};
    ctx_->timer.on = true;
    const int64_t l0 = ctx_->timer.launches[0];
    const double k0 = ctx_->timer.secs[0];
    const double e0 = ctx_->timer.secs[1] + ctx_->timer.secs[2];
    cm_status s = al_.init();
    if (s != CM_OK) return s;
    s = load_lengths();
    if (s != CM_OK) return s;
    if (scr_ && p_.screen_stages && n_ > 0) {
        feat_ = &ctx_->drv[10];
        if (!feat_->ensure(static_cast<size_t>(n_) * 1024 * 2)) return fail(CM_ENOMEM, "store features");
        s = cm_kmer_features(ctx_, al_.seqs, al_.offsets, n_, static_cast<uint16_t*>(feat_->ptr), al_.st);
        if (s != CM_OK) return s;
        if (hipStreamSynchronize(al_.st) != hipSuccess) return fail(CM_EDEVICE, "features");
    }
    // Algorithm 2: singleton sets of the elements to cluster, FIFO merge
    // order, grouped by tree level.  Classifying new elements against a
    // previous clustering: the new elements' tree, then one merge of the
    // previous final set (first) with its result.
    const int32_t first = prev_ ? prev_->n_prev : 0;
    const int32_t n_new = n_ - first;
    const int32_t n_old_cl = prev_ ? prev_->n_clusters : 0;
    cl_.resize(static_cast<size_t>(n_old_cl) + n_new);
    for (int32_t c = 0; c < n_old_cl; ++c) {
        cl_[c].rep = prev_->reps[c];
        for (int64_t k = prev_->member_offsets[c]; k < prev_->member_offsets[c + 1]; ++k)
            cl_[c].add(prev_->members[k]);
    }
    sets_.assign(n_new, {});
    std::vector<int32_t> level(n_new, 0);
    for (int32_t e = 0; e < n_new; ++e) {
        const int32_t cid = n_old_cl + e;
        cl_[cid].rep = first + e;
        cl_[cid].add(first + e);
        sets_[e].push_back(cid);
    }
    std::vector<std::vector<MergeJob>> by_level;
    auto add_job = [&](int32_t x, int32_t y) {
        const int32_t z = static_cast<int32_t>(level.size());
        const int32_t lv = std::max(level[x], level[y]) + 1;
        level.push_back(lv);
        sets_.emplace_back();
        if (static_cast<int32_t>(by_level.size()) < lv) by_level.resize(lv);
        MergeJob job;
        job.set1 = x;
        job.set2 = y;
        job.out = z;
        by_level[lv - 1].push_back(job);
        return z;
    };
    {
        std::vector<int32_t> q(n_new);
        for (int32_t e = 0; e < n_new; ++e) q[e] = e;
        size_t head = 0;
        while (q.size() - head > 1) {
            const int32_t x = q[head++], y = q[head++];
            q.push_back(add_job(x, y));
        }
        if (prev_) {
            const int32_t p_set = static_cast<int32_t>(sets_.size());
            sets_.emplace_back();
            level.push_back(0);
            for (int32_t c = 0; c < n_old_cl; ++c) sets_[p_set].push_back(c);
            if (n_new > 0) add_job(p_set, q[head]);
            // the previous run's scores (similar pairs) are known
            for (int64_t k = 0; k < prev_->n_known; ++k)
                cache_.put(unordered_key(prev_->known_pairs[2 * k], prev_->known_pairs[2 * k + 1]),
                           prev_->known_scores[k]);
        }
    }
    st_.rounds = static_cast<int64_t>(by_level.size());
    auto release_inputs = [&](std::vector<MergeJob>& jobs) {
        for (MergeJob& job : jobs) {
            std::vector<int32_t>().swap(sets_[job.set1]);
            std::vector<int32_t>().swap(sets_[job.set2]);
        }
    };
    std::vector<MergeJob>* held = nullptr;   // level whose exchange stage waits for the carried requests
    std::vector<int32_t> req;
    for (size_t lv = 0; lv < by_level.size(); ++lv) {
        std::vector<MergeJob>& jobs = by_level[lv];
        const int lvi = static_cast<int>(lv);
        s = rep_stage(jobs, lvi);
        if (s != CM_OK) return s;
        for (MergeJob& job : jobs) sets_[job.out] = std::move(job.result);
        if (held) {
            req.clear();
            s = exchange_stage(*held, req, lvi - 1);
            if (s != CM_OK) return s;
            release_inputs(*held);
            held = nullptr;
        }
        req.clear();
        const bool blocked = replay_pass(jobs, req);
        if (blocked && lv + 1 < by_level.size() && can_carry(by_level[lv + 1])) {
            carry_.swap(req);
            held = &jobs;
            continue;
        }
        s = exchange_stage(jobs, req, lvi);
        if (s != CM_OK) return s;
        release_inputs(jobs);
    }
    if (held || !carry_.empty()) return fail(CM_EDEVICE, "exchange requests left after the last level");
    if (sets_.empty()) sets_.emplace_back();
    const auto t1 = Clock::now();
    std::unique_ptr<cm_result> res(new cm_result());
    if (p_.record_candidates) {
        // every pair scored in the merge stage, once
        std::vector<std::pair<uint64_t, int32_t>>& ent = cand_;
        std::sort(ent.begin(), ent.end());
        ent.erase(std::unique(ent.begin(), ent.end(),
                              [](const std::pair<uint64_t, int32_t>& x, const std::pair<uint64_t, int32_t>& y) {
                                  return x.first == y.first;
                              }),
                  ent.end());
        res->cand_pairs.reserve(2 * ent.size());
        res->cand_scores.reserve(ent.size());
        for (const auto& e : ent) {
            res->cand_pairs.push_back(static_cast<int32_t>(e.first >> 32));
            res->cand_pairs.push_back(static_cast<int32_t>(e.first & 0xffffffffu));
            res->cand_scores.push_back(e.second);
        }
    }
    s = final_stage(res.get());
    if (s != CM_OK) return s;
    const auto t2 = Clock::now();
    int64_t needed = 0;
    // speculative work = aligned pairs the replay and the final stage never read
    needed = st_.rep_comparisons + st_.exchange_alignments + (st_.final_candidates - st_.cache_hits);
    st_.speculative_pairs = st_.aligned_pairs > needed ? st_.aligned_pairs - needed : 0;
    st_.t_merge_s = secs(t0, t1);
    st_.t_final_s = secs(t1, t2);
    st_.t_total_s = secs(t0, t2);
    st_.t_host_s = st_.t_total_s - st_.t_gpu_s;
    cmrt::drain_timers(ctx_, true);
    st_.sw_launches = ctx_->timer.launches[0] - l0;
    st_.sw_kernel_s = ctx_->timer.secs[0] - k0;
    st_.end_kernel_s = ctx_->timer.secs[1] + ctx_->timer.secs[2] - e0;
    res->stats = st_;
    *out = res.release();
    return CM_OK;
}

// ---------------------------------------------------------------------------
// all-vs-all ground truth: triangle pair tiles generated and counted on device
// ---------------------------------------------------------------------------
__global__ void k_tri_pairs(int64_t first, int64_t count, int32_t n, int32_t* pairs) {
    const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (t >= count) return;
    const int64_t idx = first + t;
    // row i owns n-1-i pairs; start(i) = i*(2n-i-1)/2; find i with start(i) <= idx
    const double nn = static_cast<double>(n);
    int64_t i = static_cast<int64_t>(nn - 0.5 - sqrt((nn - 0.5) * (nn - 0.5) - 2.0 * static_cast<double>(idx)));
    if (i < 0) i = 0;
    if (i > n - 2) i = n - 2;
    while (i > 0 && i * (2 * static_cast<int64_t>(n) - i - 1) / 2 > idx) --i;
    while ((i + 1) * (2 * static_cast<int64_t>(n) - i - 2) / 2 <= idx) ++i;
    const int64_t j = i + 1 + (idx - i * (2 * static_cast<int64_t>(n) - i - 1) / 2);
    pairs[2 * t] = static_cast<int32_t>(i);
    pairs[2 * t + 1] = static_cast<int32_t>(j);
}

__global__ void k_count_ge(const int32_t* scores, int64_t count, int32_t T, unsigned long long* total) {
    __shared__ unsigned int s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    unsigned int local = 0;
    for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < count;
         t += static_cast<int64_t>(gridDim.x) * blockDim.x)
        local += scores[t] >= T;
    if (local) atomicAdd(&s_cnt, local);
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt) atomicAdd(total, static_cast<unsigned long long>(s_cnt));
}

}  // namespace cmdrv

extern "C" {

static cm_status check_run_params(const cm_params* params) {
    cm_status s = cmrt::check_gaps(params->gap_open, params->gap_extend);
    if (s != CM_OK) return s;
    int8_t mat8[cmk::kNRes * cmk::kMatStride];
    s = cmrt::check_matrix(params->matrix, mat8);
    if (s != CM_OK) return s;
    // similarity is a property of the unordered pair: the driver keeps one
    // score per pair and aligns a pair in whichever orientation batches best
    for (int x = 0; x < 20; ++x)
        for (int y = 0; y < x; ++y)
            if (params->matrix[20 * x + y] != params->matrix[20 * y + x])
                return cmrt::fail(CM_EINVAL, "ClusterMerge needs a symmetric matrix (M[%d][%d] != M[%d][%d])",
                                  x, y, y, x);
    if (params->T < 1 || params->mT < 0 || params->mU < 0 || params->max_result_pairs < 0)
        return cmrt::fail(CM_EINVAL, "T must be >= 1; mT, mU and max_result_pairs >= 0");
    if (params->record_candidates != 0 && params->record_candidates != 1)
        return cmrt::fail(CM_EINVAL, "record_candidates must be 0 or 1");
    return CM_OK;
}

cm_status cm_clustermerge_run(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                              const cm_params* params, const cm_screen* screen, cm_result** out) {
    CM_TRY
    if (!ctx || !params || !out) return cmrt::fail(CM_EINVAL, "NULL argument");
    if (!offsets || n_seqs < 0) return cmrt::fail(CM_EINVAL, "bad store");
    *out = nullptr;
    cm_status s = check_run_params(params);
    if (s != CM_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return cmrt::fail(CM_EDEVICE, "hipSetDevice");
    cmdrv::Driver drv(ctx, seqs, offsets, n_seqs, params, screen);
    return drv.run(out);
    CM_CATCH
}

cm_status cm_clustermerge_extend(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                                 const cm_params* params, const cm_screen* screen, int32_t n_prev,
                                 int32_t n_clusters, const int32_t* reps, const int64_t* member_offsets,
                                 const int32_t* members, int64_t n_known, const int32_t* known_pairs,
                                 const int32_t* known_scores, cm_result** out) {
    CM_TRY
    if (!ctx || !params || !out) return cmrt::fail(CM_EINVAL, "NULL argument");
    if (!offsets || n_seqs < 0) return cmrt::fail(CM_EINVAL, "bad store");
    *out = nullptr;
    cm_status s = check_run_params(params);
    if (s != CM_OK) return s;
    if (n_prev < 0 || n_prev > n_seqs || n_clusters < 0 || n_known < 0)
        return cmrt::fail(CM_EINVAL, "n_prev must be in [0, n_seqs]; n_clusters, n_known >= 0");
    if (n_prev > 0 && n_clusters == 0) return cmrt::fail(CM_EINVAL, "previous elements without clusters");
    if (n_clusters > 0 && (!reps || !member_offsets || !members))
        return cmrt::fail(CM_EINVAL, "NULL previous clustering");
    if (n_known > 0 && (!known_pairs || !known_scores)) return cmrt::fail(CM_EINVAL, "NULL known pairs");
    // every previous element in at least one cluster, members in range and
    // unique within their cluster, each representative a member of its cluster
    if (n_clusters > 0 && member_offsets[0] != 0) return cmrt::fail(CM_EINVAL, "member_offsets[0] != 0");
    std::vector<int32_t> seen(static_cast<size_t>(n_prev), -1);
    std::vector<uint8_t> covered(static_cast<size_t>(n_prev), 0);
    for (int32_t c = 0; c < n_clusters; ++c) {
        const int64_t b = member_offsets[c], e = member_offsets[c + 1];
        if (e <= b) return cmrt::fail(CM_EINVAL, "cluster %d is empty or its offsets decrease", c);
        bool rep_in = false;
        for (int64_t k = b; k < e; ++k) {
            const int32_t x = members[k];
            if (x < 0 || x >= n_prev) return cmrt::fail(CM_EINVAL, "cluster %d: member %d outside [0, n_prev)", c, x);
            if (seen[x] == c) return cmrt::fail(CM_EINVAL, "cluster %d: member %d listed twice", c, x);
            seen[x] = c;
            covered[x] = 1;
            rep_in |= (x == reps[c]);
        }
        if (!rep_in) return cmrt::fail(CM_EINVAL, "cluster %d: representative %d is not a member", c, reps[c]);
    }
    for (int32_t x = 0; x < n_prev; ++x)
        if (!covered[x]) return cmrt::fail(CM_EINVAL, "previous element %d is in no cluster", x);
    for (int64_t k = 0; k < n_known; ++k) {
        const int32_t x = known_pairs[2 * k], y = known_pairs[2 * k + 1];
        if (x < 0 || y < 0 || x >= n_prev || y >= n_prev || x == y)
            return cmrt::fail(CM_EINVAL, "known pair %lld out of range", static_cast<long long>(k));
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return cmrt::fail(CM_EDEVICE, "hipSetDevice");
    cmdrv::PrevClustering prev;
    prev.n_prev = n_prev;
    prev.n_clusters = n_clusters;
    prev.reps = reps;
    prev.member_offsets = member_offsets;
    prev.members = members;
    prev.n_known = n_known;
    prev.known_pairs = known_pairs;
    prev.known_scores = known_scores;
    cmdrv::Driver drv(ctx, seqs, offsets, n_seqs, params, screen);
    drv.set_prev(&prev);
    return drv.run(out);
    CM_CATCH
}

cm_status cm_result_clusters(const cm_result* r, int32_t* n_clusters, const int32_t** reps,
                             const int64_t** member_offsets, const int32_t** members) {
    CM_TRY
    if (!r) return cmrt::fail(CM_EINVAL, "result is NULL");
    if (n_clusters) *n_clusters = static_cast<int32_t>(r->reps.size());
    if (reps) *reps = r->reps.data();
    if (member_offsets) *member_offsets = r->member_offsets.data();
    if (members) *members = r->members.data();
    return CM_OK;
    CM_CATCH
}

cm_status cm_result_pairs(const cm_result* r, int64_t* n_pairs, const int32_t** pairs, const int32_t** scores) {
    CM_TRY
    if (!r) return cmrt::fail(CM_EINVAL, "result is NULL");
    if (n_pairs) *n_pairs = static_cast<int64_t>(r->pair_scores.size());
    if (pairs) *pairs = r->pairs.data();
    if (scores) *scores = r->pair_scores.data();
    return CM_OK;
    CM_CATCH
}

cm_status cm_result_candidates(const cm_result* r, int64_t* n_pairs, const int32_t** pairs, const int32_t** scores) {
    CM_TRY
    if (!r) return cmrt::fail(CM_EINVAL, "result is NULL");
    if (n_pairs) *n_pairs = static_cast<int64_t>(r->cand_scores.size());
    if (pairs) *pairs = r->cand_pairs.data();
    if (scores) *scores = r->cand_scores.data();
    return CM_OK;
    CM_CATCH
}

cm_status cm_result_stats(const cm_result* r, cm_stats* out) {
    CM_TRY
    if (!r || !out) return cmrt::fail(CM_EINVAL, "NULL argument");
    *out = r->stats;
    return CM_OK;
    CM_CATCH
}

void cm_result_free(cm_result* r) { delete r; }

cm_status cm_allvsall_count(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                            const int32_t* matrix, int32_t gap_open, int32_t gap_extend, int32_t T,
                            int64_t* count, double* cells) {
    CM_TRY
    if (!ctx || !offsets || !count) return cmrt::fail(CM_EINVAL, "NULL argument");
    *count = 0;
    if (cells) *cells = 0;
    if (n_seqs < 2) return CM_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return cmrt::fail(CM_EDEVICE, "hipSetDevice");
    const int64_t total = static_cast<int64_t>(n_seqs) * (n_seqs - 1) / 2;
    const int64_t chunk = std::min<int64_t>(total, 1 << 23);
    cmrt::DeviceBuf& d_pairs = ctx->drv[5];
    cmrt::DeviceBuf& d_sc = ctx->drv[6];
    cmrt::DeviceBuf& d_cnt = ctx->drv[7];
    if (!d_pairs.ensure(chunk * 8) || !d_sc.ensure(chunk * 4) || !d_cnt.ensure(64))
        return cmrt::fail(CM_ENOMEM, "all-vs-all scratch");
    unsigned long long* dcnt = static_cast<unsigned long long*>(d_cnt.ptr);
    hipStream_t st = nullptr;
    if (hipMemsetAsync(dcnt, 0, 8, st) != hipSuccess) return cmrt::fail(CM_EDEVICE, "memset");
    for (int64_t first = 0; first < total; first += chunk) {
        const int64_t cnt = std::min(chunk, total - first);
        hipLaunchKernelGGL(cmdrv::k_tri_pairs, dim3(static_cast<unsigned>((cnt + 255) / 256)), dim3(256), 0, st,
                           first, cnt, n_seqs, static_cast<int32_t*>(d_pairs.ptr));
        cm_status s = cm_sw_score_batch(ctx, seqs, offsets, n_seqs, static_cast<int32_t*>(d_pairs.ptr), cnt,
                                        matrix, gap_open, gap_extend, static_cast<int32_t*>(d_sc.ptr), nullptr,
                                        nullptr, st);
        if (s != CM_OK) return s;
        hipLaunchKernelGGL(cmdrv::k_count_ge, dim3(1024), dim3(256), 0, st, static_cast<int32_t*>(d_sc.ptr), cnt,
                           T, dcnt);
    }
    unsigned long long host = 0;
    if (hipMemcpy(&host, dcnt, 8, hipMemcpyDeviceToHost) != hipSuccess) return cmrt::fail(CM_EDEVICE, "count");
    cm_status s = cm_context_sync(ctx);
    if (s != CM_OK) return s;
    *count = static_cast<int64_t>(host);
    if (cells) {
        std::vector<int64_t> off(static_cast<size_t>(n_seqs) + 1);
        if (hipMemcpy(off.data(), offsets, off.size() * 8, hipMemcpyDeviceToHost) != hipSuccess)
            return cmrt::fail(CM_EDEVICE, "offsets");
        double s1 = 0, s2 = 0;
        for (int32_t k = 0; k < n_seqs; ++k) {
            const double L = static_cast<double>(off[k + 1] - off[k]);
            s1 += L;
            s2 += L * L;
        }
        *cells = (s1 * s1 - s2) / 2;
    }
    return CM_OK;
    CM_CATCH
}

}  // extern "C"
