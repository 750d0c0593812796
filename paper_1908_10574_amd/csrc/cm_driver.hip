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
#include <algorithm>
#include <chrono>
#include <cstring>
#include <unordered_set>
#include <vector>

#include "../../include/cm.h"
#include "cm_internal.h"
#include "cm_runtime.h"

struct cm_result {
    std::vector<int32_t> reps;
    std::vector<int64_t> member_offsets;
    std::vector<int32_t> members;
    std::vector<int32_t> pairs;
    std::vector<int32_t> pair_scores;
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
    hipEvent_t e0 = nullptr, e1 = nullptr;
    Pinned h_pairs, h_out;
    cm_stats* stats = nullptr;

    cm_status init() {
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return fail(CM_EDEVICE, "stream");
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(CM_EDEVICE, "events");
        return CM_OK;
    }
    ~Aligner() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (st) (void)hipStreamDestroy(st);
    }

    // Align np pairs (flat a,b).  out receives np scores, and with spans
    // 4 more int32 per pair: end_a, end_b, start_a, start_b (start only for
    // scores > mT, else -1).
    cm_status run(const int32_t* pairs, int64_t np, bool spans, std::vector<int32_t>& out) {
        out.assign(static_cast<size_t>(np) * (spans ? 5 : 1), 0);
        if (np == 0) return CM_OK;
        const size_t pb = static_cast<size_t>(np) * 8, ob = static_cast<size_t>(np) * 4;
        cmrt::DeviceBuf& d_pairs = ctx->drv[0];
        cmrt::DeviceBuf& d_out = ctx->drv[1];
        if (!d_pairs.ensure(pb) || !d_out.ensure(ob * 5) || !h_pairs.ensure(pb) || !h_out.ensure(ob * 5))
            return fail(CM_ENOMEM, "cannot stage %lld pairs", static_cast<long long>(np));
        std::memcpy(h_pairs.ptr, pairs, pb);
        int32_t* dsc = static_cast<int32_t*>(d_out.ptr);
        int32_t* dea = dsc + np;
        int32_t* deb = dea + np;
        int32_t* dsa = deb + np;
        int32_t* dsb = dsa + np;
        hipError_t e = hipMemcpyAsync(d_pairs.ptr, h_pairs.ptr, pb, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "pairs upload");
        (void)hipEventRecord(e0, st);
        cm_status s = cm_sw_score_batch(ctx, seqs, offsets, n_seqs, static_cast<int32_t*>(d_pairs.ptr), np,
                                        p->matrix, p->gap_open, p->gap_extend, dsc, spans ? dea : nullptr,
                                        spans ? deb : nullptr, st);
        if (s != CM_OK) return s;
        if (spans) {
            s = cm_sw_span_batch(ctx, seqs, offsets, n_seqs, static_cast<int32_t*>(d_pairs.ptr), np, p->matrix,
                                 p->gap_open, p->gap_extend, dsc, dea, deb, p->mT, dsa, dsb, st);
            if (s != CM_OK) return s;
        }
        (void)hipEventRecord(e1, st);
        e = hipMemcpyAsync(h_out.ptr, dsc, ob * (spans ? 5 : 1), hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return hip_fail(e, "scores download");
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "alignment batch");
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        s = cm_context_sync(ctx);   // device-side data errors
        if (s != CM_OK) return s;
        std::memcpy(out.data(), h_out.ptr, ob * (spans ? 5 : 1));
        stats->t_gpu_s += ms * 1e-3;
        stats->waves += 1;
        stats->aligned_pairs += np;
        double cells = 0;
        for (int64_t k = 0; k < np; ++k)
            cells += static_cast<double>((*len)[pairs[2 * k]]) * (*len)[pairs[2 * k + 1]];
        stats->aligned_cells += cells;
        return CM_OK;
    }
};

// ---------------------------------------------------------------------------
// clusters and the Algorithm 1 replay
// ---------------------------------------------------------------------------
struct Cluster {
    int32_t rep;
    std::vector<int32_t> objs;
    std::unordered_set<int32_t> mem;
    bool merged = false;
    void add(int32_t x) {
        if (mem.insert(x).second) objs.push_back(x);
    }
    bool has(int32_t x) const { return mem.count(x) != 0; }
};

// representative-pair outcome bits
constexpr int32_t kSim = 1, kT21 = 2, kT12 = 4;

struct MergeJob {
    int32_t set1, set2, out;
    size_t i = 0, j = 0;          // position of the Algorithm 1 double loop
    bool done = false;
    std::vector<int32_t> result;  // clusters of the new set
};

class Driver {
public:
    Driver(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n, const cm_params* p)
        : ctx_(ctx), n_(n), p_(*p) {
        al_.ctx = ctx;
        al_.seqs = seqs;
        al_.offsets = offsets;
        al_.n_seqs = n;
        al_.p = &p_;
        al_.len = &len_;
        al_.stats = &st_;
    }

    cm_status run(cm_result** out);

private:
    cm_status load_lengths();
    cm_status merge_level(std::vector<MergeJob>& jobs);
    // replay one merge until done or blocked; returns true when blocked
    bool replay(MergeJob& job, std::vector<int32_t>& req);
    void dry_walk(const MergeJob& job, std::vector<int32_t>& req);
    void request_exchange(const Cluster& c1, const Cluster& c2, std::vector<int32_t>& req);
    cm_status align_requests(std::vector<int32_t>& req);
    cm_status final_stage(cm_result* res);

    int32_t rep_bits(int32_t r1, int32_t r2) const {
        int32_t v = 0;
        rep_.find(PairMap::key(r1, r2), &v);
        return v;
    }
    bool score_of(int32_t x, int32_t y, int32_t* s) const { return cache_.find(unordered_key(x, y), s); }

    cm_context* ctx_;
    int32_t n_;
    cm_params p_;
    Aligner al_;
    cm_stats st_{};
    std::vector<int32_t> len_;
    std::vector<Cluster> cl_;
    std::vector<std::vector<int32_t>> sets_;
    PairMap cache_;    // unordered pair -> score
    PairMap rep_;      // oriented representative pair -> outcome bits (current level)
    PairMap pending_;  // pairs requested in the current wave
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
        if (cache_.find(k, &s) || pending_.find(k, &s)) return;
        pending_.put(k, 0);
        req.push_back(m);
        req.push_back(rep);
    };
    for (int32_t m : c2.objs)
        if (!c1.has(m)) want(m, c1.rep);
    for (int32_t m : c1.objs)
        if (!c2.has(m)) want(m, c2.rep);
}

bool Driver::replay(MergeJob& job, std::vector<int32_t>& req) {
    const std::vector<int32_t>& cs1 = sets_[job.set1];
    const std::vector<int32_t>& cs2 = sets_[job.set2];
    while (job.i < cs1.size()) {
        Cluster& c1 = cl_[cs1[job.i]];
        while (job.j < cs2.size()) {
            Cluster& c2 = cl_[cs2[job.j]];
            if (c2.merged) { ++job.j; continue; }
            const int32_t bits = rep_bits(c1.rep, c2.rep);
            if (!(bits & kSim)) { ++st_.rep_comparisons; ++job.j; continue; }
            if (bits & kT21) {                       // cluster2 absorbs cluster1
                ++st_.rep_comparisons;
                for (int32_t x : c1.objs) c2.add(x);
                c1.merged = true;
                ++st_.full_merges;
                break;
            }
            if (bits & kT12) {                       // cluster1 absorbs cluster2
                ++st_.rep_comparisons;
                for (int32_t x : c2.objs) c1.add(x);
                c2.merged = true;
                ++st_.full_merges;
                ++job.j;
                continue;
            }
            // ExchangeSimilar: every member-vs-representative score must be known
            std::vector<int32_t> add1, add2;
            bool missing = false;
            int64_t tests = 0;
            for (int32_t m : c2.objs) {
                if (c1.has(m)) continue;
                ++tests;
                int32_t s;
                if (!score_of(m, c1.rep, &s)) { missing = true; continue; }
                if (s >= p_.T) add1.push_back(m);
            }
            for (int32_t m : c1.objs) {
                if (c2.has(m)) continue;
                ++tests;
                int32_t s;
                if (!score_of(m, c2.rep, &s)) { missing = true; continue; }
                if (s >= p_.T) add2.push_back(m);
            }
            if (missing) {
                request_exchange(c1, c2, req);
                dry_walk(job, req);
                return true;
            }
            ++st_.rep_comparisons;
            st_.exchange_alignments += tests;
            ++st_.exchanges;
            for (int32_t m : add1) c1.add(m);
            for (int32_t m : add2) c2.add(m);
            ++job.j;
        }
        if (!c1.merged) job.result.push_back(cs1[job.i]);
        ++job.i;
        job.j = 0;
    }
    for (int32_t c : cs2)
        if (!cl_[c].merged) job.result.push_back(c);
    job.done = true;
    return false;
}

// After the replay blocks at (i, j): walk the rest of the merge with the
// full-merge and break decisions (known from representative scores alone) and
// request the pairs of every later exchange with the memberships known now.
void Driver::dry_walk(const MergeJob& job, std::vector<int32_t>& req) {
    const std::vector<int32_t>& cs1 = sets_[job.set1];
    const std::vector<int32_t>& cs2 = sets_[job.set2];
    std::unordered_set<int32_t> merged2;   // clusters of cs2 merged during the walk
    size_t i = job.i, j = job.j + 1;
    while (i < cs1.size()) {
        const Cluster& c1 = cl_[cs1[i]];
        for (; j < cs2.size(); ++j) {
            const Cluster& c2 = cl_[cs2[j]];
            if (c2.merged || merged2.count(cs2[j])) continue;
            const int32_t bits = rep_bits(c1.rep, c2.rep);
            if (!(bits & kSim)) continue;
            if (bits & kT21) break;
            if (bits & kT12) { merged2.insert(cs2[j]); continue; }
            request_exchange(c1, c2, req);
        }
        ++i;
        j = 0;
    }
}

cm_status Driver::align_requests(std::vector<int32_t>& req) {
    std::vector<int32_t> out;
    cm_status s = al_.run(req.data(), static_cast<int64_t>(req.size() / 2), false, out);
    if (s != CM_OK) return s;
    for (size_t k = 0; k < out.size(); ++k) cache_.put(unordered_key(req[2 * k], req[2 * k + 1]), out[k]);
    pending_.clear();
    req.clear();
    return CM_OK;
}

cm_status Driver::merge_level(std::vector<MergeJob>& jobs) {
    // wave A: all representative pairs, oriented (cs1 rep, cs2 rep), with spans
    std::vector<int32_t> pairs;
    for (const MergeJob& job : jobs)
        for (int32_t a : sets_[job.set1])
            for (int32_t b : sets_[job.set2]) {
                pairs.push_back(cl_[a].rep);
                pairs.push_back(cl_[b].rep);
            }
    std::vector<int32_t> out;
    cm_status s = al_.run(pairs.data(), static_cast<int64_t>(pairs.size() / 2), true, out);
    if (s != CM_OK) return s;
    rep_.clear();
    const size_t np = pairs.size() / 2;
    for (size_t k = 0; k < np; ++k) {
        const int32_t r1 = pairs[2 * k], r2 = pairs[2 * k + 1];
        const int32_t sc = out[k];
        int32_t bits = 0;
        if (sc >= p_.T) bits |= kSim;
        if (sc > p_.mT) {
            const int32_t ea = out[np + k], eb = out[2 * np + k], sa = out[3 * np + k], sb = out[4 * np + k];
            const int32_t u1 = len_[r1] - (ea - sa + 1);
            const int32_t u2 = len_[r2] - (eb - sb + 1);
            if (u1 < p_.mU) bits |= kT21;   // cluster2's rep covers nearly all of rep1
            if (u2 < p_.mU) bits |= kT12;
        }
        rep_.put(PairMap::key(r1, r2), bits);
        cache_.put(unordered_key(r1, r2), sc);
    }
    // exchange waves
    std::vector<int32_t> req;
    while (true) {
        bool any_blocked = false;
        for (MergeJob& job : jobs)
            if (!job.done && replay(job, req)) any_blocked = true;
        if (!any_blocked) break;
        s = align_requests(req);
        if (s != CM_OK) return s;
    }
    return CM_OK;
}

// Final stage: unique (x, y), x < y, sharing a cluster, generated per x in
// sorted order; scores reused from the cache when known.
cm_status Driver::final_stage(cm_result* res) {
    const std::vector<int32_t>& fin = sets_.back();
    std::vector<std::vector<int32_t>> sorted(fin.size());
    std::vector<std::vector<int32_t>> of(n_);   // clusters containing each element
    for (size_t k = 0; k < fin.size(); ++k) {
        sorted[k] = cl_[fin[k]].objs;
        std::sort(sorted[k].begin(), sorted[k].end());
        for (int32_t x : sorted[k]) of[x].push_back(static_cast<int32_t>(k));
    }
    const int64_t kChunk = 1 << 22;
    std::vector<int32_t> batch, cand_x, cand_y, known_s;   // candidates of the current chunk
    std::vector<int8_t> known;
    std::vector<int32_t> gpu;
    uint64_t hash = 0;
    auto mixp = [](uint64_t z) {
        z += 0x9e3779b97f4a7c15ull;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    };
    auto flush = [&]() -> cm_status {
        std::vector<int32_t> out;
        cm_status s = al_.run(batch.data(), static_cast<int64_t>(batch.size() / 2), false, out);
        if (s != CM_OK) return s;
        size_t g = 0;
        for (size_t k = 0; k < cand_x.size(); ++k) {
            const int32_t sc = known[k] ? known_s[k] : out[g++];
            if (sc >= p_.T) {
                ++st_.n_similar_pairs;
                hash += mixp((static_cast<uint64_t>(cand_x[k]) << 32 | static_cast<uint32_t>(cand_y[k])) ^
                             (static_cast<uint64_t>(sc) << 17));
                if (static_cast<int64_t>(res->pair_scores.size()) < p_.max_result_pairs) {
                    res->pairs.push_back(cand_x[k]);
                    res->pairs.push_back(cand_y[k]);
                    res->pair_scores.push_back(sc);
                }
            }
        }
        batch.clear(); cand_x.clear(); cand_y.clear(); known.clear(); known_s.clear();
        return CM_OK;
    };
    std::vector<int32_t> ys;
    for (int32_t x = 0; x < n_; ++x) {
        ys.clear();
        for (int32_t k : of[x]) {
            const std::vector<int32_t>& v = sorted[k];
            auto it = std::upper_bound(v.begin(), v.end(), x);
            ys.insert(ys.end(), it, v.end());
        }
        if (of[x].size() > 1) {
            std::sort(ys.begin(), ys.end());
            ys.erase(std::unique(ys.begin(), ys.end()), ys.end());
        }
        for (int32_t y : ys) {
            ++st_.final_candidates;
            int32_t sc;
            cand_x.push_back(x);
            cand_y.push_back(y);
            if (cache_.find(PairMap::key(x, y), &sc)) {
                ++st_.cache_hits;
                known.push_back(1);
                known_s.push_back(sc);
            } else {
                known.push_back(0);
                known_s.push_back(0);
                batch.push_back(x);
                batch.push_back(y);
            }
        }
        if (static_cast<int64_t>(batch.size() / 2) >= kChunk || static_cast<int64_t>(cand_x.size()) >= 4 * kChunk) {
            cm_status s = flush();
            if (s != CM_OK) return s;
        }
    }
    cm_status s = flush();
    if (s != CM_OK) return s;
    st_.pair_set_hash = hash;
    // clusters in final-set order
    res->member_offsets.push_back(0);
    for (int32_t c : fin) {
        res->reps.push_back(cl_[c].rep);
        res->members.insert(res->members.end(), cl_[c].objs.begin(), cl_[c].objs.end());
        res->member_offsets.push_back(static_cast<int64_t>(res->members.size()));
    }
    st_.n_clusters = static_cast<int64_t>(fin.size());
    return CM_OK;
}


cm_status Driver::run(cm_result** out) {
    const auto t0 = Clock::now();
    cm_status s = al_.init();
    if (s != CM_OK) return s;
    s = load_lengths();
    if (s != CM_OK) return s;
    // Algorithm 2: singleton sets 0..n-1, FIFO merge order, grouped by tree level
    cl_.resize(n_);
    sets_.assign(n_, {});
    std::vector<int32_t> level(n_, 0);
    for (int32_t e = 0; e < n_; ++e) {
        cl_[e].rep = e;
        cl_[e].add(e);
        sets_[e].push_back(e);
    }
    std::vector<std::vector<MergeJob>> by_level;
    {
        std::vector<int32_t> q(n_);
        for (int32_t e = 0; e < n_; ++e) q[e] = e;
        size_t head = 0;
        while (q.size() - head > 1) {
            const int32_t x = q[head++], y = q[head++];
            const int32_t z = static_cast<int32_t>(level.size());
            const int32_t lv = std::max(level[x], level[y]) + 1;
            level.push_back(lv);
            sets_.emplace_back();
            q.push_back(z);
            if (static_cast<int32_t>(by_level.size()) < lv) by_level.resize(lv);
            MergeJob job;
            job.set1 = x;
            job.set2 = y;
            job.out = z;
            by_level[lv - 1].push_back(job);
        }
    }
    st_.rounds = static_cast<int64_t>(by_level.size());
    for (auto& jobs : by_level) {
        s = merge_level(jobs);
        if (s != CM_OK) return s;
        for (MergeJob& job : jobs) {
            sets_[job.out] = std::move(job.result);
            std::vector<int32_t>().swap(sets_[job.set1]);
            std::vector<int32_t>().swap(sets_[job.set2]);
        }
    }
    if (n_ == 0) sets_.emplace_back();
    const auto t1 = Clock::now();
    cm_result* res = new cm_result();
    s = final_stage(res);
    if (s != CM_OK) { delete res; return s; }
    const auto t2 = Clock::now();
    int64_t needed = 0;
    // speculative work = aligned pairs the replay and the final stage never read
    needed = st_.rep_comparisons + st_.exchange_alignments + (st_.final_candidates - st_.cache_hits);
    st_.speculative_pairs = st_.aligned_pairs > needed ? st_.aligned_pairs - needed : 0;
    st_.t_merge_s = secs(t0, t1);
    st_.t_final_s = secs(t1, t2);
    st_.t_total_s = secs(t0, t2);
    st_.t_host_s = st_.t_total_s - st_.t_gpu_s;
    res->stats = st_;
    *out = res;
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

cm_status cm_clustermerge_run(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                              const cm_params* params, const cm_screen* screen, cm_result** out) {
    if (!ctx || !params || !out) return cmrt::fail(CM_EINVAL, "NULL argument");
    if (!offsets || n_seqs < 0) return cmrt::fail(CM_EINVAL, "bad store");
    if (screen) return cmrt::fail(CM_EUNSUPPORTED, "screen not available in this build");
    *out = nullptr;
    cm_status s = cmrt::check_gaps(params->gap_open, params->gap_extend);
    if (s != CM_OK) return s;
    int8_t mat8[cmk::kNRes * cmk::kMatStride];
    s = cmrt::check_matrix(params->matrix, mat8);
    if (s != CM_OK) return s;
    if (params->T < 1 || params->mT < 0 || params->mU < 0 || params->max_result_pairs < 0)
        return cmrt::fail(CM_EINVAL, "T must be >= 1; mT, mU and max_result_pairs >= 0");
    if (hipSetDevice(ctx->device) != hipSuccess) return cmrt::fail(CM_EDEVICE, "hipSetDevice");
    cmdrv::Driver drv(ctx, seqs, offsets, n_seqs, params);
    return drv.run(out);
}

cm_status cm_result_clusters(const cm_result* r, int32_t* n_clusters, const int32_t** reps,
                             const int64_t** member_offsets, const int32_t** members) {
    if (!r) return cmrt::fail(CM_EINVAL, "result is NULL");
    if (n_clusters) *n_clusters = static_cast<int32_t>(r->reps.size());
    if (reps) *reps = r->reps.data();
    if (member_offsets) *member_offsets = r->member_offsets.data();
    if (members) *members = r->members.data();
    return CM_OK;
}

cm_status cm_result_pairs(const cm_result* r, int64_t* n_pairs, const int32_t** pairs, const int32_t** scores) {
    if (!r) return cmrt::fail(CM_EINVAL, "result is NULL");
    if (n_pairs) *n_pairs = static_cast<int64_t>(r->pair_scores.size());
    if (pairs) *pairs = r->pairs.data();
    if (scores) *scores = r->pair_scores.data();
    return CM_OK;
}

cm_status cm_result_stats(const cm_result* r, cm_stats* out) {
    if (!r || !out) return cmrt::fail(CM_EINVAL, "NULL argument");
    *out = r->stats;
    return CM_OK;
}

void cm_result_free(cm_result* r) { delete r; }

cm_status cm_allvsall_count(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                            const int32_t* matrix, int32_t gap_open, int32_t gap_extend, int32_t T,
                            int64_t* count, double* cells) {
    if (!ctx || !offsets || !count) return cmrt::fail(CM_EINVAL, "NULL argument");
    *count = 0;
    if (cells) *cells = 0;
    if (n_seqs < 2) return CM_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return cmrt::fail(CM_EDEVICE, "hipSetDevice");
    const int64_t total = static_cast<int64_t>(n_seqs) * (n_seqs - 1) / 2;
    const int64_t chunk = std::min<int64_t>(total, 1 << 23);
    cmrt::DeviceBuf& d_pairs = ctx->drv[2];
    cmrt::DeviceBuf& d_sc = ctx->drv[3];
    cmrt::DeviceBuf& d_cnt = ctx->drv[4];
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
}

}  // extern "C"
