// cm_screen.hip -- host side of the learned pair screen (C ABI in include/cm.h).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/cm.h"
#include "cm_runtime.h"
#include "screen_internal.h"

using cmrt::DeviceBuf;
using cmrt::fail;
using cmrt::hip_fail;

struct cm_screen {
    cm_context* ctx = nullptr;
    hipStream_t st = nullptr;
    DeviceBuf master, mom, vel, grad;      // fp32 [kParams]
    DeviceBuf w1, w2, w2t, w3;             // bf16 copies
    // per-batch workspace, sized for cap rows
    DeviceBuf h1, h1t, h2, z, dz, loss, dh2, dh2t, dh1t, xt, x;
    DeviceBuf zpart;                       // fp32 [cap][kHidden / 128]: layer-2 logit partials
    DeviceBuf part;                        // fp32 split-K partials of the weight gradients
    DeviceBuf gpart;                       // fp32 [cap / 64][kHidden]: layer-3 gradient partials
    // training runs: epoch orders, the current batch's rows and labels, loss log
    DeviceBuf perm, bpairs, blabels, losslog;
    int cap = 0;
    int step = 0;
};

namespace {

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

cm_status chk(hipError_t e, const char* what) { return e == hipSuccess ? CM_OK : hip_fail(e, what); }

cm_status alloc_params(cm_screen* s) {
    const size_t pf = cms::kParams * sizeof(float);
    if (!s->master.ensure(pf) || !s->mom.ensure(pf) || !s->vel.ensure(pf) || !s->grad.ensure(pf) ||
        !s->w1.ensure(cms::kW1 * 2) || !s->w2.ensure(cms::kW2 * 2) || !s->w2t.ensure(cms::kW2 * 2) ||
        !s->w3.ensure(cms::kHidden * 2))
        return fail(CM_ENOMEM, "screen parameters");
    return CM_OK;
}

// rows of a padded batch: the training products tile the batch by 128
int64_t pad_rows(int64_t n) { return round_up(n, 128); }

// largest split count <= s_max (a power of two) whose K share is a multiple
// of the products' K step (128)
int splits_for(int mb, int s_max) {
    int sp = s_max;
    while (sp > 1 && mb % (128 * sp) != 0) sp /= 2;
    return sp;
}
constexpr int kSplitW1 = 4, kSplitW2 = 8;

// training workspace for mb rows (every buffer sized for s->cap rows)
cm_status ensure_workspace(cm_screen* s, int mb) {
    if (mb <= s->cap) return CM_OK;
    const int c = mb;
    const size_t hb = static_cast<size_t>(c) * cms::kHidden * 2;
    const size_t parts = std::max<size_t>(static_cast<size_t>(kSplitW1) * cms::kW1, static_cast<size_t>(kSplitW2) * cms::kW2);
    bool ok = s->z.ensure(static_cast<size_t>(c) * 4);
    ok = ok && s->h1.ensure(hb) && s->h1t.ensure(hb) && s->h2.ensure(hb) && s->dz.ensure(c * 4) &&
         s->loss.ensure(c * 4) && s->dh2.ensure(hb) && s->dh2t.ensure(hb) && s->dh1t.ensure(hb) &&
         s->xt.ensure(static_cast<size_t>(c) * cms::kIn * 2) && s->x.ensure(static_cast<size_t>(c) * cms::kIn * 2) &&
         s->zpart.ensure(static_cast<size_t>(c) * (cms::kHidden / 128) * 4) && s->part.ensure(parts * 4) &&
         s->gpart.ensure(static_cast<size_t>(c / 64) * cms::kHidden * 4);
    if (!ok) return fail(CM_ENOMEM, "screen workspace for %d rows", c);
    s->cap = c;
    return CM_OK;
}

cms::FwdArgs fwd_args(const cm_screen* s, const uint16_t* feat, const int32_t* pairs, int n, float* z) {
    cms::FwdArgs a{};
    a.feat = feat;
    a.pairs = pairs;
    a.n = n;
    a.w1 = static_cast<const uint16_t*>(s->w1.ptr);
    a.w2 = static_cast<const uint16_t*>(s->w2.ptr);
    a.w3 = static_cast<const uint16_t*>(s->w3.ptr);
    const float* m = static_cast<const float*>(s->master.ptr);
    a.b1 = m + cms::kOffB1;
    a.b2 = m + cms::kOffB2;
    a.b3 = m + cms::kOffB3;
    a.z = z;
    return a;
}

// forward + backward of the mean BCE on one batch; gradients in s->grad.
// The batch is padded to mb rows (a multiple of 128); padding rows have zero
// inputs and contribute nothing (their dz is 0).
cm_status forward_backward(cm_screen* s, const uint16_t* feat, const int32_t* pairs, const uint8_t* labels, int n,
                           float* loss_out) {
    const int mb = static_cast<int>(pad_rows(n));
    cm_status r = ensure_workspace(s, mb);
    if (r != CM_OK) return r;
    hipStream_t st = s->st;
    uint16_t* x = static_cast<uint16_t*>(s->x.ptr);
    uint16_t* xt = static_cast<uint16_t*>(s->xt.ptr);
    uint16_t* h1 = static_cast<uint16_t*>(s->h1.ptr);
    uint16_t* h1t = static_cast<uint16_t*>(s->h1t.ptr);
    uint16_t* h2 = static_cast<uint16_t*>(s->h2.ptr);
    uint16_t* dh2 = static_cast<uint16_t*>(s->dh2.ptr);
    uint16_t* dh2t = static_cast<uint16_t*>(s->dh2t.ptr);
    uint16_t* dh1t = static_cast<uint16_t*>(s->dh1t.ptr);
    float* part = static_cast<float*>(s->part.ptr);
    float* zpart = static_cast<float*>(s->zpart.ptr);
    float* g = static_cast<float*>(s->grad.ptr);
    const float* master = static_cast<const float*>(s->master.ptr);
    const uint16_t* w1 = static_cast<const uint16_t*>(s->w1.ptr);
    const uint16_t* w2 = static_cast<const uint16_t*>(s->w2.ptr);
    const uint16_t* w2t = static_cast<const uint16_t*>(s->w2t.ptr);
    const uint16_t* w3 = static_cast<const uint16_t*>(s->w3.ptr);
    if ((r = chk(cms::launch_build_x(feat, pairs, n, mb, x, xt, st), "pair inputs")) != CM_OK) return r;
    cms::Gemm2Args q{};
    // h1 = relu(X W1^T + b1), row-major and transposed
    q.A = x; q.B = w1; q.M = mb; q.N = cms::kHidden; q.lda = cms::kIn; q.ldb = cms::kIn; q.kper = cms::kIn;
    q.Cb = h1; q.ldcb = cms::kHidden; q.Ct = h1t; q.ldct = mb; q.bias = master + cms::kOffB1;
    if ((r = chk(cms::launch_gemm2(q, 64, cms::kEpi2BiasRelu, 1, st), "layer 1")) != CM_OK) return r;
    // h2 = relu(h1 W2^T + b2) and the logit partials of every 128 units
    q = {};
    q.A = h1; q.B = w2; q.M = mb; q.N = cms::kHidden; q.lda = cms::kHidden; q.ldb = cms::kHidden;
    q.kper = cms::kHidden; q.Cb = h2; q.ldcb = cms::kHidden; q.bias = master + cms::kOffB2; q.w3 = w3;
    q.zpart = zpart;
    if ((r = chk(cms::launch_gemm2(q, 64, cms::kEpi2Logit, 1, st), "layer 2")) != CM_OK) return r;
    if ((r = chk(cms::launch_logit_bce(zpart, cms::kHidden / 128, master + cms::kOffB3, labels, n, mb,
                                       static_cast<float*>(s->z.ptr), static_cast<float*>(s->dz.ptr),
                                       static_cast<float*>(s->loss.ptr), st),
                 "loss")) != CM_OK)
        return r;
    // dH2 (both layouts), layer-3 gradients
    if ((r = chk(cms::launch_backward_tail(static_cast<float*>(s->dz.ptr), n, mb, h2, w3, dh2, dh2t,
                                           static_cast<float*>(s->gpart.ptr), g + cms::kOffW3, g + cms::kOffB3, st),
                 "layer-3 backward")) != CM_OK)
        return r;
    // dW2[i][j] = sum_m dH2[m][i] H1[m][j]: split over the batch, partials added in order
    const int s2 = splits_for(mb, kSplitW2);
    q = {};
    q.A = dh2t; q.B = h1t; q.M = cms::kHidden; q.N = cms::kHidden; q.lda = mb; q.ldb = mb; q.kper = mb / s2;
    q.Cp = part;
    if ((r = chk(cms::launch_gemm2(q, 128, cms::kEpi2Partial, s2, st), "dW2")) != CM_OK) return r;
    if ((r = chk(cms::launch_reduce(part, s2, cms::kW2, g + cms::kOffW2, st), "dW2 sum")) != CM_OK) return r;
    // dH1^T[j][m] = (sum_i dH2[m][i] W2[i][j]) * [h1[m][j] > 0]
    q = {};
    q.A = dh2; q.B = w2t; q.M = mb; q.N = cms::kHidden; q.lda = cms::kHidden; q.ldb = cms::kHidden;
    q.kper = cms::kHidden; q.Ct = dh1t; q.ldct = mb; q.mask = h1; q.ldm = cms::kHidden;
    if ((r = chk(cms::launch_gemm2(q, 64, cms::kEpi2MaskT, 1, st), "dH1")) != CM_OK) return r;
    // dW1[i][k] = sum_m dH1[m][i] X[m][k]
    const int s1 = splits_for(mb, kSplitW1);
    q = {};
    q.A = dh1t; q.B = xt; q.M = cms::kHidden; q.N = cms::kIn; q.lda = mb; q.ldb = mb; q.kper = mb / s1; q.Cp = part;
    if ((r = chk(cms::launch_gemm2(q, 128, cms::kEpi2Partial, s1, st), "dW1")) != CM_OK) return r;
    if ((r = chk(cms::launch_reduce(part, s1, cms::kW1, g + cms::kOffW1, st), "dW1 sum")) != CM_OK) return r;
    if ((r = chk(cms::launch_rowsum(dh2t, cms::kHidden, mb, g + cms::kOffB2, st), "db2")) != CM_OK) return r;
    if ((r = chk(cms::launch_rowsum(dh1t, cms::kHidden, mb, g + cms::kOffB1, st), "db1")) != CM_OK) return r;
    if (loss_out) {
        std::vector<float> lv(n);
        if ((r = chk(hipMemcpyAsync(lv.data(), s->loss.ptr, n * 4, hipMemcpyDeviceToHost, st), "loss")) != CM_OK)
            return r;
        if ((r = chk(hipStreamSynchronize(st), "screen step")) != CM_OK) return r;
        double t = 0;
        for (float v : lv) t += v;
        *loss_out = static_cast<float>(t / n);
    }
    return CM_OK;
}

uint64_t splitmix(uint64_t& x) {
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// the order of epoch `e`: 0..n-1 shuffled by Fisher-Yates with a splitmix64
// stream seeded from (seed, e), or the identity
void epoch_order(int64_t n, bool shuffle, uint64_t seed, int64_t e, int32_t* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = static_cast<int32_t>(i);
    if (!shuffle) return;
    uint64_t x = seed ^ (0xd1b54a32d192ed03ull * static_cast<uint64_t>(e + 1));
    for (int64_t i = n - 1; i > 0; --i) {
        // uniform j in [0, i] by rejection on the top bits
        const uint64_t bound = static_cast<uint64_t>(i) + 1;
        const uint64_t lim = UINT64_MAX - UINT64_MAX % bound;
        uint64_t r;
        do { r = splitmix(x); } while (r >= lim);
        const int64_t j = static_cast<int64_t>(r % bound);
        const int32_t t = out[i];
        out[i] = out[j];
        out[j] = t;
    }
}

cm_status upload_master(cm_screen* s, const float* host) {
    cm_status r = chk(hipMemcpyAsync(s->master.ptr, host, cms::kParams * 4, hipMemcpyHostToDevice, s->st), "weights");
    if (r != CM_OK) return r;
    r = chk(cms::launch_pack(static_cast<const float*>(s->master.ptr), static_cast<uint16_t*>(s->w1.ptr),
                             static_cast<uint16_t*>(s->w2.ptr), static_cast<uint16_t*>(s->w2t.ptr),
                             static_cast<uint16_t*>(s->w3.ptr), s->st),
            "pack");
    if (r != CM_OK) return r;
    return chk(hipStreamSynchronize(s->st), "upload");
}

// one Adam update of the master weights from s->grad and, in the same pass,
// the bf16 copies the network reads
cm_status adam_step(cm_screen* s, float lr) {
    s->step += 1;
    return chk(cms::launch_adam_pack(static_cast<float*>(s->master.ptr), static_cast<const float*>(s->grad.ptr),
                                     static_cast<float*>(s->mom.ptr), static_cast<float*>(s->vel.ptr), cms::kParams,
                                     lr, 0.9f, 0.999f, 1e-8f, s->step, static_cast<uint16_t*>(s->w1.ptr),
                                     static_cast<uint16_t*>(s->w2.ptr), static_cast<uint16_t*>(s->w2t.ptr),
                                     static_cast<uint16_t*>(s->w3.ptr), s->st),
               "adam");
}

int64_t train_steps(int64_t n, const cm_train_cfg* c) {
    return c->drop_last ? n / c->batch : (n + c->batch - 1) / c->batch;
}

cm_status reset_adam(cm_screen* s) {
    s->step = 0;
    cm_status r = chk(hipMemsetAsync(s->mom.ptr, 0, cms::kParams * 4, s->st), "adam state");
    if (r == CM_OK) r = chk(hipMemsetAsync(s->vel.ptr, 0, cms::kParams * 4, s->st), "adam state");
    return r;
}

}  // namespace

extern "C" {

cm_status cm_kmer_features(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                           uint16_t* feat, void* stream) {
    CM_TRY
    if (!ctx || !offsets || !feat || n_seqs < 0) return fail(CM_EINVAL, "bad argument");
    if (n_seqs == 0) return CM_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(CM_EDEVICE, "hipSetDevice");
    return chk(cms::launch_kmer(seqs ? seqs : ctx->dummy, offsets, n_seqs, feat, ctx->err_flag,
                                static_cast<hipStream_t>(stream)),
               "features");
    CM_CATCH
}

cm_status cm_screen_create(cm_context* ctx, uint64_t seed, cm_screen** out) {
    CM_TRY
    if (!ctx || !out) return fail(CM_EINVAL, "bad argument");
    *out = nullptr;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(CM_EDEVICE, "hipSetDevice");
    cm_screen* s = new cm_screen();
    s->ctx = ctx;
    cm_status r = chk(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking), "stream");
    if (r == CM_OK) r = alloc_params(s);
    if (r != CM_OK) { cm_screen_destroy(s); return r; }
    // Kaiming-uniform weights (bound sqrt(6 / fan_in)), zero biases
    std::vector<float> w(cms::kParams, 0.f);
    uint64_t x = seed;
    auto fill = [&](int64_t off, int64_t count, int fan_in) {
        const double bound = std::sqrt(6.0 / fan_in);
        for (int64_t i = 0; i < count; ++i) {
            const double u = static_cast<double>(splitmix(x) >> 11) * (1.0 / 9007199254740992.0);
            w[off + i] = static_cast<float>((2.0 * u - 1.0) * bound);
        }
    };
    fill(cms::kOffW1, cms::kW1, cms::kIn);
    fill(cms::kOffW2, cms::kW2, cms::kHidden);
    fill(cms::kOffW3, cms::kHidden, cms::kHidden);
    r = upload_master(s, w.data());
    if (r == CM_OK) r = reset_adam(s);
    if (r == CM_OK) r = chk(hipStreamSynchronize(s->st), "screen init");
    if (r != CM_OK) { cm_screen_destroy(s); return r; }
    *out = s;
    return CM_OK;
    CM_CATCH
}

void cm_screen_destroy(cm_screen* s) {
    CM_TRY
    if (!s) return;
    if (s->st) { (void)hipStreamSynchronize(s->st); (void)hipStreamDestroy(s->st); }
    for (DeviceBuf* b : {&s->master, &s->mom, &s->vel, &s->grad, &s->w1, &s->w2, &s->w2t, &s->w3, &s->h1, &s->h1t,
                         &s->h2, &s->z, &s->dz, &s->loss, &s->dh2, &s->dh2t, &s->dh1t, &s->xt, &s->x,
                         &s->zpart, &s->part, &s->gpart,
                         &s->perm, &s->bpairs, &s->blabels, &s->losslog})
        b->release();
    delete s;
    CM_CATCH_VOID
}

int64_t cm_screen_num_params(void) { return cms::kParams; }

cm_status cm_screen_set_weights(cm_screen* s, const float* host_fp32_master) {
    CM_TRY
    if (!s || !host_fp32_master) return fail(CM_EINVAL, "bad argument");
    cm_status r = upload_master(s, host_fp32_master);
    if (r == CM_OK) r = reset_adam(s);
    if (r == CM_OK) r = chk(hipStreamSynchronize(s->st), "set weights");
    return r;
    CM_CATCH
}

cm_status cm_screen_get_weights(const cm_screen* s, float* host_fp32_master, uint16_t* host_bf16) {
    CM_TRY
    if (!s) return fail(CM_EINVAL, "bad argument");
    if (host_fp32_master) {
        cm_status r = chk(hipMemcpy(host_fp32_master, s->master.ptr, cms::kParams * 4, hipMemcpyDeviceToHost), "get");
        if (r != CM_OK) return r;
    }
    if (host_bf16) {
        // W1, W2, W3 bf16 copies, concatenated
        cm_status r = chk(hipMemcpy(host_bf16, s->w1.ptr, cms::kW1 * 2, hipMemcpyDeviceToHost), "get");
        if (r == CM_OK) r = chk(hipMemcpy(host_bf16 + cms::kW1, s->w2.ptr, cms::kW2 * 2, hipMemcpyDeviceToHost), "get");
        if (r == CM_OK)
            r = chk(hipMemcpy(host_bf16 + cms::kW1 + cms::kW2, s->w3.ptr, cms::kHidden * 2, hipMemcpyDeviceToHost),
                    "get");
        if (r != CM_OK) return r;
    }
    return CM_OK;
    CM_CATCH
}

cm_status cm_screen_infer(const cm_screen* s_, const uint16_t* feat, const int32_t* pairs, int64_t n_pairs,
                          float* logits, void* stream) {
    CM_TRY
    cm_screen* s = const_cast<cm_screen*>(s_);
    if (!s || !feat || !pairs || !logits || n_pairs < 0) return fail(CM_EINVAL, "bad argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t chunk = 1 << 24;
    for (int64_t first = 0; first < n_pairs; first += chunk) {
        const int n = static_cast<int>(n_pairs - first < chunk ? n_pairs - first : chunk);
        cms::FwdArgs a = fwd_args(s, feat, pairs + 2 * first, n, logits + first);
        cm_status r = chk(cms::launch_infer(a, st), "screen inference");
        if (r != CM_OK) return r;
    }
    return CM_OK;
    CM_CATCH
}

cm_status cm_screen_grads(cm_screen* s, const uint16_t* feat, const int32_t* pairs, const uint8_t* labels,
                          int64_t n_pairs, float* host_grads, float* loss) {
    CM_TRY
    if (!s || !feat || !pairs || !labels || n_pairs <= 0 || n_pairs > (1 << 20)) return fail(CM_EINVAL, "bad argument");
    cm_status r = forward_backward(s, feat, pairs, labels, static_cast<int>(n_pairs), loss);
    if (r != CM_OK) return r;
    if (host_grads) r = chk(hipMemcpy(host_grads, s->grad.ptr, cms::kParams * 4, hipMemcpyDeviceToHost), "grads");
    return r;
    CM_CATCH
}

cm_status cm_screen_train_step(cm_screen* s, const uint16_t* feat, const int32_t* pairs, const uint8_t* labels,
                               int64_t n_pairs, float lr, float* loss) {
    CM_TRY
    if (!s || !feat || !pairs || !labels || n_pairs <= 0 || n_pairs > (1 << 20) || !(lr > 0.f))
        return fail(CM_EINVAL, "bad argument");
    cm_status r = forward_backward(s, feat, pairs, labels, static_cast<int>(n_pairs), loss);
    if (r != CM_OK) return r;
    r = adam_step(s, lr);
    if (r != CM_OK) return r;
    return chk(hipStreamSynchronize(s->st), "train step");
    CM_CATCH
}

int64_t cm_screen_train_steps(int64_t n_pairs, const cm_train_cfg* cfg) {
    if (!cfg || n_pairs < 0 || cfg->batch < 1 || cfg->epochs < 0) return -1;
    return static_cast<int64_t>(cfg->epochs) * train_steps(n_pairs, cfg);
}

cm_status cm_screen_train(cm_screen* s, const uint16_t* feat, const int32_t* pairs, const uint8_t* labels,
                          int64_t n_pairs, const cm_train_cfg* cfg, float* loss_log) {
    CM_TRY
    if (!s || !feat || !pairs || !labels || !cfg) return fail(CM_EINVAL, "NULL argument");
    if (n_pairs < 1 || n_pairs > 0x7fffffff) return fail(CM_EINVAL, "n_pairs must be in [1, 2^31 - 1]");
    if (cfg->epochs < 1 || cfg->batch < 1 || cfg->batch > (1 << 20) || !(cfg->lr > 0.f) ||
        (cfg->shuffle != 0 && cfg->shuffle != 1) || (cfg->drop_last != 0 && cfg->drop_last != 1))
        return fail(CM_EINVAL, "training config: epochs >= 1, batch in [1, 2^20], lr > 0, shuffle and drop_last 0/1");
    const int64_t per_epoch = train_steps(n_pairs, cfg);
    if (per_epoch < 1) return fail(CM_EINVAL, "no full batch of %d pairs in %lld", cfg->batch,
                                   static_cast<long long>(n_pairs));
    const int64_t steps = per_epoch * cfg->epochs;
    const int mb_max = static_cast<int>(pad_rows(std::min<int64_t>(cfg->batch, n_pairs)));
    cm_status r = ensure_workspace(s, mb_max);
    if (r != CM_OK) return r;
    if (!s->perm.ensure(static_cast<size_t>(n_pairs) * 4 * cfg->epochs) ||
        !s->bpairs.ensure(static_cast<size_t>(mb_max) * 8) || !s->blabels.ensure(static_cast<size_t>(mb_max)) ||
        !s->losslog.ensure(static_cast<size_t>(steps) * 4))
        return fail(CM_ENOMEM, "training run buffers");
    // every epoch's order, uploaded once (the host copy lives until the end)
    std::vector<int32_t> order(static_cast<size_t>(n_pairs) * cfg->epochs);
    for (int e = 0; e < cfg->epochs; ++e)
        epoch_order(n_pairs, cfg->shuffle != 0, cfg->seed, e, order.data() + static_cast<size_t>(e) * n_pairs);
    hipStream_t st = s->st;
    r = chk(hipMemcpyAsync(s->perm.ptr, order.data(), order.size() * 4, hipMemcpyHostToDevice, st), "orders");
    if (r != CM_OK) return r;
    int32_t* bp = static_cast<int32_t*>(s->bpairs.ptr);
    uint8_t* by = static_cast<uint8_t*>(s->blabels.ptr);
    float* log = static_cast<float*>(s->losslog.ptr);
    int64_t k = 0;
    for (int e = 0; e < cfg->epochs; ++e) {
        const int32_t* perm = static_cast<const int32_t*>(s->perm.ptr) + static_cast<size_t>(e) * n_pairs;
        for (int64_t b = 0; b < per_epoch; ++b, ++k) {
            const int64_t first = b * cfg->batch;
            const int n = static_cast<int>(std::min<int64_t>(cfg->batch, n_pairs - first));
            const int mb = static_cast<int>(pad_rows(n));
            r = chk(cms::launch_gather_batch(perm + first, pairs, labels, n, mb, bp, by, st), "batch gather");
            if (r == CM_OK) r = forward_backward(s, feat, bp, by, n, nullptr);
            if (r == CM_OK) r = chk(cms::launch_mean(static_cast<const float*>(s->loss.ptr), n, log + k, st), "loss");
            if (r == CM_OK) r = adam_step(s, cfg->lr);
            if (r != CM_OK) return r;
        }
    }
    if (loss_log) {
        r = chk(hipMemcpyAsync(loss_log, log, static_cast<size_t>(steps) * 4, hipMemcpyDeviceToHost, st), "loss log");
        if (r != CM_OK) return r;
    }
    return chk(hipStreamSynchronize(st), "training run");
    CM_CATCH
}

cm_status cm_screen_save(const cm_screen* s, const char* path) {
    CM_TRY
    if (!s || !path) return fail(CM_EINVAL, "bad argument");
    std::vector<float> buf(3 * cms::kParams);
    cm_status r = chk(hipMemcpy(buf.data(), s->master.ptr, cms::kParams * 4, hipMemcpyDeviceToHost), "save");
    if (r == CM_OK) r = chk(hipMemcpy(buf.data() + cms::kParams, s->mom.ptr, cms::kParams * 4, hipMemcpyDeviceToHost), "save");
    if (r == CM_OK)
        r = chk(hipMemcpy(buf.data() + 2 * cms::kParams, s->vel.ptr, cms::kParams * 4, hipMemcpyDeviceToHost), "save");
    if (r != CM_OK) return r;
    FILE* f = fopen(path, "wb");
    if (!f) return fail(CM_EINVAL, "cannot open %s", path);
    const char magic[8] = {'C', 'M', 'S', 'C', 'R', 'N', '0', '1'};
    const int64_t hdr[2] = {cms::kParams, s->step};
    bool ok = fwrite(magic, 1, 8, f) == 8 && fwrite(hdr, 8, 2, f) == 2 &&
              fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    ok = (fclose(f) == 0) && ok;
    return ok ? CM_OK : fail(CM_EINVAL, "write failed: %s", path);
    CM_CATCH
}

cm_status cm_screen_load(cm_context* ctx, const char* path, cm_screen** out) {
    CM_TRY
    if (!ctx || !path || !out) return fail(CM_EINVAL, "bad argument");
    *out = nullptr;
    FILE* f = fopen(path, "rb");
    if (!f) return fail(CM_EINVAL, "cannot open %s", path);
    char magic[8];
    int64_t hdr[2];
    std::vector<float> buf(3 * cms::kParams);
    const bool ok = fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "CMSCRN01", 8) == 0 &&
                    fread(hdr, 8, 2, f) == 2 && hdr[0] == cms::kParams &&
                    fread(buf.data(), 4, buf.size(), f) == buf.size();
    fclose(f);
    if (!ok) return fail(CM_EINVAL, "not a screen file: %s", path);
    cm_screen* s = nullptr;
    cm_status r = cm_screen_create(ctx, 0, &s);
    if (r != CM_OK) return r;
    r = upload_master(s, buf.data());
    if (r == CM_OK)
        r = chk(hipMemcpy(s->mom.ptr, buf.data() + cms::kParams, cms::kParams * 4, hipMemcpyHostToDevice), "load");
    if (r == CM_OK)
        r = chk(hipMemcpy(s->vel.ptr, buf.data() + 2 * cms::kParams, cms::kParams * 4, hipMemcpyHostToDevice), "load");
    if (r != CM_OK) { cm_screen_destroy(s); return r; }
    s->step = static_cast<int>(hdr[1]);
    *out = s;
    return CM_OK;
    CM_CATCH
}

}  // extern "C"
