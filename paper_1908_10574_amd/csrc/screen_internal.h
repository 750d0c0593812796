// screen_internal.h -- shapes and launchers of the learned pair screen.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cms {

constexpr int kBuckets = 1024;                 // hashed 3-mer features per protein
constexpr int kIn = 2 * kBuckets;              // pair input: |a - b| and a * b
constexpr int kHidden = 512;
constexpr int64_t kW1 = static_cast<int64_t>(kHidden) * kIn;
constexpr int64_t kW2 = static_cast<int64_t>(kHidden) * kHidden;
// fp32 master vector: W1, b1, W2, b2, W3, b3
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + kW1;
constexpr int64_t kOffW2 = kOffB1 + kHidden;
constexpr int64_t kOffB2 = kOffW2 + kW2;
constexpr int64_t kOffW3 = kOffB2 + kHidden;
constexpr int64_t kOffB3 = kOffW3 + kHidden;
constexpr int64_t kParams = kOffB3 + 1;

constexpr int kEpiF32 = 0;     // C fp32 row-major
constexpr int kEpiMaskT = 1;   // C^T bf16, zero where mask == 0

struct FwdArgs {
    const uint16_t* feat;
    const int32_t* pairs;
    int32_t n;
    int32_t ld_t;              // leading dimension of h1t (padded batch)
    const uint16_t* w1;
    const float* b1;
    const uint16_t* w2;
    const float* b2;
    const uint16_t* w3;
    const float* b3;
    float* z;                  // [n] logits
    uint16_t* h1;              // optional [mb][512]
    uint16_t* h1t;             // optional [512][ld_t]
    uint16_t* h2;              // optional [mb][512]
};

struct GemmArgs {
    const uint16_t* A;
    const uint16_t* B;
    int32_t M, N, K, lda, ldb, ldc;
    float* Cf;                 // kEpiF32
    uint16_t* Cb;              // kEpiMaskT
    const uint16_t* mask;
    int32_t ldm;
};

hipError_t launch_kmer(const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs, uint16_t* feat, uint32_t* err,
                       hipStream_t s);
hipError_t launch_fwd(const FwdArgs& a, int mb, hipStream_t s);
// inference only (logits): 128 pairs per block, any n
hipError_t launch_infer(const FwdArgs& a, hipStream_t s);
hipError_t launch_pair_xt(const uint16_t* feat, const int32_t* pairs, int n, int mb, uint16_t* xt, hipStream_t s);
hipError_t launch_gemm(const GemmArgs& g, int epi, hipStream_t s);
hipError_t launch_backward_tail(const float* z, const uint8_t* y, int n, int mb, const uint16_t* h2,
                                const uint16_t* w3, float* dz, float* loss, uint16_t* dh2, uint16_t* dh2t,
                                float* gpart, float* gw3, float* gb3, hipStream_t s);
hipError_t launch_rowsum(const uint16_t* x, int rows, int mb, float* out, hipStream_t s);
hipError_t launch_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s);
hipError_t launch_pack(const float* master, uint16_t* w1, uint16_t* w2, uint16_t* w2t, uint16_t* w3, hipStream_t s);
// rows m < n: pair and label perm[m]; rows n..mb-1: padding (label 0)
hipError_t launch_gather_batch(const int32_t* perm, const int32_t* pairs, const uint8_t* labels, int n, int mb,
                               int32_t* bp, uint8_t* by, hipStream_t s);
// out[0] = mean of loss[0..n), fixed summation order
hipError_t launch_mean(const float* loss, int n, float* out, hipStream_t s);

}  // namespace cms
