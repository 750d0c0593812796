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

struct FwdArgs {
    const uint16_t* feat;
    const int32_t* pairs;
    int32_t n;
    const uint16_t* w1;
    const float* b1;
    const uint16_t* w2;
    const float* b2;
    const uint16_t* w3;
    const float* b3;
    float* z;                  // [n] logits
};


// C = A . B^T (bf16, K contiguous in both; fp32 accumulation) over tiles of
// bm (64 or 128) x 128; blockIdx.z picks the K range [z kper, (z+1) kper)
constexpr int kEpi2Partial = 0;    // Cp[z][m][n] = fp32 partial (bm 64 or 128)
constexpr int kEpi2BiasRelu = 1;   // h = bf16(relu(C + bias[n])) to Cb[m][n] and Ct[n][m] (bm 64)
constexpr int kEpi2MaskT = 2;      // Ct[n][m] = bf16(C) where mask[m][n] != 0, else 0 (bm 64)
constexpr int kEpi2Logit = 3;      // h to Cb[m][n]; zpart[m][n/128] = sum over the tile's n of h w3[n] (bm 64)
struct Gemm2Args {
    const uint16_t* A;         // [M][lda]
    const uint16_t* B;         // [N][ldb]
    int32_t M, N, lda, ldb;
    int32_t kper;              // K per split, a multiple of 128
    float* Cp;
    uint16_t* Cb;
    int32_t ldcb;
    uint16_t* Ct;
    int32_t ldct;
    const float* bias;
    const uint16_t* mask;
    int32_t ldm;
    const uint16_t* w3;
    float* zpart;
};

hipError_t launch_build_x(const uint16_t* feat, const int32_t* pairs, int n, int mb, uint16_t* x, uint16_t* xt,
                          hipStream_t s);
hipError_t launch_gemm2(const Gemm2Args& g, int bm, int epi, int splits, hipStream_t s);
hipError_t launch_reduce(const float* part, int splits, int64_t count, float* out, hipStream_t s);
hipError_t launch_logit_bce(const float* zpart, int tiles, const float* b3, const uint8_t* y, int n, int mb, float* z,
                            float* dz, float* loss, hipStream_t s);
hipError_t launch_adam_pack(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                            float eps, int step, uint16_t* w1, uint16_t* w2, uint16_t* w2t, uint16_t* w3,
                            hipStream_t s);
hipError_t launch_kmer(const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs, uint16_t* feat, uint32_t* err,
                       hipStream_t s);
// inference only (logits): 128 pairs per block, any n
hipError_t launch_infer(const FwdArgs& a, hipStream_t s);
// dH2 = bf16(dz W3 [h2 > 0]) in both layouts; layer-3 weight and bias gradients
hipError_t launch_backward_tail(const float* dz, int n, int mb, const uint16_t* h2, const uint16_t* w3, uint16_t* dh2,
                                uint16_t* dh2t, float* gpart, float* gw3, float* gb3, hipStream_t s);
hipError_t launch_rowsum(const uint16_t* x, int rows, int mb, float* out, hipStream_t s);
hipError_t launch_pack(const float* master, uint16_t* w1, uint16_t* w2, uint16_t* w2t, uint16_t* w3, hipStream_t s);
// rows m < n: pair and label perm[m]; rows n..mb-1: padding (label 0)
hipError_t launch_gather_batch(const int32_t* perm, const int32_t* pairs, const uint8_t* labels, int n, int mb,
                               int32_t* bp, uint8_t* by, hipStream_t s);
// out[0] = mean of loss[0..n), fixed summation order
hipError_t launch_mean(const float* loss, int n, float* out, hipStream_t s);

}  // namespace cms
