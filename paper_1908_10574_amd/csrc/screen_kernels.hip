// screen_kernels.hip -- learned pair screen for gfx950: hashed 3-mer features,
// a 2048-512-512-1 MLP on bf16 MFMA with fp32 accumulation, its backward pass
// and Adam.  The screen sits in front of the exact alignment (it decides which
// candidate pairs are aligned at all); it never changes a score.
//
// Layouts (row-major, bf16 stored as uint16 bit patterns):
//   feat  [n_seqs][1024]   count/8 of hashed 3-mers
//   X     [M][2048]        [|fa - fb|, fa * fb] per pair, built on the fly
//   W1    [512][2048], W2 [512][512], W2T [512][512] (= W2 transposed), W3 [512]
//   master fp32: W1, b1, W2, b2, W3, b3 (one vector, 1,312,257 values)
// MFMA v_mfma_f32_16x16x32_bf16 operand layout (lane l):
//   A[l%16][8*(l/16) + j], B[8*(l/16) + j][l%16], D[4*(l/16) + i][l%16].
#include "screen_internal.h"

namespace cms {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
    // round to nearest even on the fp32 bit pattern (inputs here are finite)
    const uint32_t u = __float_as_uint(f);
    return static_cast<uint16_t>((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) { return *reinterpret_cast<const bf16x8*>(p); }

// ---------------------------------------------------------------------------
// features: one block per protein, LDS histogram of hashed 3-mers
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_kmer(const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs,
                                              uint16_t* feat, uint32_t* err) {
    __shared__ int hist[kBuckets];
    const int s = blockIdx.x;
    for (int b = threadIdx.x; b < kBuckets; b += 256) hist[b] = 0;
    __syncthreads();
    const uint8_t* q = seqs + offsets[s];
    const int64_t L = offsets[s + 1] - offsets[s];
    bool bad = false;
    for (int64_t p = threadIdx.x; p + 2 < L; p += 256) {
        const uint32_t a = q[p], b = q[p + 1], c = q[p + 2];
        if (a > 19 || b > 19 || c > 19) { bad = true; continue; }
        const uint32_t code = 400u * a + 20u * b + c;
        atomicAdd(&hist[(code * 2654435761u) >> 22], 1);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBuckets; b += 256)
        feat[static_cast<int64_t>(s) * kBuckets + b] = f2bf(static_cast<float>(hist[b]) * 0.125f);
    if (bad) atomicOr(err, 1u);
}

// ---------------------------------------------------------------------------
// fused forward: 32 pairs per block, 4 waves, each wave owns 128 hidden units
// ---------------------------------------------------------------------------
constexpr int kRows = 32;          // pairs per block
constexpr int kKc = 256;           // layer-1 K chunk staged in LDS

__global__ __launch_bounds__(256) void k_mlp_fwd(FwdArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t xs[kRows][kKc + 8];
    __shared__ __attribute__((aligned(16))) uint16_t h1s[kRows][kHidden + 8];
    __shared__ float zpart[4][kRows];
    __shared__ int pa[kRows], pb[kRows];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m0 = blockIdx.x * kRows;
    if (tid < kRows) {
        const int m = m0 + tid;
        pa[tid] = m < a.n ? a.pairs[2 * m] : 0;
        pb[tid] = m < a.n ? a.pairs[2 * m + 1] : 0;
    }
    __syncthreads();
    const int r = lane & 15, kq = (lane >> 4) * 8;
    const int nw = wave * 128;                       // this wave's first hidden unit
    f32x4 acc[2][8];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[i][c] = f32x4{0.f, 0.f, 0.f, 0.f};

    // ---- layer 1: X [32 x 2048] . W1^T
    const int br = tid >> 3, bk = (tid & 7) * 32;    // builder: row, 32-wide k slice
    for (int kc = 0; kc < kIn; kc += kKc) {
        {
            const int kk = (kc + bk) & (kBuckets - 1);
            const uint16_t* fa = a.feat + static_cast<int64_t>(pa[br]) * kBuckets + kk;
            const uint16_t* fb = a.feat + static_cast<int64_t>(pb[br]) * kBuckets + kk;
            const bool diff = (kc + bk) < kBuckets;
#pragma unroll
            for (int v = 0; v < 32; v += 8) {
                const bf16x8 va = ld8(fa + v), vb = ld8(fb + v);
                uint16_t o[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const float x = static_cast<float>(va[j]), y = static_cast<float>(vb[j]);
                    o[j] = f2bf(diff ? fabsf(x - y) : x * y);
                }
#pragma unroll
                for (int j = 0; j < 8; ++j) xs[br][bk + v + j] = o[j];
            }
        }
        __syncthreads();
#pragma unroll 2
        for (int ks = 0; ks < kKc; ks += 32) {
            const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(&xs[r][ks + kq]);
            const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(&xs[16 + r][ks + kq]);
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const bf16x8 b = ld8(a.w1 + static_cast<int64_t>(nw + 16 * c + r) * kIn + kc + ks + kq);
                acc[0][c] = mfma(a0, b, acc[0][c]);
                acc[1][c] = mfma(a1, b, acc[1][c]);
            }
        }
        __syncthreads();
    }
    // epilogue 1: h1 = bf16(relu(acc + b1)) -> LDS (and global for training)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int n = nw + 16 * c + r;
            const float bias = a.b1[n];
            uint16_t h[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 16 * i + 4 * (lane >> 4) + q;
                h[q] = f2bf(fmaxf(acc[i][c][q] + bias, 0.f));
                h1s[row][n] = h[q];
                if (a.h1) a.h1[static_cast<int64_t>(m0 + row) * kHidden + n] = h[q];
            }
            if (a.h1t) {
                const int row = 16 * i + 4 * (lane >> 4);
                uint2 pk;
                pk.x = static_cast<uint32_t>(h[0]) | (static_cast<uint32_t>(h[1]) << 16);
                pk.y = static_cast<uint32_t>(h[2]) | (static_cast<uint32_t>(h[3]) << 16);
                *reinterpret_cast<uint2*>(a.h1t + static_cast<int64_t>(n) * a.ld_t + m0 + row) = pk;
            }
            acc[i][c] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    __syncthreads();

    // ---- layer 2: h1 [32 x 512] . W2^T
#pragma unroll 2
    for (int ks = 0; ks < kHidden; ks += 32) {
        const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(&h1s[r][ks + kq]);
        const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(&h1s[16 + r][ks + kq]);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const bf16x8 b = ld8(a.w2 + static_cast<int64_t>(nw + 16 * c + r) * kHidden + ks + kq);
            acc[0][c] = mfma(a0, b, acc[0][c]);
            acc[1][c] = mfma(a1, b, acc[1][c]);
        }
    }
    // epilogue 2: h2 = bf16(relu(acc + b2)); partial logit sum over this wave's units
    float zp[2][4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int n = nw + 16 * c + r;
            const float bias = a.b2[n];
            const float w3 = bf2f(a.w3[n]);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 16 * i + 4 * (lane >> 4) + q;
                const uint16_t h = f2bf(fmaxf(acc[i][c][q] + bias, 0.f));
                if (a.h2) a.h2[static_cast<int64_t>(m0 + row) * kHidden + n] = h;
                zp[i][q] += bf2f(h) * w3;
            }
        }
    // sum over the 16 lanes that share rows (they hold different units)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float v = zp[i][q];
#pragma unroll
            for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 16);
            zp[i][q] = v;
        }
    if (r == 0) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) zpart[wave][16 * i + 4 * (lane >> 4) + q] = zp[i][q];
    }
    __syncthreads();
    if (tid < kRows) {
        const int m = m0 + tid;
        const float z = zpart[0][tid] + zpart[1][tid] + zpart[2][tid] + zpart[3][tid] + a.b3[0];
        if (m < a.n) a.z[m] = z;
    }
}

// ---------------------------------------------------------------------------
// inference forward: 128 pairs per block, 8 waves, each wave owns 64 hidden
// units for all 128 rows, so every weight fragment loaded from L2 feeds 8
// row tiles (4x the reuse of k_mlp_fwd).  Same rounding points as k_mlp_fwd
// (X, h1, h2 rounded to bf16; fp32 accumulation), no training outputs.
// The pair input is built 32 columns at a time into a double-buffered LDS
// tile, its feature loads issued one step ahead.
// ---------------------------------------------------------------------------
constexpr int kIR = 128;           // pairs per block
constexpr int kIW = 8;             // waves per block
constexpr int kIK = 32;            // layer-1 K step

__global__ __launch_bounds__(512) void k_mlp_infer(FwdArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t xs[2][kIR][kIK + 8];
    __shared__ __attribute__((aligned(16))) uint16_t h1s[kIR][kHidden + 8];
    __shared__ float zpart[kIW][kIR];
    __shared__ int pa[kIR], pb[kIR];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t m0 = static_cast<int64_t>(blockIdx.x) * kIR;
    if (tid < kIR) {
        const int64_t m = m0 + tid;
        pa[tid] = m < a.n ? a.pairs[2 * m] : 0;
        pb[tid] = m < a.n ? a.pairs[2 * m + 1] : 0;
    }
    __syncthreads();
    const int r = lane & 15, kq = (lane >> 4) * 8;
    const int nw = wave * 64;                        // this wave's first hidden unit
    f32x4 acc[8][4];
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};

    // ---- layer 1: X [128 x 2048] . W1^T
    const int br = tid >> 2, bk = (tid & 3) * 8;     // builder: row, 8 columns of the step
    const uint16_t* fa = a.feat + static_cast<int64_t>(pa[br]) * kBuckets;
    const uint16_t* fb = a.feat + static_cast<int64_t>(pb[br]) * kBuckets;
    bf16x8 va = ld8(fa + bk), vb = ld8(fb + bk);
    constexpr int kSteps = kIn / kIK;
    for (int s = 0; s < kSteps; ++s) {
        const int kc = s * kIK;
        bf16x8 b[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) b[c] = ld8(a.w1 + static_cast<int64_t>(nw + 16 * c + r) * kIn + kc + kq);
        {
            const bool diff = kc < kBuckets;
            uint16_t o[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float x = static_cast<float>(va[j]), y = static_cast<float>(vb[j]);
                o[j] = f2bf(diff ? fabsf(x - y) : x * y);
            }
            uint4 pk;
            pk.x = static_cast<uint32_t>(o[0]) | (static_cast<uint32_t>(o[1]) << 16);
            pk.y = static_cast<uint32_t>(o[2]) | (static_cast<uint32_t>(o[3]) << 16);
            pk.z = static_cast<uint32_t>(o[4]) | (static_cast<uint32_t>(o[5]) << 16);
            pk.w = static_cast<uint32_t>(o[6]) | (static_cast<uint32_t>(o[7]) << 16);
            *reinterpret_cast<uint4*>(&xs[s & 1][br][bk]) = pk;
            if (s + 1 < kSteps) {
                const int kk = (kc + kIK + bk) & (kBuckets - 1);
                va = ld8(fa + kk);
                vb = ld8(fb + kk);
            }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const bf16x8 av = *reinterpret_cast<const bf16x8*>(&xs[s & 1][16 * t + r][kq]);
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[t][c] = mfma(av, b[c], acc[t][c]);
        }
    }
    // epilogue 1: h1 = bf16(relu(acc + b1)) -> LDS
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int n = nw + 16 * c + r;
        const float bias = a.b1[n];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
#pragma unroll
            for (int q = 0; q < 4; ++q) h1s[16 * t + 4 * (lane >> 4) + q][n] = f2bf(fmaxf(acc[t][c][q] + bias, 0.f));
            acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    }
    __syncthreads();

    // ---- layer 2: h1 [128 x 512] . W2^T
#pragma unroll 2
    for (int ks = 0; ks < kHidden; ks += 32) {
        bf16x8 b[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) b[c] = ld8(a.w2 + static_cast<int64_t>(nw + 16 * c + r) * kHidden + ks + kq);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const bf16x8 av = *reinterpret_cast<const bf16x8*>(&h1s[16 * t + r][ks + kq]);
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[t][c] = mfma(av, b[c], acc[t][c]);
        }
    }
    // epilogue 2: h2 = bf16(relu(acc + b2)); partial logit over this wave's units
    float zp[8][4];
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) zp[t][q] = 0.f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int n = nw + 16 * c + r;
        const float bias = a.b2[n];
        const float w3 = bf2f(a.w3[n]);
#pragma unroll
        for (int t = 0; t < 8; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) zp[t][q] += bf2f(f2bf(fmaxf(acc[t][c][q] + bias, 0.f))) * w3;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float v = zp[t][q];
#pragma unroll
            for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 16);
            if (r == 0) zpart[wave][16 * t + 4 * (lane >> 4) + q] = v;
        }
    __syncthreads();
    if (tid < kIR) {
        const int64_t m = m0 + tid;
        float z = a.b3[0];
#pragma unroll
        for (int w = 0; w < kIW; ++w) z += zpart[w][tid];
        if (m < a.n) a.z[m] = z;
    }
}

// ---------------------------------------------------------------------------
// X transposed [2048][ld] for the layer-1 weight gradient (training only)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pair_xt(const uint16_t* feat, const int32_t* pairs, int n, int ld,
                                                 uint16_t* xt) {
    // block: 64 pairs x 64 features; transpose through LDS
    __shared__ uint16_t t[64][66];
    const int m0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int rr = ty; rr < 64; rr += 4) {
        const int m = m0 + rr;
        uint16_t v = 0;
        if (m < n) {
            const int k = k0 + tx;
            const int kk = k & (kBuckets - 1);
            const float x = bf2f(feat[static_cast<int64_t>(pairs[2 * m]) * kBuckets + kk]);
            const float y = bf2f(feat[static_cast<int64_t>(pairs[2 * m + 1]) * kBuckets + kk]);
            v = f2bf(k < kBuckets ? fabsf(x - y) : x * y);
        }
        t[rr][tx] = v;
    }
    __syncthreads();
    for (int kk = ty; kk < 64; kk += 4) xt[static_cast<int64_t>(k0 + kk) * ld + m0 + tx] = t[tx][kk];
}

// ---------------------------------------------------------------------------
// generic C = A . B^T on MFMA (A [M][K], B [N][K], bf16, K contiguous)
// tile 64 x 64 per block, 4 waves of 32 x 32
// ---------------------------------------------------------------------------
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_nt(GemmArgs g) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const int n0 = blockIdx.x * 64 + (wave & 1) * 32;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t* a0 = g.A + static_cast<int64_t>(m0 + r) * g.lda + kq;
    const uint16_t* a1 = a0 + static_cast<int64_t>(16) * g.lda;
    const uint16_t* b0 = g.B + static_cast<int64_t>(n0 + r) * g.ldb + kq;
    const uint16_t* b1 = b0 + static_cast<int64_t>(16) * g.ldb;
#pragma unroll 2
    for (int k = 0; k < g.K; k += 32) {
        const bf16x8 fa0 = ld8(a0 + k), fa1 = ld8(a1 + k);
        const bf16x8 fb0 = ld8(b0 + k), fb1 = ld8(b1 + k);
        acc[0][0] = mfma(fa0, fb0, acc[0][0]);
        acc[0][1] = mfma(fa0, fb1, acc[0][1]);
        acc[1][0] = mfma(fa1, fb0, acc[1][0]);
        acc[1][1] = mfma(fa1, fb1, acc[1][1]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + 16 * j + r;
            const int mb = m0 + 16 * i + 4 * (lane >> 4);
            if constexpr (EPI == kEpiF32) {
#pragma unroll
                for (int q = 0; q < 4; ++q) g.Cf[static_cast<int64_t>(mb + q) * g.ldc + n] = acc[i][j][q];
            } else {   // kEpiMaskT: out^T[n][m] = bf16(acc * (mask[m][n] > 0))
                uint16_t h[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool on = g.mask[static_cast<int64_t>(mb + q) * g.ldm + n] != 0;
                    h[q] = on ? f2bf(acc[i][j][q]) : static_cast<uint16_t>(0);
                }
                uint2 pk;
                pk.x = static_cast<uint32_t>(h[0]) | (static_cast<uint32_t>(h[1]) << 16);
                pk.y = static_cast<uint32_t>(h[2]) | (static_cast<uint32_t>(h[3]) << 16);
                *reinterpret_cast<uint2*>(g.Cb + static_cast<int64_t>(n) * g.ldc + mb) = pk;
            }
        }
}

// ---------------------------------------------------------------------------
// loss, dz, layer-3 backward
// ---------------------------------------------------------------------------
// one thread per pair: dz = (sigmoid(z) - y) / n; loss terms
__global__ void k_bce(const float* z, const uint8_t* y, int n, int mb, float* dz, float* loss) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= mb) return;
    if (m >= n) { dz[m] = 0.f; loss[m] = 0.f; return; }
    const float v = z[m], t = y[m] ? 1.f : 0.f;
    dz[m] = (1.f / (1.f + expf(-v)) - t) / static_cast<float>(n);
    loss[m] = fmaxf(v, 0.f) - v * t + log1pf(expf(-fabsf(v)));
}

// dH2 = bf16(dz * W3 * [h2 > 0]) in both layouts; the same pass leaves the
// layer-3 weight gradient's partial sums of its 64 rows,
// gpart[row tile][j] = sum over the tile's m of dz[m] h2[m][j]
__global__ __launch_bounds__(256) void k_dh2(const float* dz, const uint16_t* h2, const uint16_t* w3, int mb,
                                             uint16_t* dh2, uint16_t* dh2t, float* gpart) {
    __shared__ uint16_t t[64][66];
    __shared__ float part[4][64];
    const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    float acc = 0.f;
    for (int rr = ty; rr < 64; rr += 4) {
        const int m = m0 + rr, n = n0 + tx;
        const uint16_t hv = h2[static_cast<int64_t>(m) * kHidden + n];
        const float d = dz[m];
        const uint16_t v = hv ? f2bf(d * bf2f(w3[n])) : static_cast<uint16_t>(0);
        dh2[static_cast<int64_t>(m) * kHidden + n] = v;
        t[rr][tx] = v;
        acc += d * bf2f(hv);
    }
    part[ty][tx] = acc;
    __syncthreads();
    for (int nn = ty; nn < 64; nn += 4) dh2t[static_cast<int64_t>(n0 + nn) * mb + m0 + tx] = t[tx][nn];
    if (ty == 0)
        gpart[static_cast<int64_t>(blockIdx.x) * kHidden + n0 + tx] =
            part[0][tx] + part[1][tx] + part[2][tx] + part[3][tx];
}

// gW3[j] = sum of k_dh2's row-tile partials in tile order (the first
// kHidden / 256 blocks, a thread per column); gb3 = sum dz as a fixed tree
// over 256 threads (the last block)
__global__ __launch_bounds__(256) void k_gw3(const float* dz, const float* gpart, int mb, float* gw3, float* gb3) {
    __shared__ float part[256];
    const int tiles = mb / 64;
    if (blockIdx.x < kHidden / 256) {
        const int n = blockIdx.x * 256 + threadIdx.x;
        float s = 0.f;
        for (int k = 0; k < tiles; ++k) s += gpart[static_cast<int64_t>(k) * kHidden + n];
        gw3[n] = s;
        return;
    }
    float s = 0.f;
    for (int m = threadIdx.x; m < mb; m += 256) s += dz[m];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) gb3[0] = part[0];
}

// row sums of a bf16 [R][mb] matrix (bias gradients), block per row
__global__ __launch_bounds__(256) void k_rowsum(const uint16_t* x, int mb, float* out) {
    __shared__ float part[256];
    const int row = blockIdx.x;
    float s = 0.f;
    for (int m = threadIdx.x; m < mb; m += 256) s += bf2f(x[static_cast<int64_t>(row) * mb + m]);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[row] = part[0];
}

// ---------------------------------------------------------------------------
// Adam on the fp32 master, then the bf16 copies the network reads
// ---------------------------------------------------------------------------
__global__ void k_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_pack(const float* master, uint16_t* w1, uint16_t* w2, uint16_t* w2t, uint16_t* w3) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i < kW1) w1[i] = f2bf(master[kOffW1 + i]);
    if (i < kW2) {
        const uint16_t v = f2bf(master[kOffW2 + i]);
        w2[i] = v;
        const int64_t row = i / kHidden, col = i % kHidden;
        w2t[col * kHidden + row] = v;
    }
    if (i < kHidden) w3[i] = f2bf(master[kOffW3 + i]);
}

// ---------------------------------------------------------------------------
// training-run helpers: the batch's pair rows and labels gathered through the
// epoch's permutation, and the batch's mean loss written to the loss log
// ---------------------------------------------------------------------------
__global__ void k_gather_batch(const int32_t* perm, const int32_t* pairs, const uint8_t* labels, int n, int mb,
                               int32_t* bp, uint8_t* by) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= mb) return;
    if (m < n) {
        const int64_t src = perm[m];
        bp[2 * m] = pairs[2 * src];
        bp[2 * m + 1] = pairs[2 * src + 1];
        by[m] = labels[src];
    } else {   // padding rows of the last tile: a valid pair, masked out by k_bce
        bp[2 * m] = bp[0];
        bp[2 * m + 1] = bp[1];
        by[m] = 0;
    }
}

// fixed-order mean of loss[0..n): per-thread strided partial sums, then a tree
__global__ __launch_bounds__(256) void k_mean(const float* loss, int n, float* out) {
    __shared__ float part[256];
    float t = 0.f;
    for (int m = threadIdx.x; m < n; m += 256) t += loss[m];
    part[threadIdx.x] = t;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0] / static_cast<float>(n);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_kmer(const uint8_t* seqs, const int64_t* offsets, int32_t n_seqs, uint16_t* feat, uint32_t* err,
                       hipStream_t s) {
    if (n_seqs > 0) hipLaunchKernelGGL(k_kmer, dim3(n_seqs), dim3(256), 0, s, seqs, offsets, n_seqs, feat, err);
    return hipGetLastError();
}
hipError_t launch_fwd(const FwdArgs& a, int mb, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_fwd, dim3(mb / kRows), dim3(256), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_infer(const FwdArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_infer, dim3(static_cast<unsigned>((a.n + kIR - 1) / kIR)), dim3(512), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_pair_xt(const uint16_t* feat, const int32_t* pairs, int n, int mb, uint16_t* xt, hipStream_t s) {
    hipLaunchKernelGGL(k_pair_xt, dim3(mb / 64, kIn / 64), dim3(256), 0, s, feat, pairs, n, mb, xt);
    return hipGetLastError();
}
hipError_t launch_gemm(const GemmArgs& g, int epi, hipStream_t s) {
    const dim3 grid(g.N / 64, g.M / 64);
    if (epi == kEpiF32) hipLaunchKernelGGL(k_gemm_nt<kEpiF32>, grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL(k_gemm_nt<kEpiMaskT>, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}
hipError_t launch_backward_tail(const float* z, const uint8_t* y, int n, int mb, const uint16_t* h2,
                                const uint16_t* w3, float* dz, float* loss, uint16_t* dh2, uint16_t* dh2t,
                                float* gpart, float* gw3, float* gb3, hipStream_t s) {
    hipLaunchKernelGGL(k_bce, dim3((mb + 255) / 256), dim3(256), 0, s, z, y, n, mb, dz, loss);
    hipLaunchKernelGGL(k_dh2, dim3(mb / 64, kHidden / 64), dim3(256), 0, s, dz, h2, w3, mb, dh2, dh2t, gpart);
    hipLaunchKernelGGL(k_gw3, dim3(kHidden / 256 + 1), dim3(256), 0, s, dz, gpart, mb, gw3, gb3);
    return hipGetLastError();
}
hipError_t launch_rowsum(const uint16_t* x, int rows, int mb, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_rowsum, dim3(rows), dim3(256), 0, s, x, mb, out);
    return hipGetLastError();
}
hipError_t launch_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s) {
    const float c1 = 1.f - powf(b1, static_cast<float>(step));
    const float c2 = 1.f - powf(b2, static_cast<float>(step));
    hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, w, g, m, v, n, lr, b1,
                       b2, eps, c1, c2);
    return hipGetLastError();
}
hipError_t launch_gather_batch(const int32_t* perm, const int32_t* pairs, const uint8_t* labels, int n, int mb,
                               int32_t* bp, uint8_t* by, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_batch, dim3((mb + 255) / 256), dim3(256), 0, s, perm, pairs, labels, n, mb, bp, by);
    return hipGetLastError();
}
hipError_t launch_mean(const float* loss, int n, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_mean, dim3(1), dim3(256), 0, s, loss, n, out);
    return hipGetLastError();
}
hipError_t launch_pack(const float* master, uint16_t* w1, uint16_t* w2, uint16_t* w2t, uint16_t* w3, hipStream_t s) {
    hipLaunchKernelGGL(k_pack, dim3(static_cast<unsigned>((kW1 + 255) / 256)), dim3(256), 0, s, master, w1, w2, w2t,
                       w3);
    return hipGetLastError();
}

}  // namespace cms
