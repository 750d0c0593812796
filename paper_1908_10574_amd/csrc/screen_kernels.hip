// screen_kernels.hip -- learned pair screen for gfx950: hashed 3-mer features,
// a 2048-512-512-1 MLP on bf16 MFMA with fp32 accumulation, its backward pass
// and Adam.  The screen sits in front of the exact alignment (it decides which
// candidate pairs are aligned at all); it never changes a score.
//
// Layouts (row-major, bf16 stored as uint16 bit patterns):
//   feat  [n_seqs][1024]   count/8 of hashed 3-mers
//   X     [M][2048]        [|fa - fb|, fa * fb] per pair (inference: built on the fly)
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
// inference forward: 128 pairs per block, 8 waves, each wave owns 64 hidden
// units for all 128 rows, so every weight fragment loaded from L2 feeds 8
// row tiles.  Same rounding points as k_mlp_fwd (X, h1, h2 rounded to bf16;
// fp32 accumulation), no training outputs.
// Layer 1 runs in K steps of 64: the pair input of a step is built (16
// columns per thread, fp32 arithmetic, one hardware round-to-nearest-even
// conversion per two values) into one of two LDS tiles while the other tile
// feeds the MFMAs, with one barrier per step; each wave's W1 fragments are
// loaded one 32-wide sub-step ahead of their MFMAs.  The two pair-input tiles
// share their LDS with the layer-1 output (used only after the last step).
// ---------------------------------------------------------------------------
constexpr int kIR = 128;           // pairs per block
constexpr int kIW = 8;             // waves per block
constexpr int kIK = 64;            // layer-1 K step
constexpr int kXS = kIK + 8;       // pair-input tile row stride (elements)
constexpr int kHS = kHidden + 8;   // layer-1 output row stride (elements)
static_assert(2 * kIR * kXS <= kIR * kHS, "pair-input tiles must fit in the layer-1 output buffer");

typedef __attribute__((__vector_size__(2 * sizeof(float)))) float f32x2v;
typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2v;

// two fp32 values rounded to bf16 (nearest even), packed low = a, high = b
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    const f32x2v v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2v));
}

__global__ __launch_bounds__(512) void k_mlp_infer(FwdArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t lds[kIR * kHS];
    __shared__ float zpart[kIW][kIR];
    __shared__ int pa[kIR], pb[kIR];
    uint16_t* const h1s = lds;
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
    const int br = tid >> 2, bk = (tid & 3) * 16;    // builder: row, 16 columns of the step
    const uint16_t* fa = a.feat + static_cast<int64_t>(pa[br]) * kBuckets;
    const uint16_t* fb = a.feat + static_cast<int64_t>(pb[br]) * kBuckets;
    bf16x8 va0 = ld8(fa + bk), va1 = ld8(fa + bk + 8), vb0 = ld8(fb + bk), vb1 = ld8(fb + bk + 8);
    const uint16_t* wrow[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) wrow[c] = a.w1 + static_cast<int64_t>(nw + 16 * c + r) * kIn + kq;
    bf16x8 bcur[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) bcur[c] = ld8(wrow[c]);
    constexpr int kSteps = kIn / kIK;
    for (int s = 0; s < kSteps; ++s) {
        const int kc = s * kIK;
        uint16_t* xs = lds + (s & 1) * (kIR * kXS);
        {
            const bool diff = kc < kBuckets;
            uint32_t o[8];
#pragma unroll
            for (int j = 0; j < 8; j += 2) {
                const float x0 = static_cast<float>(va0[j]), y0 = static_cast<float>(vb0[j]);
                const float x1 = static_cast<float>(va0[j + 1]), y1 = static_cast<float>(vb0[j + 1]);
                o[j / 2] = diff ? pack_bf16(fabsf(x0 - y0), fabsf(x1 - y1)) : pack_bf16(x0 * y0, x1 * y1);
                const float x2 = static_cast<float>(va1[j]), y2 = static_cast<float>(vb1[j]);
                const float x3 = static_cast<float>(va1[j + 1]), y3 = static_cast<float>(vb1[j + 1]);
                o[4 + j / 2] = diff ? pack_bf16(fabsf(x2 - y2), fabsf(x3 - y3)) : pack_bf16(x2 * y2, x3 * y3);
            }
            uint4* dst = reinterpret_cast<uint4*>(xs + br * kXS + bk);
            dst[0] = make_uint4(o[0], o[1], o[2], o[3]);
            dst[1] = make_uint4(o[4], o[5], o[6], o[7]);
            if (s + 1 < kSteps) {
                const int kk = (kc + kIK + bk) & (kBuckets - 1);
                va0 = ld8(fa + kk);
                va1 = ld8(fa + kk + 8);
                vb0 = ld8(fb + kk);
                vb1 = ld8(fb + kk + 8);
            }
        }
        __syncthreads();
        // sub-step 0 (columns kc..kc+31): the next sub-step's fragments load meanwhile
        bf16x8 bnx[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) bnx[c] = ld8(wrow[c] + kc + 32);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const bf16x8 av = *reinterpret_cast<const bf16x8*>(xs + (16 * t + r) * kXS + kq);
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[t][c] = mfma(av, bcur[c], acc[t][c]);
        }
        // sub-step 1 (columns kc+32..kc+63): the next step's first fragments load meanwhile
        if (s + 1 < kSteps) {
#pragma unroll
            for (int c = 0; c < 4; ++c) bcur[c] = ld8(wrow[c] + kc + kIK);
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const bf16x8 av = *reinterpret_cast<const bf16x8*>(xs + (16 * t + r) * kXS + 32 + kq);
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[t][c] = mfma(av, bnx[c], acc[t][c]);
        }
    }
    __syncthreads();   // every wave is done with the pair-input tiles, which h1s overwrites
    // epilogue 1: h1 = bf16(relu(acc + b1)) -> LDS
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int n = nw + 16 * c + r;
        const float bias = a.b1[n];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                h1s[(16 * t + 4 * (lane >> 4) + q) * kHS + n] = f2bf(fmaxf(acc[t][c][q] + bias, 0.f));
            acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    }
    __syncthreads();

    // ---- layer 2: h1 [128 x 512] . W2^T (fragments loaded one step ahead)
    const uint16_t* w2row[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) w2row[c] = a.w2 + static_cast<int64_t>(nw + 16 * c + r) * kHidden + kq;
#pragma unroll
    for (int c = 0; c < 4; ++c) bcur[c] = ld8(w2row[c]);
#pragma unroll 2
    for (int ks = 0; ks < kHidden; ks += 32) {
        bf16x8 bb[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) bb[c] = bcur[c];
        if (ks + 32 < kHidden) {
#pragma unroll
            for (int c = 0; c < 4; ++c) bcur[c] = ld8(w2row[c] + ks + 32);
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const bf16x8 av = *reinterpret_cast<const bf16x8*>(h1s + (16 * t + r) * kHS + ks + kq);
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[t][c] = mfma(av, bb[c], acc[t][c]);
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
// loss, dz, layer-3 backward
// ---------------------------------------------------------------------------
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

// gW3[j] = sum of k_dh2's row-tile partials (the first kHidden / 64 blocks:
// 64 columns each, four threads per column summing every fourth tile, the
// four sums added in order); gb3 = sum dz as a fixed tree over 256 threads
// (the last block)
__global__ __launch_bounds__(256) void k_gw3(const float* dz, const float* gpart, int mb, float* gw3, float* gb3) {
    __shared__ float part[256];
    const int tiles = mb / 64;
    if (blockIdx.x < kHidden / 64) {
        const int n = blockIdx.x * 64 + (threadIdx.x & 63), p = threadIdx.x >> 6;
        float s = 0.f;
#pragma unroll 8
        for (int k = p; k < tiles; k += 4) s += gpart[static_cast<int64_t>(k) * kHidden + n];
        part[threadIdx.x] = s;
        __syncthreads();
        if (p == 0) gw3[n] = ((part[threadIdx.x] + part[threadIdx.x + 64]) + part[threadIdx.x + 128]) + part[threadIdx.x + 192];
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
// bf16 copies of weights set from the host
// ---------------------------------------------------------------------------
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
// training step kernels
//
// X and X^T once per batch (k_build_x), then every product of the forward and
// backward pass is one tiled MFMA kernel, C = A . B^T with K contiguous in
// both operands (k_gemm2): 256 threads, tiles of BM x 128 (4 waves of
// BM/2 x 64), K steps of 128 staged through two LDS buffers (the next step's
// tiles are loaded into registers during the current step's MFMAs; one
// barrier per step).  The weight gradients (K = batch) are split over K into
// fp32 partials, added in split order by k_reduce (deterministic).
// ---------------------------------------------------------------------------

// X [mb][2048] and X^T [2048][mb]: a 64-row x 64-feature tile per block
__global__ __launch_bounds__(256) void k_build_x(const uint16_t* feat, const int32_t* pairs, int n, int mb,
                                                 uint16_t* x, uint16_t* xt) {
    __shared__ uint16_t t[64][66];
    const int m0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int k = k0 + tx;
    const int kk = k & (kBuckets - 1);
    for (int rr = ty; rr < 64; rr += 4) {
        const int m = m0 + rr;
        uint16_t v = 0;
        if (m < n) {
            const float fa = bf2f(feat[static_cast<int64_t>(pairs[2 * m]) * kBuckets + kk]);
            const float fb = bf2f(feat[static_cast<int64_t>(pairs[2 * m + 1]) * kBuckets + kk]);
            v = f2bf(k < kBuckets ? fabsf(fa - fb) : fa * fb);
        }
        x[static_cast<int64_t>(m) * kIn + k] = v;
        t[rr][tx] = v;
    }
    __syncthreads();
    for (int c = ty; c < 64; c += 4) xt[static_cast<int64_t>(k0 + c) * mb + m0 + tx] = t[tx][c];
}

// One K step of k_gemm2 on LDS buffer `buf` (= s % 2).  On entry (ca, cb)
// are receiving step s+1 and (na, nb) are free.  The step loads step s+2
// into (na, nb), runs its MFMAs over the buffer, stores (ca, cb) into the
// other buffer and waits at the barrier.  Nothing in it is conditional: the
// last two steps re-load the final step (an L2 hit) and the last store goes
// to the idle buffer, because a load whose only use sits behind a branch is
// sunk to that use, which serialises it.
template <int BM, int TI, int NA, int LS>
__device__ __forceinline__ void gemm2_step(int s, int steps, int buf, const uint16_t* ga, const uint16_t* gb, int ar,
                                           int ac, int lr, int lc, int wm, int wn, int r, int kq,
                                           uint16_t (*As)[BM * LS], uint16_t (*Bs)[128 * LS], bf16x8 (&ca)[NA],
                                           bf16x8 (&cb)[8], bf16x8 (&na)[NA], bf16x8 (&nb)[8],
                                           f32x4 (&acc)[TI][4]) {
    constexpr int BK = 128;
    const int k = min(s + 2, steps - 1) * BK;
#pragma unroll
    for (int q = 0; q < NA; ++q) na[q] = ld8(ga + k + 8 * q);
#pragma unroll
    for (int q = 0; q < 8; ++q) nb[q] = ld8(gb + k + 8 * q);
    __builtin_amdgcn_sched_barrier(0);   // the scheduler would sink the loads below the MFMAs
    const uint16_t* as = As[buf];
    const uint16_t* bs = Bs[buf];
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
        bf16x8 af[TI], bfr[4];
#pragma unroll
        for (int i = 0; i < TI; ++i)
            af[i] = *reinterpret_cast<const bf16x8*>(as + (wm * (BM / 2) + 16 * i + r) * LS + kk + kq);
#pragma unroll
        for (int j = 0; j < 4; ++j) bfr[j] = *reinterpret_cast<const bf16x8*>(bs + (wn * 64 + 16 * j + r) * LS + kk + kq);
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = mfma(af[i], bfr[j], acc[i][j]);
    }
    uint16_t* an = As[buf ^ 1];
    uint16_t* bn = Bs[buf ^ 1];
#pragma unroll
    for (int q = 0; q < NA; ++q) *reinterpret_cast<bf16x8*>(an + ar * LS + ac + 8 * q) = ca[q];
#pragma unroll
    for (int q = 0; q < 8; ++q) *reinterpret_cast<bf16x8*>(bn + lr * LS + lc + 8 * q) = cb[q];
    __syncthreads();
}

template <int BM, int EPI>
__global__ __launch_bounds__(256) void k_gemm2(Gemm2Args g) {
    // K steps of 128 with two steps of operand loads in flight (96-128 KB per
    // block): with one block per compute unit, that is what hides the L2/HBM latency
    constexpr int BN = 128, BK = 128, LS = BK + 8;     // LDS row stride: 136 elements (272 bytes)
    constexpr int TI = BM / 32;                         // 16-row tiles per wave (a wave holds BM/2 rows)
    constexpr int NA = BM / 16;                         // 16-byte A loads per thread and step
    __shared__ __attribute__((aligned(16))) uint16_t As[2][BM * LS];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN * LS];
    __shared__ float zl[2][BM];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    // XCD-aware tile order: blocks are dealt round-robin to the 8 XCDs in
    // launch order, so block b runs on XCD b % 8.  Each XCD takes a contiguous
    // range of tiles (N fastest), so the column tiles that share an A row
    // block run on one XCD and read it through that XCD's L2 once.
    int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
    {
        const int gx = gridDim.x, gy = gridDim.y;
        const int total = gx * gy * gridDim.z;
        if ((total & 7) == 0) {
            const int lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
            const int q = (lin & 7) * (total >> 3) + (lin >> 3);
            bx = q % gx;
            by = (q / gx) % gy;
            bz = q / (gx * gy);
        }
    }
    const int m0 = by * BM, n0 = bx * BN;
    const int64_t kbeg = static_cast<int64_t>(bz) * g.kper;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    // loaders: B row tid / 2, 64 columns at (tid & 1) * 64 (8 x 16 B); A likewise
    // when BM = 128, and row tid / 4, 32 columns at (tid & 3) * 32 (4 x 16 B) when BM = 64
    const int lr = tid >> 1, lc = (tid & 1) * 64;
    const int ar = BM == 128 ? lr : tid >> 2, ac = BM == 128 ? lc : (tid & 3) * 32;
    const uint16_t* ga = g.A + static_cast<int64_t>(m0 + ar) * g.lda + kbeg + ac;
    const uint16_t* gb = g.B + static_cast<int64_t>(n0 + lr) * g.ldb + kbeg + lc;
    // Two steps of operand loads in flight: at the top of step s, LDS buffer
    // s%2 holds step s and one register set is receiving step s+1 (see
    // gemm2_step).  The loop runs steps in pairs with the two register sets
    // swapped, so no register is copied (a copy would wait for its load); an
    // odd last step runs after it.  The registers are native vectors (an
    // array of HIP's vector class stays in memory).
    bf16x8 ra0[NA], rb0[8], ra1[NA], rb1[8];
    const int steps = g.kper / BK;
#pragma unroll
    for (int q = 0; q < NA; ++q) ra0[q] = ld8(ga + 8 * q);
#pragma unroll
    for (int q = 0; q < 8; ++q) rb0[q] = ld8(gb + 8 * q);
#pragma unroll
    for (int q = 0; q < NA; ++q) *reinterpret_cast<bf16x8*>(&As[0][ar * LS + ac + 8 * q]) = ra0[q];
#pragma unroll
    for (int q = 0; q < 8; ++q) *reinterpret_cast<bf16x8*>(&Bs[0][lr * LS + lc + 8 * q]) = rb0[q];
    {
        const int k1 = min(1, steps - 1) * BK;
#pragma unroll
        for (int q = 0; q < NA; ++q) ra1[q] = ld8(ga + k1 + 8 * q);
#pragma unroll
        for (int q = 0; q < 8; ++q) rb1[q] = ld8(gb + k1 + 8 * q);
    }
    f32x4 acc[TI][4];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    __syncthreads();
    int s = 0;
    for (; s + 1 < steps; s += 2) {
        gemm2_step<BM, TI, NA, LS>(s, steps, 0, ga, gb, ar, ac, lr, lc, wm, wn, r, kq, As, Bs, ra1, rb1, ra0, rb0, acc);
        gemm2_step<BM, TI, NA, LS>(s + 1, steps, 1, ga, gb, ar, ac, lr, lc, wm, wn, r, kq, As, Bs, ra0, rb0, ra1, rb1,
                                   acc);
    }
    if (s < steps)
        gemm2_step<BM, TI, NA, LS>(s, steps, 0, ga, gb, ar, ac, lr, lc, wm, wn, r, kq, As, Bs, ra1, rb1, ra0, rb0, acc);
    // epilogue: acc[i][j][q] is C[m0 + wm*BM/2 + 16i + 4(lane/16) + q][n0 + wn*64 + 16j + r]
    const int mrow = m0 + wm * (BM / 2) + 4 * (lane >> 4);
    if constexpr (EPI == kEpi2Partial) {
        float* out = g.Cp + static_cast<int64_t>(bz) * g.M * g.N;
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int n = n0 + wn * 64 + 16 * j + r;
#pragma unroll
                for (int q = 0; q < 4; ++q) out[static_cast<int64_t>(mrow + 16 * i + q) * g.N + n] = acc[i][j][q];
            }
    } else if constexpr (EPI == kEpi2MaskT) {
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int n = n0 + wn * 64 + 16 * j + r;
                const int m = mrow + 16 * i;
                uint16_t h[4];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    h[q] = g.mask[static_cast<int64_t>(m + q) * g.ldm + n] ? f2bf(acc[i][j][q]) : static_cast<uint16_t>(0);
                *reinterpret_cast<uint2*>(g.Ct + static_cast<int64_t>(n) * g.ldct + m) =
                    make_uint2(static_cast<uint32_t>(h[0]) | (static_cast<uint32_t>(h[1]) << 16),
                               static_cast<uint32_t>(h[2]) | (static_cast<uint32_t>(h[3]) << 16));
            }
    } else {   // kEpi2BiasRelu, kEpi2Logit: h = bf16(relu(acc + bias)) row-major (+ transposed / logit partials)
        float zp[TI][4];
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) zp[i][q] = 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + wn * 64 + 16 * j + r;
            const float bias = g.bias[n];
            const float w3 = EPI == kEpi2Logit ? bf2f(g.w3[n]) : 0.f;
#pragma unroll
            for (int i = 0; i < TI; ++i) {
                const int m = mrow + 16 * i;
                uint16_t h[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    h[q] = f2bf(fmaxf(acc[i][j][q] + bias, 0.f));
                    g.Cb[static_cast<int64_t>(m + q) * g.ldcb + n] = h[q];
                    if constexpr (EPI == kEpi2Logit) zp[i][q] += bf2f(h[q]) * w3;
                }
                if constexpr (EPI == kEpi2BiasRelu)
                    *reinterpret_cast<uint2*>(g.Ct + static_cast<int64_t>(n) * g.ldct + m) =
                        make_uint2(static_cast<uint32_t>(h[0]) | (static_cast<uint32_t>(h[1]) << 16),
                                   static_cast<uint32_t>(h[2]) | (static_cast<uint32_t>(h[3]) << 16));
            }
        }
        if constexpr (EPI == kEpi2Logit) {
            // the wave's 64 columns: across the 16 lanes sharing rows, then the two column waves
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float v = zp[i][q];
#pragma unroll
                    for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 16);
                    if (r == 0) zl[wn][wm * (BM / 2) + 16 * i + 4 * (lane >> 4) + q] = v;
                }
            __syncthreads();
            if (tid < BM)
                g.zpart[static_cast<int64_t>(m0 + tid) * (g.N / BN) + bx] = zl[0][tid] + zl[1][tid];
        }
    }
}

// out[i] = sum over s of part[s][i], in split order
__global__ void k_reduce(const float* part, int splits, int64_t count, float* out) {
    const int64_t i = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) * 4;
    if (i >= count) return;
    float4 a = *reinterpret_cast<const float4*>(part + i);
    for (int s = 1; s < splits; ++s) {
        const float4 b = *reinterpret_cast<const float4*>(part + s * count + i);
        a.x += b.x; a.y += b.y; a.z += b.z; a.w += b.w;
    }
    *reinterpret_cast<float4*>(out + i) = a;
}

// logits from the layer-2 partials (column tiles in order, then b3), then
// dz = (sigmoid(z) - y) / n and the loss terms
__global__ void k_logit_bce(const float* zpart, int tiles, const float* b3, const uint8_t* y, int n, int mb, float* z,
                            float* dz, float* loss) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= mb) return;
    if (m >= n) { dz[m] = 0.f; loss[m] = 0.f; return; }
    float v = 0.f;
    for (int t = 0; t < tiles; ++t) v += zpart[static_cast<int64_t>(m) * tiles + t];
    v += b3[0];
    z[m] = v;
    const float yy = y[m] ? 1.f : 0.f;
    dz[m] = (1.f / (1.f + expf(-v)) - yy) / static_cast<float>(n);
    loss[m] = fmaxf(v, 0.f) - v * yy + log1pf(expf(-fabsf(v)));
}

// Adam on the fp32 master, and in the same pass the bf16 copies the network reads
__global__ void k_adam_pack(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2, uint16_t* w1, uint16_t* w2, uint16_t* w2t, uint16_t* w3) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    const uint16_t h = f2bf(wi);
    if (i < kOffB1) {
        w1[i - kOffW1] = h;
    } else if (i >= kOffW2 && i < kOffB2) {
        const int64_t e = i - kOffW2;
        w2[e] = h;
        w2t[(e % kHidden) * kHidden + e / kHidden] = h;
    } else if (i >= kOffW3 && i < kOffB3) {
        w3[i - kOffW3] = h;
    }
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
hipError_t launch_infer(const FwdArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_infer, dim3(static_cast<unsigned>((a.n + kIR - 1) / kIR)), dim3(512), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_backward_tail(const float* dz, int n, int mb, const uint16_t* h2, const uint16_t* w3, uint16_t* dh2,
                                uint16_t* dh2t, float* gpart, float* gw3, float* gb3, hipStream_t s) {
    (void)n;
    hipLaunchKernelGGL(k_dh2, dim3(mb / 64, kHidden / 64), dim3(256), 0, s, dz, h2, w3, mb, dh2, dh2t, gpart);
    hipLaunchKernelGGL(k_gw3, dim3(kHidden / 64 + 1), dim3(256), 0, s, dz, gpart, mb, gw3, gb3);
    return hipGetLastError();
}
hipError_t launch_rowsum(const uint16_t* x, int rows, int mb, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_rowsum, dim3(rows), dim3(256), 0, s, x, mb, out);
    return hipGetLastError();
}
hipError_t launch_build_x(const uint16_t* feat, const int32_t* pairs, int n, int mb, uint16_t* x, uint16_t* xt,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_build_x, dim3(mb / 64, kIn / 64), dim3(256), 0, s, feat, pairs, n, mb, x, xt);
    return hipGetLastError();
}
hipError_t launch_gemm2(const Gemm2Args& g, int bm, int epi, int splits, hipStream_t s) {
    const dim3 grid(g.N / 128, g.M / bm, splits);
    if (bm == 64) {
        switch (epi) {
            case kEpi2Partial: hipLaunchKernelGGL((k_gemm2<64, kEpi2Partial>), grid, dim3(256), 0, s, g); break;
            case kEpi2BiasRelu: hipLaunchKernelGGL((k_gemm2<64, kEpi2BiasRelu>), grid, dim3(256), 0, s, g); break;
            case kEpi2MaskT: hipLaunchKernelGGL((k_gemm2<64, kEpi2MaskT>), grid, dim3(256), 0, s, g); break;
            default: hipLaunchKernelGGL((k_gemm2<64, kEpi2Logit>), grid, dim3(256), 0, s, g); break;
        }
    } else {
        hipLaunchKernelGGL((k_gemm2<128, kEpi2Partial>), grid, dim3(256), 0, s, g);
    }
    return hipGetLastError();
}
hipError_t launch_reduce(const float* part, int splits, int64_t count, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(static_cast<unsigned>((count / 4 + 255) / 256)), dim3(256), 0, s, part, splits,
                       count, out);
    return hipGetLastError();
}
hipError_t launch_logit_bce(const float* zpart, int tiles, const float* b3, const uint8_t* y, int n, int mb, float* z,
                            float* dz, float* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_logit_bce, dim3((mb + 255) / 256), dim3(256), 0, s, zpart, tiles, b3, y, n, mb, z, dz, loss);
    return hipGetLastError();
}
hipError_t launch_adam_pack(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                            float eps, int step, uint16_t* w1, uint16_t* w2, uint16_t* w2t, uint16_t* w3,
                            hipStream_t s) {
    const float c1 = 1.f - powf(b1, static_cast<float>(step));
    const float c2 = 1.f - powf(b2, static_cast<float>(step));
    hipLaunchKernelGGL(k_adam_pack, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, w, g, m, v, n, lr,
                       b1, b2, eps, c1, c2, w1, w2, w2t, w3);
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
