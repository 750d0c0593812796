// sw_kernels.hip -- batched Smith-Waterman (Gotoh affine gaps) for gfx950.
//
// Computes, for every pair of a batch, the local-alignment score of Section 4
// of the ClusterMerge paper (the similarity function f), optionally the end
// cell, and in a second pass the start cell used by the coverage test of the
// protein transitivity function.
//
// Recurrence (E and F kept clamped at zero, which is exact because the gap
// extension is never positive: max(E,0) obeys the same recurrence with a 0
// term, and H already takes a max with 0):
//     E'[i][j+1] = max(E'[i][j] + ge, H[i][j] + go, 0)
//     F'[i+1][j] = max(F'[i][j] + ge, H[i][j] + go, 0)
//     H[i][j]    = max(H[i-1][j-1] + M[a_i][b_j], E'[i][j], F'[i][j])
// which is 8 int32 VALU operations per cell (add, max3, max, add, add, max3,
// add, max3).
//
// Work decomposition (MI355X, wave64):
//   * one 16-lane DPP row ("group") aligns one pair; a wavefront carries four
//     pairs of the same shape class;
//   * lane l of a group owns R consecutive query rows of a 16*R-row strip and
//     sweeps the subject columns with a one-column skew per lane (lane l works
//     on column t-l at step t); the H and F' values leaving a lane's bottom row
//     reach the lane below through a DPP row_shr:1 move, so no LDS round trip
//     is needed for the wavefront carries;
//   * the query profile of the strip (score of each row against each of the
//     20 residues plus a sentinel) lives in LDS as int8, one 4/8/16-byte read
//     per lane per column; the byte operands feed the adds through SDWA;
//   * subject residues enter lane 0 from a 16-column register chunk rotated by
//     DPP row_shl:1; queries longer than one strip hand the bottom row (H, F')
//     to the next strip through a per-group global boundary row, staged with
//     the same 16-column rotation;
//   * pairs are sorted by (rows per lane, strips, columns) by the plan pass and
//     handed out four at a time from an atomic ticket to a persistent grid.
//
// Cells outside the pair (padding rows below the query, columns before the
// skew reaches a lane or after the subject ends) use a sentinel score of -128.
// Their values are either 0 (before the pair starts) or strictly below the best
// real score (they derive from real cells through gap penalties or a negative
// sentinel substitution), so they never change a score, an end cell or a start
// cell.
#include "cm_internal.h"

#include <type_traits>

namespace cmk {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int dpp_shr1(int old_v, int src) {
    // lane k <- lane k-1 of the same 16-lane row; lane 0 of the row keeps old_v
    return __builtin_amdgcn_update_dpp(old_v, src, 0x111, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_shl1(int old_v, int src) {
    // lane k <- lane k+1 of the same 16-lane row; lane 15 of the row keeps old_v
    return __builtin_amdgcn_update_dpp(old_v, src, 0x101, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_shr1_zero(int src) {
    // lane k <- lane k-1 of the same 16-lane row; lane 0 of the row reads 0
    return __builtin_amdgcn_mov_dpp(src, 0x111, 0xf, 0xf, true);
}
__device__ __forceinline__ int dpp_shl1_any(int src) {
    // lane k <- lane k+1 of the same 16-lane row; lane 15 of the row reads 0
    return __builtin_amdgcn_mov_dpp(src, 0x101, 0xf, 0xf, true);
}
// The same moves over a lane group of G: one 16-lane row (row_shr / row_shl)
// or the whole 64-lane wavefront (wave_shr / wave_shl).
template <int G>
__device__ __forceinline__ int dpp_shr1g(int old_v, int src) {
    if constexpr (G == 16) return dpp_shr1(old_v, src);
    else return __builtin_amdgcn_update_dpp(old_v, src, 0x138, 0xf, 0xf, false);
}
template <int G>
__device__ __forceinline__ int dpp_shl1g(int old_v, int src) {
    if constexpr (G == 16) return dpp_shl1(old_v, src);
    else return __builtin_amdgcn_update_dpp(old_v, src, 0x130, 0xf, 0xf, false);
}
template <int G>
__device__ __forceinline__ int dpp_shr1_zerog(int src) {
    if constexpr (G == 16) return dpp_shr1_zero(src);
    else return __builtin_amdgcn_mov_dpp(src, 0x138, 0xf, 0xf, true);
}
template <int G>
__device__ __forceinline__ int dpp_shl1_anyg(int src) {
    if constexpr (G == 16) return dpp_shl1_any(src);
    else return __builtin_amdgcn_mov_dpp(src, 0x130, 0xf, 0xf, true);
}
__device__ __forceinline__ int max3i(int a, int b, int c) { return max(max(a, b), c); }

template <int W>
struct ProfWords { uint32_t w[W]; };

template <int W, int G = kGroup>
__device__ __forceinline__ ProfWords<W> load_prof(const uint8_t* prof, int c, int gl) {
    const uint8_t* p = prof + (c * G + gl) * (4 * W);
    ProfWords<W> r;
    if constexpr (W == 4) {
        uint4 v = *reinterpret_cast<const uint4*>(p);
        r.w[0] = v.x; r.w[1] = v.y; r.w[2] = v.z; r.w[3] = v.w;
    } else if constexpr (W == 2) {
        uint2 v = *reinterpret_cast<const uint2*>(p);
        r.w[0] = v.x; r.w[1] = v.y;
    } else {
        r.w[0] = *reinterpret_cast<const uint32_t*>(p);
    }
    return r;
}

__device__ __forceinline__ int sbyte(uint32_t w, int k) {
    return static_cast<int>(static_cast<int8_t>(static_cast<uint8_t>(w >> (8 * k))));
}

__device__ __forceinline__ int wave_max4(int v) {
    // max of the values held by lanes 0, 16, 32, 48
    int a = __builtin_amdgcn_readlane(v, 0);
    int b = __builtin_amdgcn_readlane(v, 16);
    int c = __builtin_amdgcn_readlane(v, 32);
    int d = __builtin_amdgcn_readlane(v, 48);
    return max(max(a, b), max(c, d));
}

// rows per lane for a query of m rows under a per-lane limit rmax: fewest
// strips, then fewest rows per lane (rounded up to an even count for the int32
// kernel, which is instantiated for even R; the packed kernel takes any R)
__device__ __forceinline__ void shape_for(int m, int rmax, bool even, int& R, int& strips) {
    strips = (m + kGroup * rmax - 1) / (kGroup * rmax);
    R = (m + kGroup * strips - 1) / (kGroup * strips);
    if (even) R += R & 1;
    if (R > rmax) R = rmax;
}

// ---------------------------------------------------------------------------
// plan: validate, write trivial results, build sort keys
// ---------------------------------------------------------------------------
__global__ void k_zero_counters(Counters* c) {
    if (threadIdx.x == 0) {
        c->n_work = 0; c->ticket = 0; c->n_over = 0; c->ticket_over = 0;
        c->n_sel[0] = 0; c->n_sel[1] = 0; c->ticket_b = 0;
    }
}

__global__ void k_plan(SwArgs a, int pass, uint32_t* keys, int32_t* vals) {
    const int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (p >= a.n_pairs) return;
    const Pass P = static_cast<Pass>(pass);
    uint32_t key = kSkipKey;
    if (a.n_live && p >= *a.n_live) {      // padding row of a fixed-capacity launch
        keys[p] = key;
        vals[p] = static_cast<int32_t>(p);
        return;
    }
    const int x = a.pairs[2 * p], y = a.pairs[2 * p + 1];
    int m = 0, n = 0;
    bool trivial = true;
    bool keep_score = false;   // filtered score+end pass: the known score stays
    if (x < 0 || x >= a.n_seqs || y < 0 || y >= a.n_seqs) {
        atomicOr(a.err, kErrIndex);
    } else {
        const int64_t lx = a.offsets[x + 1] - a.offsets[x];
        const int64_t ly = a.offsets[y + 1] - a.offsets[y];
        if (lx > kMaxLen || ly > kMaxLen || lx < 0 || ly < 0) {
            atomicOr(a.err, kErrLength);
        } else if (P == Pass::Span) {
            const int s = a.scores[p];
            if (s > a.min_score) {
                const int ea = a.end_a[p], eb = a.end_b[p];
                if (ea < 0 || ea >= lx || eb < 0 || eb >= ly) {
                    atomicOr(a.err, kErrCell);
                } else {
                    m = ea + 1; n = eb + 1; trivial = false;
                }
            }
        } else if (P == Pass::ScoreEnd && a.end_filter && a.scores[p] <= a.min_score) {
            keep_score = true;
        } else {
            m = static_cast<int>(lx); n = static_cast<int>(ly);
            trivial = (m == 0 || n == 0);
        }
    }
    if (trivial) {
        if (P == Pass::Span) {
            a.start_a[p] = -1; a.start_b[p] = -1;
        } else {
            if (!keep_score) a.scores[p] = 0;
            if (a.end_a) { a.end_a[p] = -1; a.end_b[p] = -1; }
        }
    } else {
        int R, strips;
        shape_for(m, a.rmax, !a.packed, R, strips);
        key = (static_cast<uint32_t>(kRMax - R) << 24) |
              (static_cast<uint32_t>(255 - min(strips, 255)) << 16) |
              static_cast<uint32_t>(65535 - n);
        atomicAdd(&a.ctr->n_work, 1);
    }
    keys[p] = key;
    vals[p] = static_cast<int32_t>(p);
}

// ---------------------------------------------------------------------------
// one wavefront item: 64 / G pairs of the same rows-per-lane class, each on a
// group of G lanes (16: four pairs, one DPP row each; 64: one pair on the
// whole wavefront, for launches with few pairs, whose time is the serial
// latency of their longest pair: G lanes hold G * R rows of a strip, so a pair
// of m rows takes m / (G * R) strips of n + G - 1 steps)
// ---------------------------------------------------------------------------
template <int R, Pass P, int RMAXT, int G = kGroup>
__device__ __forceinline__ void run_item(const SwArgs& a, const int32_t* __restrict__ order, int item,
                                         int n_work, const int8_t* __restrict__ s_mat,
                                         uint8_t* __restrict__ s_prof) {
    constexpr int RP = R <= 4 ? 4 : (R <= 8 ? 8 : 16);
    constexpr int W = RP / 4;
    constexpr int kRows = G * R;
    constexpr bool kEnd = (P != Pass::Score);
    const int lane = threadIdx.x;
    const int g = lane / G;
    const int gl = lane % G;
    const int go = a.go, ge = a.ge;
    // the clamp value is a kernel argument (always 0) so the compiler keeps the
    // signed three-input max instead of splitting it on a known sign
    const int z = a.zero;

    const int64_t pos = static_cast<int64_t>(item) * (64 / G) + g;
    const bool has = pos < n_work;
    int p = 0, m = 0, n = 0, ea = 0, eb = 0;
    const uint8_t* A = a.seqs;
    const uint8_t* B = a.seqs;
    if (has) {
        p = order[pos];
        const int x = a.pairs[2 * p], y = a.pairs[2 * p + 1];
        A = a.seqs + a.offsets[x];
        B = a.seqs + a.offsets[y];
        if constexpr (P == Pass::Span) {
            ea = a.end_a[p]; eb = a.end_b[p];
            m = ea + 1; n = eb + 1;
        } else {
            m = static_cast<int>(a.offsets[x + 1] - a.offsets[x]);
            n = static_cast<int>(a.offsets[y + 1] - a.offsets[y]);
        }
    }
    const int S = (m + kRows - 1) / kRows;
    const int s_max = wave_max4(S);
    uint8_t* prof = s_prof + g * (kNRes * G * prof_row_bytes(RMAXT));
    int2* bnd = a.bnd + (static_cast<int64_t>(blockIdx.x) * kPairsPerWave + g) * a.bnd_stride;

    bool bad = false;
    int best = 0, bi = -1, bj = -1;
    unsigned long long computed = 0;   // lane-rows x steps of the item (wave-uniform)

    for (int s = 0; s < s_max; ++s) {
        const bool act = s < S;
        const bool rd = act && s > 0;
        const bool wr = act && s + 1 < S;
        const int row0 = s * kRows;
        const int n_act = act ? n : 0;
        const int n_max = wave_max4(n_act);
        computed += static_cast<unsigned long long>((n_max + G - 1 + 1) & ~1) * 64 * R;
        const bool rd_any = wave_max4(rd ? 1 : 0) != 0;
        const bool wr_any = wave_max4(wr ? 1 : 0) != 0;

        // ---- query profile of this strip: prof[c][gl][r] = M[a_i][c]
        {
            int code[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = row0 + gl * R + r;
                int v = kSent;
                if (act && i < m) {
                    v = (P == Pass::Span) ? A[ea - i] : A[i];
                    if (v > 19) { bad = true; v = kSent; }
                }
                code[r] = v * kMatStride;
            }
            __syncthreads();   // previous strip's readers are done with prof
#pragma unroll 1
            for (int c = 0; c < kNRes; ++c) {
                uint32_t w[W];
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    uint32_t word = 0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int r = 4 * q + k;
                        const int8_t v = (r < R) ? s_mat[code[r] + c] : int8_t(-128);
                        word |= static_cast<uint32_t>(static_cast<uint8_t>(v)) << (8 * k);
                    }
                    w[q] = word;
                }
                uint8_t* dst = prof + (c * G + gl) * RP;
                if constexpr (W == 4) {
                    *reinterpret_cast<uint4*>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
                } else if constexpr (W == 2) {
                    *reinterpret_cast<uint2*>(dst) = make_uint2(w[0], w[1]);
                } else {
                    *reinterpret_cast<uint32_t*>(dst) = w[0];
                }
            }
            __syncthreads();
        }

        // Prefetch loads are unconditional (the index is clamped into the
        // sequence or redirected to a small dummy buffer); whether a loaded
        // value is real is decided when its chunk is switched in, so the loads
        // stay in flight for a whole 16-column chunk.
        const bool live = act && n > 0;
        auto col_raw = [&](int col) -> int {
            const int k = min(col, n - 1);
            const uint8_t* src = live ? ((P == Pass::Span) ? B + (eb - k) : B + k) : a.dummy;
            return *src;
        };
        auto col_in = [&](int v, int col) -> int {
            if (!(act && col < n)) return kSent;
            if (v > 19) { bad = true; v = kSent; }
            return v;
        };
        auto bnd_raw = [&](int col) -> int2 { return bnd[min(col, a.bnd_stride - 1)]; };

        auto sweep = [&](auto multi) {
            constexpr bool kMulti = decltype(multi)::value;
            int HA[R], HB[R], E[R];
#pragma unroll
            for (int r = 0; r < R; ++r) { HA[r] = 0; E[r] = 0; }
            int hdiag = 0, Hout = 0, Fout = 0;
            int feedR = col_in(col_raw(gl), gl);
            int nfeedR = col_raw(G + gl);
            int feedH = 0, feedF = 0;
            int2 nfeed = make_int2(0, 0);
            if constexpr (kMulti) {
                const int2 v0 = bnd_raw(gl);
                feedH = (rd && gl < n) ? v0.x : 0;
                feedF = (rd && gl < n) ? v0.y : 0;
                nfeed = bnd_raw(G + gl);
            }
            int collH = 0, collF = 0;
            int c = dpp_shr1g<G>(feedR, kSent);
            ProfWords<W> pwA = load_prof<W, G>(prof, c, gl);
            ProfWords<W> pwB;

            // one column step: previous column Hi -> this column Ho
            auto cells = [&](int t, const int (&Hi)[R], int (&Ho)[R], const ProfWords<W>& pw) {
                int Htop, F;
                if constexpr (kMulti) {
                    Htop = dpp_shr1g<G>(feedH, Hout);
                    F = dpp_shr1g<G>(feedF, Fout);
                } else {
                    Htop = dpp_shr1_zerog<G>(Hout);
                    F = dpp_shr1_zerog<G>(Fout);
                }
                int colmax = z;
#pragma unroll
                for (int r = 0; r < R; r += 2) {
                    const int d0 = (r == 0) ? hdiag : Hi[r - 1];
                    const int h0 = max3i(d0 + sbyte(pw.w[r >> 2], r & 3), E[r], F);
                    const int g0 = h0 + go;
                    E[r] = max3i(E[r] + ge, g0, z);
                    F = max3i(F + ge, g0, z);
                    Ho[r] = h0;
                    const int h1 = max3i(Hi[r] + sbyte(pw.w[(r + 1) >> 2], (r + 1) & 3), E[r + 1], F);
                    const int g1 = h1 + go;
                    E[r + 1] = max3i(E[r + 1] + ge, g1, z);
                    F = max3i(F + ge, g1, z);
                    Ho[r + 1] = h1;
                    if constexpr (kEnd) colmax = max3i(colmax, h0, h1);
                    else best = max3i(best, h0, h1);
                }
                hdiag = Htop;
                Hout = Ho[R - 1];
                Fout = F;
                if constexpr (kEnd) {
                    if (colmax >= best && colmax > 0) {
                        int ri = R - 1;
#pragma unroll
                        for (int r = R - 1; r >= 0; --r) ri = (Ho[r] == colmax) ? r : ri;
                        const int row = row0 + gl * R + ri;
                        if (colmax > best || row < bi) { best = colmax; bi = row; bj = t - gl; }
                    }
                }
            };
            // boundary row after step t: lane 0 feed advances, lane 15 leaves column t-15
            auto boundary = [&](int t, bool chunk_end) {
                if constexpr (kMulti) {
                    if (chunk_end) {
                        const int col = t + 1 + gl;
                        feedH = (rd && col < n) ? nfeed.x : 0;
                        feedF = (rd && col < n) ? nfeed.y : 0;
                        nfeed = bnd_raw(t + 1 + G + gl);
                    } else {
                        feedH = dpp_shl1_anyg<G>(feedH);
                        feedF = dpp_shl1_anyg<G>(feedF);
                    }
                    collH = dpp_shl1g<G>(Hout, collH);
                    collF = dpp_shl1g<G>(Fout, collF);
                    if ((t & (G - 1)) == G - 1) {
                        const int col = t - 2 * (G - 1) + gl;
                        if (wr && col >= 0 && col < n) bnd[col] = make_int2(collH, collF);
                    }
                }
            };

            // steps rounded up to even: an extra step only touches columns past
            // every subject's end
            const int steps = (n_max + G - 1 + 1) & ~1;
#pragma unroll 1
            for (int t = 0; t < steps; t += 2) {
                {   // step t (even, never the last step of a 16-column chunk)
                    const int feedR2 = dpp_shl1_anyg<G>(feedR);
                    const int cn = dpp_shr1g<G>(feedR2, c);
                    pwB = load_prof<W, G>(prof, cn, gl);
                    // keep the read ahead of this step's cells: the scheduler
                    // would otherwise sink it next to its use a step later
                    __builtin_amdgcn_sched_barrier(0);
                    cells(t, HA, HB, pwA);
                    boundary(t, false);
                    feedR = feedR2;
                    c = cn;
                }
                {   // step t+1
                    const bool chunk_end = ((t + 2) & (G - 1)) == 0;
                    int feedR2;
                    if (chunk_end) {
                        feedR2 = col_in(nfeedR, t + 2 + gl);
                        nfeedR = col_raw(t + 2 + G + gl);
                    } else {
                        feedR2 = dpp_shl1_anyg<G>(feedR);
                    }
                    const int cn = dpp_shr1g<G>(feedR2, c);
                    pwA = load_prof<W, G>(prof, cn, gl);
                    __builtin_amdgcn_sched_barrier(0);
                    cells(t + 1, HB, HA, pwB);
                    boundary(t + 1, chunk_end);
                    feedR = feedR2;
                    c = cn;
                }
            }
            if constexpr (kMulti) {
                const int col = (steps - 1) - 2 * (G - 1) + gl;
                if (wr && col >= 0 && col < n) bnd[col] = make_int2(collH, collF);
                __threadfence();
            }
        };
        if (rd_any || wr_any) sweep(std::true_type{});
        else sweep(std::false_type{});
    }

    // ---- group reductions and output
    int Sbest = best;
#pragma unroll
    for (int k = 1; k < G; k <<= 1) Sbest = max(Sbest, __shfl_xor(Sbest, k, G));
    if constexpr (kEnd) {
        uint32_t key = (best == Sbest && Sbest > 0)
                           ? ((static_cast<uint32_t>(bi) << 16) | static_cast<uint32_t>(bj))
                           : 0xffffffffu;
#pragma unroll
        for (int k = 1; k < G; k <<= 1) {
            const uint32_t o = static_cast<uint32_t>(__shfl_xor(static_cast<int>(key), k, G));
            key = min(key, o);
        }
        bi = Sbest > 0 ? static_cast<int>(key >> 16) : -1;
        bj = Sbest > 0 ? static_cast<int>(key & 0xffffu) : -1;
    }
    if (has && gl == 0) {
        if constexpr (P == Pass::Score) {
            a.scores[p] = Sbest;
        } else if constexpr (P == Pass::ScoreEnd) {
            a.scores[p] = Sbest;
            a.end_a[p] = bi;
            a.end_b[p] = bj;
        } else {
            if (Sbest != a.scores[p] || bi < 0) {
                atomicOr(a.err, kErrCell);
                a.start_a[p] = -1; a.start_b[p] = -1;
            } else {
                a.start_a[p] = ea - bi;
                a.start_b[p] = eb - bj;
            }
        }
    }
    if (bad) atomicOr(a.err, kErrResidue);
    if (a.cells_acc && lane == 0) atomicAdd(a.cells_acc, computed);
}

template <Pass P, int RMAXT>
__global__ __launch_bounds__(64) void k_sw(SwArgs a) {
    __shared__ int8_t s_mat[kNRes * kMatStride];
    __shared__ __attribute__((aligned(16))) uint8_t
        s_prof[kPairsPerWave * kNRes * kGroup * prof_row_bytes(RMAXT)];
    for (int i = threadIdx.x; i < kNRes * kMatStride; i += 64) s_mat[i] = a.mat[i];
    __syncthreads();
    const int n_work = a.ctr->n_work;
    if constexpr (P != Pass::Score && RMAXT == 16) {
        // End and start cells of a few pairs (ClusterMerge's representative
        // pairs above mT: a few thousand per level): at most four pairs per
        // persistent wavefront, so every pair gets a whole wavefront of 64
        // lanes, a quarter of the strips of the 16-lane layout.  The plan's
        // order (rows-per-lane class, strips, columns, descending) takes the
        // longest pairs first.
        if (n_work <= 4 * static_cast<int>(gridDim.x)) {
            while (true) {
                int item = 0;
                if (threadIdx.x == 0) item = atomicAdd(&a.ctr->ticket, 1);
                item = __builtin_amdgcn_readfirstlane(item);
                if (item >= n_work) break;
                const int p = a.order[item];
                const int x = a.pairs[2 * p];
                const int m = (P == Pass::Span) ? a.end_a[p] + 1 : static_cast<int>(a.offsets[x + 1] - a.offsets[x]);
                int strips = (m + 64 * RMAXT - 1) / (64 * RMAXT);
                strips = max(strips, 1);
                int R = (m + 64 * strips - 1) / (64 * strips);
                R += R & 1;
                R = __builtin_amdgcn_readfirstlane(min(max(R, 2), RMAXT));
                if (R <= 2) run_item<2, P, RMAXT, 64>(a, a.order, item, n_work, s_mat, s_prof);
                else if (R <= 4) run_item<4, P, RMAXT, 64>(a, a.order, item, n_work, s_mat, s_prof);
                else if (R <= 6) run_item<6, P, RMAXT, 64>(a, a.order, item, n_work, s_mat, s_prof);
                else if (R <= 8) run_item<8, P, RMAXT, 64>(a, a.order, item, n_work, s_mat, s_prof);
                else if (R <= 10) run_item<10, P, RMAXT, 64>(a, a.order, item, n_work, s_mat, s_prof);
                else if (R <= 12) run_item<12, P, RMAXT, 64>(a, a.order, item, n_work, s_mat, s_prof);
                else if (R <= 14) run_item<14, P, RMAXT, 64>(a, a.order, item, n_work, s_mat, s_prof);
                else run_item<16, P, RMAXT, 64>(a, a.order, item, n_work, s_mat, s_prof);
            }
            return;
        }
    }
    const int n_items = (n_work + kPairsPerWave - 1) / kPairsPerWave;
    while (true) {
        int item = 0;
        if (threadIdx.x == 0) item = atomicAdd(&a.ctr->ticket, 1);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= n_items) break;
        const uint32_t key = a.keys[static_cast<int64_t>(item) * kPairsPerWave];
        const int R = kRMax - static_cast<int>(key >> 24);
        if (R <= 2) run_item<2, P, RMAXT>(a, a.order, item, n_work, s_mat, s_prof);
        else if (R <= 4) run_item<4, P, RMAXT>(a, a.order, item, n_work, s_mat, s_prof);
        else if (R <= 6) run_item<6, P, RMAXT>(a, a.order, item, n_work, s_mat, s_prof);
        else if (R <= 8 || RMAXT == 8) run_item<8, P, RMAXT>(a, a.order, item, n_work, s_mat, s_prof);
        else if constexpr (RMAXT >= 12) {
            if (R <= 10) run_item<10, P, RMAXT>(a, a.order, item, n_work, s_mat, s_prof);
            else if (R <= 12 || RMAXT == 12) run_item<12, P, RMAXT>(a, a.order, item, n_work, s_mat, s_prof);
            else if constexpr (RMAXT >= 16) {
                if (R <= 14) run_item<14, P, RMAXT>(a, a.order, item, n_work, s_mat, s_prof);
                else run_item<16, P, RMAXT>(a, a.order, item, n_work, s_mat, s_prof);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// packed 16-bit score kernel
//
// The same strip / skew / DPP decomposition as run_item, but every register
// holds two pairs: the low 16 bits belong to one pair and the high 16 bits to
// another pair of the same shape class, so each VOP3P instruction advances two
// cells.  E' and F' are clamped at zero, and H, E', F' and the best carry a
// bias B = kPkBias = 128 (the magnitude of the most negative profile byte), so
// Hdiag + s is never negative and every value is a non-negative 16-bit
// integer.  Such integers below 0x7C00 order exactly like binary16 numbers
// (+0, subnormals, normals), so the maxima of three values are one
// v_pk_maximum3_f16 each, and the cell update is 7.5 packed operations for
// two cells:
//     t  = Hdiag + s                   signed saturating add
//     h  = maximum3(t, E', F')         (= max(t, E', F', 0) + B)
//     g  = h - |go|                    unsigned saturating subtract
//     E' = maximum3(E' - |ge|, g, B)   (likewise for F'; B is the zero clamp)
//     best = maximum3(best, h_r, h_r+1)  (two rows at a time)
// plus the sign extension of the int8 profile bytes into 16-bit halves (one
// v_perm per two cells, one shift per four).  No value exceeds the biased
// best, and values of 0x7C00 and above (+Inf and NaN patterns) propagate
// through maximum3, so a pair whose biased best stays below 0x7C00 (score
// below 31616) has its exact score; any other pair is queued for the int32
// kernel (k_sw_over).
// ---------------------------------------------------------------------------
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_adds(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_add_sat(__builtin_bit_cast(s16x2, a),
                                                                      __builtin_bit_cast(s16x2, b)));
}
__device__ __forceinline__ uint32_t pk_maxs(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, a),
                                                                  __builtin_bit_cast(s16x2, b)));
}
__device__ __forceinline__ uint32_t pk_subu(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, a),
                                                                      __builtin_bit_cast(u16x2, b)));
}
// Largest of three pairs of non-negative 16-bit values, compared as binary16
// (v_pk_maximum3_f16).  Patterns 0..0x7BFF are +0, subnormals and finite
// positives, whose order is the integer order; 0x7C00 is +Inf and above are
// NaNs, which the IEEE maximum propagates.  So the result equals the integer
// maximum whenever that is below 0x7C00, and is at least 0x7C00 otherwise.
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pk_max3f(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_maximum(
        __builtin_elementwise_maximum(__builtin_bit_cast(f16x2, a), __builtin_bit_cast(f16x2, b)),
        __builtin_bit_cast(f16x2, c)));
}
// (sign-extended byte k of wa, sign-extended byte k of wb) as two 16-bit
// halves.  v_perm can replicate the sign bit of bytes 1 and 3 of either source
// (selectors 8..11), so odd bytes come straight from the words and even bytes
// from the words shifted left by 8 (sa = wa << 8, sb = wb << 8).
template <int K>
__device__ __forceinline__ uint32_t pk_sbyte(uint32_t wa, uint32_t wb, uint32_t sa, uint32_t sb) {
    constexpr uint32_t kSel1 = 0x0A050801u;   // bytes: a1, sign(a1), b1, sign(b1)
    constexpr uint32_t kSel3 = 0x0B070903u;   // bytes: a3, sign(a3), b3, sign(b3)
    if constexpr (K == 0) return __builtin_amdgcn_perm(sb, sa, kSel1);
    else if constexpr (K == 1) return __builtin_amdgcn_perm(wb, wa, kSel1);
    else if constexpr (K == 2) return __builtin_amdgcn_perm(sb, sa, kSel3);
    else return __builtin_amdgcn_perm(wb, wa, kSel3);
}

template <int W>
__device__ __forceinline__ ProfWords<W> load_prof_at(const uint8_t* p) {
    ProfWords<W> r;
    if constexpr (W >= 4) {
#pragma unroll
        for (int q = 0; q < W; q += 4) {
            uint4 v = *reinterpret_cast<const uint4*>(p + 4 * q);
            r.w[q] = v.x; r.w[q + 1] = v.y; r.w[q + 2] = v.z; r.w[q + 3] = v.w;
        }
    } else if constexpr (W == 2) {
        uint2 v = *reinterpret_cast<const uint2*>(p);
        r.w[0] = v.x; r.w[1] = v.y;
    } else {
        r.w[0] = *reinterpret_cast<const uint32_t*>(p);
    }
    return r;
}

// W words of a lane's profile row: 16-bit profiles are 8-byte aligned
template <int W, bool k16>
__device__ __forceinline__ ProfWords<W> load_prof_any(const uint8_t* p) {
    if constexpr (k16) {
        static_assert(W % 2 == 0, "16-bit profile rows are padded to 8 bytes");
        ProfWords<W> r;
#pragma unroll
        for (int q = 0; q < W; q += 2) {
            uint2 v = *reinterpret_cast<const uint2*>(p + 4 * q);
            r.w[q] = v.x; r.w[q + 1] = v.y;
        }
        return r;
    } else {
        return load_prof_at<W>(p);
    }
}

// kShared: the eight pairs of the item share their query (the plan groups
// them), so one profile serves the whole wavefront; each group builds a
// quarter of its residue rows.  Up to kR16Max rows per lane the shared profile
// holds 16-bit values, so the halves of a register are one v_perm of the two
// pairs' profile words with no shift; above it, int8 values as in the
// two-profile kernel (the LDS of eight wavefronts per CU bounds the 16-bit
// profile at 28 rows per lane).
template <int R, int RMAXT, bool kShared>
__device__ __forceinline__ void run_item_pk(const SwArgs& a, const int32_t* __restrict__ order, int item,
                                            int n_work, const int8_t* __restrict__ s_mat,
                                            uint8_t* __restrict__ s_prof, uint2* __restrict__ s_stage,
                                            uint32_t* __restrict__ s_code) {
    constexpr bool k16 = kShared && R <= kR16Max;   // 16-bit shared profile
    constexpr int RP = k16 ? prof16_row_bytes(R) : prof_row_bytes(R);   // bytes per lane and residue
    constexpr int W = RP / 4;
    constexpr int kRows = kGroup * R;
    constexpr int kColStride = kGroup * RP;          // bytes between the residue rows of a profile
    constexpr int kProfBytes = kNRes * kGroup * prof_row_bytes(RMAXT);
    constexpr uint32_t kSentPk = static_cast<uint32_t>(kSent * kColStride) * 0x10001u;
    const int lane = threadIdx.x;
    const int g = lane >> 4;
    const int gl = lane & 15;
    const uint32_t GO = a.go_pk, GE = a.ge_pk;

    bool has[2];
    int p[2], m[2], n[2];
    const uint8_t* A[2];
    const uint8_t* B[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t pos = static_cast<int64_t>(item) * kPairsPerWavePk + 2 * g + h;
        has[h] = pos < n_work;
        p[h] = 0; m[h] = 0; n[h] = 0;
        A[h] = a.seqs; B[h] = a.seqs;
        if (has[h]) {
            p[h] = order[pos];
            const int x = a.pairs[2 * p[h]], y = a.pairs[2 * p[h] + 1];
            A[h] = a.seqs + a.offsets[x];
            B[h] = a.seqs + a.offsets[y];
            m[h] = static_cast<int>(a.offsets[x + 1] - a.offsets[x]);
            n[h] = static_cast<int>(a.offsets[y + 1] - a.offsets[y]);
        }
    }
    const int S0 = (m[0] + kRows - 1) / kRows;
    const int S1 = (m[1] + kRows - 1) / kRows;
    const int s_max = wave_max4(max(S0, S1));
    uint8_t* prof0 = kShared ? s_prof : s_prof + (2 * g) * kProfBytes;
    uint8_t* prof1 = kShared ? s_prof : prof0 + kProfBytes;
    bool bad_plan = false;
    if constexpr (kShared) {
        // every pair of the item must have group 0's first query
        const uint64_t a0 = reinterpret_cast<uint64_t>(A[0]);
        const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(a0 & 0xffffffffu)));
        const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(a0 >> 32)));
        const uint64_t first = (static_cast<uint64_t>(hi) << 32) | lo;
        bad_plan = (has[0] && reinterpret_cast<uint64_t>(A[0]) != first) ||
                   (has[1] && reinterpret_cast<uint64_t>(A[1]) != first);
    }
    const uint8_t* lp0 = prof0 + gl * RP;
    const uint8_t* lp1 = prof1 + gl * RP;
    int2* bnd = a.bnd + (static_cast<int64_t>(blockIdx.x) * kPairsPerWave + g) * a.bnd_stride;
    uint2* stg = s_stage + g * (kGroup + 1);   // this group's staged boundary chunk (padded: distinct banks)
    // this group's column codes (both pairs' profile offsets) of kGroup
    // columns, column j at j mod kGroup: every lane reads the code of column
    // t + 2 at step t (a broadcast); two steps before a 16-column chunk ends
    // the lanes write the next chunk's codes, just before that step's read
    uint32_t* ring = s_code + g * (kGroup + 1);   // padded: the groups' broadcasts hit different banks

    bool bad = false;
    int badcode = 0;
    // every H, E, F and best value carries the bias kPkBias (in both halves)
    constexpr uint32_t KB = static_cast<uint32_t>(kPkBias) * 0x10001u;
    uint32_t best = KB;
    int sh8 = 8;
    asm("" : "+s"(sh8));   // the profile words' byte shift, as an unknown wave-uniform amount
    unsigned long long computed = 0;   // lane-rows x halves x steps of the item (wave-uniform)

    for (int s = 0; s < s_max; ++s) {
        const bool act0 = s < S0, act1 = s < S1;
        const bool rd0 = act0 && s > 0, rd1 = act1 && s > 0;
        const bool wr0 = act0 && s + 1 < S0, wr1 = act1 && s + 1 < S1;
        const int row0 = s * kRows;
        const int n_act = max(act0 ? n[0] : 0, act1 ? n[1] : 0);
        const int n_max = wave_max4(n_act);
        computed += static_cast<unsigned long long>((n_max + kGroup - 1 + 1) & ~1) * 128 * R;
        const bool rd_any = wave_max4((rd0 || rd1) ? 1 : 0) != 0;
        const bool wr_any = wave_max4((wr0 || wr1) ? 1 : 0) != 0;

        // ---- the two query profiles of this strip: prof_h[c][gl][r] = M[a_i][c]
        {
            int code0[R], code1[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = row0 + gl * R + r;
                int v0 = kSent, v1 = kSent;
                if (act0 && i < m[0]) {
                    v0 = A[0][i];
                    if (v0 > 19) { bad = true; v0 = kSent; }
                }
                if (act1 && i < m[1]) {
                    v1 = A[1][i];
                    if (v1 > 19) { bad = true; v1 = kSent; }
                }
                code0[r] = v0 * kMatStride;
                code1[r] = v1 * kMatStride;
            }
            __syncthreads();   // previous strip's readers are done with the profiles
#pragma unroll 1
            for (int c = kShared ? g : 0; c < kNRes; c += kShared ? kPairsPerWave : 1) {
#pragma unroll
                for (int h = 0; h < (kShared ? 1 : 2); ++h) {
                    uint32_t w[W];
                    constexpr int kPer = k16 ? 2 : 4;        // rows per word
#pragma unroll
                    for (int q = 0; q < W; ++q) {
                        uint32_t word = 0;
#pragma unroll
                        for (int k = 0; k < kPer; ++k) {
                            const int r = kPer * q + k;
                            const int8_t v = (r < R) ? s_mat[(h ? code1[r] : code0[r]) + c] : int8_t(-128);
                            if constexpr (k16)
                                word |= static_cast<uint32_t>(static_cast<uint16_t>(static_cast<int16_t>(v))) << (16 * k);
                            else
                                word |= static_cast<uint32_t>(static_cast<uint8_t>(v)) << (8 * k);
                        }
                        w[q] = word;
                    }
                    uint8_t* dst = (h ? prof1 : prof0) + c * kColStride + gl * RP;
                    if constexpr (k16) {
#pragma unroll
                        for (int q = 0; q < W; q += 2)
                            *reinterpret_cast<uint2*>(dst + 4 * q) = make_uint2(w[q], w[q + 1]);
                    } else if constexpr (W >= 4) {
#pragma unroll
                        for (int q = 0; q < W; q += 4)
                            *reinterpret_cast<uint4*>(dst + 4 * q) = make_uint4(w[q], w[q + 1], w[q + 2], w[q + 3]);
                    } else if constexpr (W == 2) {
                        *reinterpret_cast<uint2*>(dst) = make_uint2(w[0], w[1]);
                    } else {
                        *reinterpret_cast<uint32_t*>(dst) = w[0];
                    }
                }
            }
            __syncthreads();
        }

        // column residues of both pairs, as profile byte offsets in the two halves
        const bool live0 = act0 && n[0] > 0, live1 = act1 && n[1] > 0;
        // the two bytes stay separate until their chunk is switched in, so
        // the loads remain in flight for a whole 16-column chunk
        auto col_raw = [&](int col) -> int2 {
            const uint8_t* s0 = live0 ? B[0] + min(col, n[0] - 1) : a.dummy;
            const uint8_t* s1 = live1 ? B[1] + min(col, n[1] - 1) : a.dummy;
            return make_int2(*s0, *s1);
        };
        // columns outside a pair read the sentinel; a code above 19 is
        // recorded in badcode (reported after the item) and scores as the sentinel
        auto col_in = [&](int2 v, int col) -> uint32_t {
            const bool in0 = act0 && col < n[0], in1 = act1 && col < n[1];
            badcode = max(badcode, max(in0 ? v.x : 0, in1 ? v.y : 0));
            const int c0 = in0 ? min(v.x, kSent) : kSent;
            const int c1 = in1 ? min(v.y, kSent) : kSent;
            return static_cast<uint32_t>(c0 * kColStride) | (static_cast<uint32_t>(c1 * kColStride) << 16);
        };
        auto rd_mask = [&](int col) -> uint32_t {
            return ((rd0 && col < n[0]) ? 0xffffu : 0u) | ((rd1 && col < n[1]) ? 0xffff0000u : 0u);
        };
        auto bnd_raw = [&](int col) -> int2 { return bnd[min(col, a.bnd_stride - 1)]; };

        auto sweep = [&](auto multi) {
            constexpr bool kMulti = decltype(multi)::value;
            uint32_t HA[R], HB[R], E[R];
#pragma unroll
            for (int r = 0; r < R; ++r) { HA[r] = KB; E[r] = KB; }
            uint32_t hdiag = KB, Hout = KB, Fout = KB;
            const uint32_t code0 = col_in(col_raw(gl), gl);
            ring[gl] = code0;
            int2 nfeedR = col_raw(kGroup + gl);
            // lane 0's code of the next step's column (column 1 here)
            uint32_t nc = static_cast<uint32_t>(dpp_shl1_any(static_cast<int>(code0)));
            uint32_t collH = 0, collF = 0;
            uint32_t sH = 0, sF = 0;     // staged top row (H, F) of this step's column
            int2 nfeed = make_int2(0, 0);
            if constexpr (kMulti) {
                const int2 v0 = bnd_raw(gl);
                const uint32_t mk = rd_mask(gl);
                stg[gl] = make_uint2((static_cast<uint32_t>(v0.x) & mk) | (KB & ~mk),
                                     (static_cast<uint32_t>(v0.y) & mk) | (KB & ~mk));
                nfeed = bnd_raw(kGroup + gl);
                const uint2 v = stg[0];
                sH = v.x;
                sF = v.y;
            }
            uint32_t c = static_cast<uint32_t>(dpp_shr1(static_cast<int>(code0), static_cast<int>(kSentPk)));
            ProfWords<W> pa0 = load_prof_any<W, k16>(lp0 + (c & 0xffffu));
            ProfWords<W> pa1 = load_prof_any<W, k16>(lp1 + (c >> 16));
            ProfWords<W> pb0, pb1;

            // staged top row of column t + 1 (multi-strip); a chunk's last
            // step first stages the next chunk
            auto stage_next = [&](int t, bool chunk_last, uint32_t& nsH, uint32_t& nsF) {
                if constexpr (kMulti) {
                    if (chunk_last) {   // stage columns t+1 .. t+16
                        const uint32_t mk = rd_mask(t + 1 + gl);
                        stg[gl] = make_uint2((static_cast<uint32_t>(nfeed.x) & mk) | (KB & ~mk),
                                             (static_cast<uint32_t>(nfeed.y) & mk) | (KB & ~mk));
                        nfeed = bnd_raw(t + 1 + kGroup + gl);
                    }
                    const uint2 v = stg[(t + 1) & (kGroup - 1)];
                    nsH = v.x;
                    nsF = v.y;
                }
            };
            // One column step t.  Multi-strip: lane 0 takes the top row from
            // the group's 16-column chunk of the boundary row staged in LDS
            // (all lanes read the next step's column one step ahead: in the
            // two-profile kernel before the step's cells, in the shared-query
            // kernel, which has no registers to spare, within them; when a
            // chunk ends its lanes stage the next chunk, loaded from global
            // memory 16 steps earlier), and lane 15's bottom row of the
            // previous step is collected into a 16-column register that is
            // written to the boundary row every 16 steps.
            auto cells = [&](int t, const uint32_t (&Hi)[R], uint32_t (&Ho)[R], const ProfWords<W>& w0,
                             const ProfWords<W>& w1, bool chunk_last, bool store) {
                uint32_t Htop, F;
                if constexpr (kMulti) {
                    Htop = static_cast<uint32_t>(dpp_shr1(static_cast<int>(sH), static_cast<int>(Hout)));
                    F = static_cast<uint32_t>(dpp_shr1(static_cast<int>(sF), static_cast<int>(Fout)));
                    if constexpr (kShared) stage_next(t, chunk_last, sH, sF);
                    collH = static_cast<uint32_t>(dpp_shl1(static_cast<int>(Hout), static_cast<int>(collH)));
                    collF = static_cast<uint32_t>(dpp_shl1(static_cast<int>(Fout), static_cast<int>(collF)));
                    if (store) {   // lane j holds the bottom row of column t - 31 + j
                        // keeps the per-lane test inside this rarely taken branch
                        asm volatile("" ::: "memory");
                        const int col = t - 31 + gl;
                        if (col >= 0 && ((wr0 && col < n[0]) || (wr1 && col < n[1])))
                            bnd[col] = make_int2(static_cast<int>(collH), static_cast<int>(collF));
                    }
                } else {
                    // lane 0's top row is the border (biased zero), taken
                    // after the rows below; a zero F there is equivalent,
                    // since every E is at least the bias
                    Htop = 0;
                    F = static_cast<uint32_t>(dpp_shr1_zero(static_cast<int>(Fout)));
                }
                constexpr int kPer = k16 ? 2 : 4;            // rows per profile word
                // int8 rows in even bytes are sign-extended from the words
                // shifted left by 8; a pair's two words of one load form a
                // 64-bit register pair, shifted at once (the byte carried in
                // lands in byte 0, which no selector reads; the amount is
                // opaque to the compiler, which would split a shift by a
                // constant into 32-bit parts)
                uint32_t sw0[W], sw1[W];
                if constexpr (!k16) {
#pragma unroll
                    for (int q = 0; q < W; q += 2) {
                        if (q + 1 < W) {
                            const uint64_t x0 = __builtin_bit_cast(uint64_t, make_uint2(w0.w[q], w0.w[q + 1])) << sh8;
                            const uint64_t x1 = __builtin_bit_cast(uint64_t, make_uint2(w1.w[q], w1.w[q + 1])) << sh8;
                            sw0[q] = static_cast<uint32_t>(x0);
                            sw0[q + 1] = static_cast<uint32_t>(x0 >> 32);
                            sw1[q] = static_cast<uint32_t>(x1);
                            sw1[q + 1] = static_cast<uint32_t>(x1 >> 32);
                        } else {
                            sw0[q] = w0.w[q] << 8;
                            sw1[q] = w1.w[q] << 8;
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const uint32_t wa = w0.w[q], wb = w1.w[q];
                    const uint32_t sa = k16 ? 0u : sw0[q], sb = k16 ? 0u : sw1[q];
#pragma unroll
                    for (int k = 0; k < kPer; ++k) {
                        const int r = kPer * q + k;
                        if (r >= R) break;
                        uint32_t sub;
                        if constexpr (k16) {
                            // 16-bit rows: (row of pair 0, row of pair 1)
                            sub = __builtin_amdgcn_perm(wb, wa, k == 0 ? 0x05040100u : 0x07060302u);
                        } else {
                            if (k == 0) sub = pk_sbyte<0>(wa, wb, sa, sb);
                            else if (k == 1) sub = pk_sbyte<1>(wa, wb, sa, sb);
                            else if (k == 2) sub = pk_sbyte<2>(wa, wb, sa, sb);
                            else sub = pk_sbyte<3>(wa, wb, sa, sb);
                        }
                        const uint32_t d = (r == 0) ? hdiag : Hi[r - 1];
                        // biased: t >= 0 because the bias covers the most
                        // negative profile byte, so H = max(t, E, F) is one
                        // binary16 maximum; the zero clamps become the bias
                        const uint32_t h = pk_max3f(pk_adds(d, sub), E[r], F);
                        const uint32_t go = pk_subu(h, GO);
                        E[r] = pk_max3f(pk_subu(E[r], GE), go, KB);
                        F = pk_max3f(pk_subu(F, GE), go, KB);
                        Ho[r] = h;
                        // two rows per update of the running best
                        if (r & 1) best = pk_max3f(best, Ho[r - 1], h);
                        else if (r == R - 1) best = pk_maxs(best, h);
                    }
                }
                if constexpr (kMulti) {
                    hdiag = Htop;
                } else {
                    // lane 0 of hdiag holds the border from the start and
                    // keeps it (its row_shr source is invalid); hdiag is dead
                    // after row 0, so the move needs no copy
                    (void)Htop;
                    hdiag = static_cast<uint32_t>(dpp_shr1(static_cast<int>(hdiag), static_cast<int>(Hout)));
                }
                Hout = Ho[R - 1];
                Fout = F;
            };

            // column code of step t + 1 from the ring (lane 0) and the lane
            // above (the rest); the code of column t + 2 is read for the next
            // step, after the next chunk's codes when t + 2 starts a chunk
            auto next_code = [&](int t, bool code_chunk) -> uint32_t {
                if (code_chunk) {   // codes of columns t+2 .. t+17
                    ring[(t + 2 + gl) & (kGroup - 1)] = col_in(nfeedR, t + 2 + gl);
                    nfeedR = col_raw(t + 2 + kGroup + gl);
                }
                const uint32_t cn = static_cast<uint32_t>(dpp_shr1(static_cast<int>(nc), static_cast<int>(c)));
                nc = ring[(t + 2) & (kGroup - 1)];
                return cn;
            };
            // step t (even: never the last step of a 16-column chunk)
            auto step_even = [&](int t, bool store, bool code_chunk) {
                uint32_t nsH = sH, nsF = sF;
                if constexpr (!kShared) stage_next(t, false, nsH, nsF);
                const uint32_t cn = next_code(t, code_chunk);
                pb0 = load_prof_any<W, k16>(lp0 + (cn & 0xffffu));
                pb1 = load_prof_any<W, k16>(lp1 + (cn >> 16));
                __builtin_amdgcn_sched_barrier(0);
                cells(t, HA, HB, pa0, pa1, false, store);
                c = cn;
                if constexpr (!kShared) { sH = nsH; sF = nsF; }
            };
            // step t (odd: never two steps before a chunk's end)
            auto step_odd = [&](int t, bool chunk_last) {
                uint32_t nsH = sH, nsF = sF;
                if constexpr (!kShared) stage_next(t, chunk_last, nsH, nsF);
                const uint32_t cn = next_code(t, false);
                pa0 = load_prof_any<W, k16>(lp0 + (cn & 0xffffu));
                pa1 = load_prof_any<W, k16>(lp1 + (cn >> 16));
                __builtin_amdgcn_sched_barrier(0);
                cells(t, HB, HA, pb0, pb1, chunk_last, false);
                c = cn;
                if constexpr (!kShared) { sH = nsH; sF = nsF; }
            };
            const int steps = (n_max + kGroup - 1 + 1) & ~1;
            // Two-profile kernel: whole 16-column chunks fully unrolled, so that
            // which step ends a chunk (feed reload) or starts one (boundary
            // store) is known at compile time; the two-step loop takes the
            // remaining steps.  The shared-query kernel runs every step in the
            // two-step loop (its rows per lane leave no registers for the
            // unrolled code).
            const int full = kShared ? 0 : steps & ~(kGroup - 1);
            int t = 0;
#pragma unroll 1
            for (; t < full; t += kGroup) {
                const bool st = t > 0;
#pragma unroll
                for (int u = 0; u < kGroup; u += 2) {
                    step_even(t + u, u == 0 && st, u + 2 == kGroup);
                    step_odd(t + u + 1, u + 2 == kGroup);
                }
            }
#pragma unroll 1
            for (; t < steps; t += 2) {
                step_even(t, (t & (kGroup - 1)) == 0 && t > 0, ((t + 2) & (kGroup - 1)) == 0);
                step_odd(t + 1, ((t + 2) & (kGroup - 1)) == 0);
            }
            if constexpr (kMulti) {
                // collect the last step's bottom row and write the final columns
                collH = static_cast<uint32_t>(dpp_shl1(static_cast<int>(Hout), static_cast<int>(collH)));
                collF = static_cast<uint32_t>(dpp_shl1(static_cast<int>(Fout), static_cast<int>(collF)));
                const int col = steps - 31 + gl;
                if (col >= 0 && ((wr0 && col < n[0]) || (wr1 && col < n[1])))
                    bnd[col] = make_int2(static_cast<int>(collH), static_cast<int>(collF));
                __threadfence();
            }
        };
        if (rd_any || wr_any) sweep(std::true_type{});
        else sweep(std::false_type{});
    }

    // ---- group reduction (both halves at once) and output
    uint32_t Sb = best;
#pragma unroll
    for (int k = 1; k < kGroup; k <<= 1)
        Sb = pk_maxs(Sb, static_cast<uint32_t>(__shfl_xor(static_cast<int>(Sb), k, kGroup)));
    if (gl == 0) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (!has[h]) continue;
            const int v = static_cast<int>(h ? (Sb >> 16) : (Sb & 0xffffu));
            if (v >= kPkSaturated) {
                const int slot = atomicAdd(&a.ctr->n_over, 1);
                a.over[slot] = p[h];
            } else {
                a.scores[p[h]] = v - kPkBias;
            }
        }
    }
    if (bad || badcode > 19) atomicOr(a.err, kErrResidue);
    if (bad_plan) atomicOr(a.err, kErrPlan);
    if (a.cells_acc && lane == 0) atomicAdd(a.cells_acc, computed);
}

// rows per lane of an item from its first pair's query (lists without keys)
__device__ __forceinline__ int item_rows(const SwArgs& a, const int32_t* order, int item, int per_item, int rmax,
                                         bool even) {
    const int p = order[static_cast<int64_t>(item) * per_item];
    const int x = a.pairs[2 * p];
    const int m = static_cast<int>(a.offsets[x + 1] - a.offsets[x]);
    int R, strips;
    shape_for(m, rmax, even, R, strips);
    return __builtin_amdgcn_readfirstlane(R);
}

template <int RMAXT>
__global__ __launch_bounds__(64) void k_sw_pk(SwArgs a) {
    __shared__ int8_t s_mat[kNRes * kMatStride];
    __shared__ __attribute__((aligned(16))) uint8_t
        s_prof[kPairsPerWave * 2 * kNRes * kGroup * prof_row_bytes(RMAXT)];
    __shared__ uint2 s_stage[kPairsPerWave * (kGroup + 1)];
    __shared__ uint32_t s_code[kPairsPerWave * (kGroup + 1)];
    const int n_work = a.n_work_ptr ? *a.n_work_ptr : a.ctr->n_work;
    if (n_work == 0) return;
    int* ticket = a.ticket ? a.ticket : &a.ctr->ticket;
    for (int i = threadIdx.x; i < kNRes * kMatStride; i += 64) s_mat[i] = a.mat[i];
    __syncthreads();
    const int n_items = (n_work + kPairsPerWavePk - 1) / kPairsPerWavePk;
    while (true) {
        int item = 0;
        if (threadIdx.x == 0) item = atomicAdd(ticket, 1);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= n_items) break;
        int R;
        if (a.keys) R = kRMax - static_cast<int>(a.keys[static_cast<int64_t>(item) * kPairsPerWavePk] >> 24);
        else R = item_rows(a, a.order, item, kPairsPerWavePk, RMAXT, false);
        if (R <= 1) run_item_pk<1, RMAXT, false>(a, a.order, item, n_work, s_mat, s_prof, s_stage, s_code);
        else if (R == 2) run_item_pk<2, RMAXT, false>(a, a.order, item, n_work, s_mat, s_prof, s_stage, s_code);
        else if (R == 3) run_item_pk<3, RMAXT, false>(a, a.order, item, n_work, s_mat, s_prof, s_stage, s_code);
        else if (R == 4 || RMAXT == 4) run_item_pk<4, RMAXT, false>(a, a.order, item, n_work, s_mat, s_prof, s_stage, s_code);
        else if constexpr (RMAXT >= 8) {
            if (R == 5) run_item_pk<5, RMAXT, false>(a, a.order, item, n_work, s_mat, s_prof, s_stage, s_code);
            else if (R == 6) run_item_pk<6, RMAXT, false>(a, a.order, item, n_work, s_mat, s_prof, s_stage, s_code);
            else if (R == 7) run_item_pk<7, RMAXT, false>(a, a.order, item, n_work, s_mat, s_prof, s_stage, s_code);
            else run_item_pk<8, RMAXT, false>(a, a.order, item, n_work, s_mat, s_prof, s_stage, s_code);
        }
    }
}

// Shared-query packed kernel: items of eight pairs with one query, any rows
// per lane up to 32 (strips of up to 512 rows), one LDS profile per wavefront.
template <int R>
__device__ __forceinline__ void run_pkq_range(const SwArgs& a, int Rw, int item, int n_work, const int8_t* s_mat,
                                              uint8_t* s_prof, uint2* s_stage, uint32_t* s_code) {
    if (Rw == R) run_item_pk<R, kRMaxQ, true>(a, a.order, item, n_work, s_mat, s_prof, s_stage, s_code);
    else if constexpr (R < kRMaxQ) run_pkq_range<R + 1>(a, Rw, item, n_work, s_mat, s_prof, s_stage, s_code);
}

__global__ __launch_bounds__(64) void k_sw_pkq(SwArgs a) {
    __shared__ int8_t s_mat[kNRes * kMatStride];
    __shared__ __attribute__((aligned(16))) uint8_t
        s_prof[kNRes * kGroup * cmax(prof_row_bytes(kRMaxQ), prof16_row_bytes(kR16Max))];
    __shared__ uint2 s_stage[kPairsPerWave * (kGroup + 1)];
    __shared__ uint32_t s_code[kPairsPerWave * (kGroup + 1)];
    const int n_work = a.n_work_ptr ? *a.n_work_ptr : a.ctr->n_work;
    if (n_work == 0) return;
    int* ticket = a.ticket ? a.ticket : &a.ctr->ticket;
    for (int i = threadIdx.x; i < kNRes * kMatStride; i += 64) s_mat[i] = a.mat[i];
    __syncthreads();
    const int n_items = (n_work + kPairsPerWavePk - 1) / kPairsPerWavePk;
    while (true) {
        int item = 0;
        if (threadIdx.x == 0) item = atomicAdd(ticket, 1);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= n_items) break;
        const int R = item_rows(a, a.order, item, kPairsPerWavePk, kRMaxQ, false);
        run_pkq_range<1>(a, R, item, n_work, s_mat, s_prof, s_stage, s_code);
    }
}

// ---- shared-query plan
// the two-profile kernel's shape key (rows-per-lane class, strips, columns)
// for every pair of a list (entries at or past *count: skip key)
__global__ void k_keys_list(SwArgs a, const int32_t* list, const int32_t* count, int64_t n, uint32_t* keys) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    uint32_t key = kSkipKey;
    if (i < *count) {
        const int p = list[i];
        const int x = a.pairs[2 * p], y = a.pairs[2 * p + 1];
        const int m = static_cast<int>(a.offsets[x + 1] - a.offsets[x]);
        const int nn = static_cast<int>(a.offsets[y + 1] - a.offsets[y]);
        int R, strips;
        shape_for(m, a.rmax, false, R, strips);
        key = (static_cast<uint32_t>(kRMax - R) << 24) | (static_cast<uint32_t>(255 - min(strips, 255)) << 16) |
              static_cast<uint32_t>(65535 - nn);
    }
    keys[i] = key;
}

__global__ void k_plan_q(SwArgs a, uint64_t* keys, int32_t* vals) {
    const int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (p >= a.n_pairs) return;
    uint64_t key = ~0ull;
    if (a.n_live && p >= *a.n_live) {
        keys[p] = key;
        vals[p] = static_cast<int32_t>(p);
        return;
    }
    const int x = a.pairs[2 * p], y = a.pairs[2 * p + 1];
    if (x < 0 || x >= a.n_seqs || y < 0 || y >= a.n_seqs) {
        atomicOr(a.err, kErrIndex);
    } else {
        const int64_t lx = a.offsets[x + 1] - a.offsets[x];
        const int64_t ly = a.offsets[y + 1] - a.offsets[y];
        if (lx > kMaxLen || ly > kMaxLen || lx < 0 || ly < 0) {
            atomicOr(a.err, kErrLength);
        } else if (lx == 0 || ly == 0) {
            a.scores[p] = 0;
        } else {
            int R, strips;
            shape_for(static_cast<int>(lx), kRMaxQ, false, R, strips);
            key = (static_cast<uint64_t>(kRMaxQ - R) << 58) |
                  (static_cast<uint64_t>(255 - min(strips, 255)) << 50) |
                  (static_cast<uint64_t>(static_cast<uint32_t>(x)) << 16) |
                  static_cast<uint64_t>(65535 - static_cast<int>(ly));
            atomicAdd(&a.ctr->n_work, 1);
        }
    }
    keys[p] = key;
    vals[p] = static_cast<int32_t>(p);
}

// start_in[i] = i at the first pair of a query run, else 0 (a max-scan then
// gives every position its run start)
__global__ void k_heads_q(const uint64_t* keys, int64_t n, const int32_t* n_work, int32_t* start_in) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    const bool head = i < *n_work && (i == 0 || (keys[i] >> 16) != (keys[i - 1] >> 16));
    start_in[i] = head ? static_cast<int32_t>(i) : 0;
}

// run length at each run start (binary search for the run's end), then the
// item lists: the first 8 * floor(len / 8) pairs of a run go to list A
__global__ void k_runlen_q(const uint64_t* keys, const int32_t* start, int64_t n, const int32_t* n_work,
                           int32_t* run_len) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int64_t w = *n_work;
    if (i >= n || i >= w || start[i] != i) return;
    const uint64_t q = keys[i] >> 16;
    int64_t lo = i, hi = w - 1;          // last index with the same run key
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if ((keys[mid] >> 16) == q) lo = mid;
        else hi = mid - 1;
    }
    run_len[i] = static_cast<int32_t>(lo - i + 1);
}
// An item goes to list A only if its subjects' lengths are close (the
// shortest at least 7/8 of the longest, the item runs to the longest);
// otherwise its pairs are packed with like shapes from other queries.
__global__ void k_flags_q(const uint64_t* keys, const int32_t* start, const int32_t* run_len, int64_t n,
                          const int32_t* n_work, uint8_t* flag_a, uint8_t* flag_b) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    uint8_t fa = 0, fb = 0;
    if (i < *n_work) {
        const int32_t s = start[i];
        const int32_t len = run_len[s];
        if ((i - s) < (len & ~7)) {
            const int64_t first = s + ((i - s) & ~7);       // columns sorted longest first
            const int n_long = 65535 - static_cast<int>(keys[first] & 0xffffu);
            const int n_short = 65535 - static_cast<int>(keys[first + 7] & 0xffffu);
            fa = 8 * n_short >= 7 * n_long;
        }
        fb = !fa;
    }
    flag_a[i] = fa;
    flag_b[i] = fb;
}

// int32 re-run of the pairs whose packed score saturated (usually none): the
// widest rows-per-lane shape handles any query length
__global__ __launch_bounds__(64) void k_sw_over(SwArgs a) {
    __shared__ int8_t s_mat[kNRes * kMatStride];
    __shared__ __attribute__((aligned(16))) uint8_t s_prof[kPairsPerWave * kNRes * kGroup * prof_row_bytes(kRMax)];
    const int n_work = a.ctr->n_over;
    if (n_work == 0) return;
    for (int i = threadIdx.x; i < kNRes * kMatStride; i += 64) s_mat[i] = a.mat[i];
    __syncthreads();
    const int n_items = (n_work + kPairsPerWave - 1) / kPairsPerWave;
    while (true) {
        int item = 0;
        if (threadIdx.x == 0) item = atomicAdd(&a.ctr->ticket_over, 1);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= n_items) break;
        run_item<kRMax, Pass::Score, kRMax>(a, a.over, item, n_work, s_mat, s_prof);
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t launch_plan(const SwArgs& a, Pass pass, uint32_t* keys, int32_t* vals, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, a.ctr);
    if (a.n_pairs > 0) {
        const int64_t blocks = (a.n_pairs + 255) / 256;
        hipLaunchKernelGGL(k_plan, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, a,
                           static_cast<int>(pass), keys, vals);
    }
    return hipGetLastError();
}

template <Pass P>
static hipError_t launch_pass(const SwArgs& a, int grid, hipStream_t s) {
    switch (a.rmax) {
        case 8:  hipLaunchKernelGGL((k_sw<P, 8>), dim3(grid), dim3(64), 0, s, a); break;
        case 12: hipLaunchKernelGGL((k_sw<P, 12>), dim3(grid), dim3(64), 0, s, a); break;
        default: hipLaunchKernelGGL((k_sw<P, 16>), dim3(grid), dim3(64), 0, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_sw(const SwArgs& a, Pass pass, int grid, hipStream_t s) {
    switch (pass) {
        case Pass::Score:    return launch_pass<Pass::Score>(a, grid, s);
        case Pass::ScoreEnd: return launch_pass<Pass::ScoreEnd>(a, grid, s);
        default:             return launch_pass<Pass::Span>(a, grid, s);
    }
}

template <Pass P>
static int occupancy(int rmax) {
    int nb = 0;
    hipError_t e;
    switch (rmax) {
        case 8:  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sw<P, 8>, 64, 0); break;
        case 12: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sw<P, 12>, 64, 0); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sw<P, 16>, 64, 0); break;
    }
    return (e != hipSuccess || nb < 1) ? 1 : nb;
}

hipError_t launch_plan_q(const SwArgs& a, uint64_t* keys, int32_t* vals, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, a.ctr);
    if (a.n_pairs > 0)
        hipLaunchKernelGGL(k_plan_q, dim3(static_cast<unsigned>((a.n_pairs + 255) / 256)), dim3(256), 0, s, a, keys,
                           vals);
    return hipGetLastError();
}
hipError_t launch_runs_q(const uint64_t* keys_sorted, int64_t n, const int32_t* n_work, int32_t* start_in,
                         hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_heads_q, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, keys_sorted, n,
                           n_work, start_in);
    return hipGetLastError();
}
hipError_t launch_flags_q(const uint64_t* keys_sorted, const int32_t* start, int64_t n, const int32_t* n_work,
                          int32_t* run_len, uint8_t* flag_a, uint8_t* flag_b, hipStream_t s) {
    if (n > 0) {
        const dim3 g(static_cast<unsigned>((n + 255) / 256));
        hipLaunchKernelGGL(k_runlen_q, g, dim3(256), 0, s, keys_sorted, start, n, n_work, run_len);
        hipLaunchKernelGGL(k_flags_q, g, dim3(256), 0, s, keys_sorted, start, run_len, n, n_work, flag_a, flag_b);
    }
    return hipGetLastError();
}
hipError_t launch_keys_list(const SwArgs& a, const int32_t* list, const int32_t* count, int64_t n, uint32_t* keys,
                            hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_keys_list, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, a, list, count,
                           n, keys);
    return hipGetLastError();
}
hipError_t launch_sw_pkq(const SwArgs& a_list, const SwArgs& b_list, int grid, int grid_b, int grid_over,
                         hipStream_t s, hipStream_t side, hipEvent_t fork, hipEvent_t join) {
    // list B runs on the side stream, concurrently with list A: its blocks
    // take the compute units that list A leaves free (its tail, or the slots
    // its occupancy leaves); the saturated pairs of both are rescored after
    // the join
    hipError_t e = hipEventRecord(fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, fork, 0);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sw_pk<8>), dim3(grid_b), dim3(64), 0, side, b_list);
    hipLaunchKernelGGL(k_sw_pkq, dim3(grid), dim3(64), 0, s, a_list);
    e = hipEventRecord(join, side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, join, 0);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sw_over, dim3(grid_over), dim3(64), 0, s, a_list);
    return hipGetLastError();
}
int sw_pkq_blocks_per_cu() {
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sw_pkq, 64, 0);
    return (e != hipSuccess || nb < 1) ? 1 : nb;
}

hipError_t launch_sw_pk(const SwArgs& a, int grid, int grid_over, hipStream_t s) {
    switch (a.rmax) {
        case 4:  hipLaunchKernelGGL((k_sw_pk<4>), dim3(grid), dim3(64), 0, s, a); break;
        default: hipLaunchKernelGGL((k_sw_pk<8>), dim3(grid), dim3(64), 0, s, a); break;
    }
    hipLaunchKernelGGL(k_sw_over, dim3(grid_over), dim3(64), 0, s, a);
    return hipGetLastError();
}

int sw_pk_blocks_per_cu(int rmax) {
    int nb = 0;
    hipError_t e = (rmax == 4) ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sw_pk<4>, 64, 0)
                               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sw_pk<8>, 64, 0);
    return (e != hipSuccess || nb < 1) ? 1 : nb;
}

int sw_over_blocks_per_cu() {
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sw_over, 64, 0);
    return (e != hipSuccess || nb < 1) ? 1 : nb;
}

int sw_blocks_per_cu(Pass pass, int rmax) {
    switch (pass) {
        case Pass::Score:    return occupancy<Pass::Score>(rmax);
        case Pass::ScoreEnd: return occupancy<Pass::ScoreEnd>(rmax);
        default:             return occupancy<Pass::Span>(rmax);
    }
}

}  // namespace cmk
