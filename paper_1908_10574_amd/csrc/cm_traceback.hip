// cm_traceback.hip -- alignment columns of found pairs (cm_sw_traceback_batch).
//
// For a pair with score S > 0, end cell (ea, eb) and start cell (sa, sb)
// (from cm_sw_score_batch and cm_sw_span_batch), the optimal local alignment
// between those cells is a global alignment of a[sa..ea] with b[sb..eb] that
// begins and ends with an aligned pair (a leading or trailing gap would only
// lower the score), and the best such alignment scores exactly S.  Three
// Gotoh states over the box (r = i - sa, c = j - sb):
//   Mt[r][c] = s(a_i, b_j) + max(Mt, X, Y)[r-1][c-1]     Mt[0][0] = s (the start)
//   X[r][c]  = max(Mt[r-1][c] + go, X[r-1][c] + ge, Y[r-1][c] + go)   a_i against a gap: 'I'
//   Y[r][c]  = max(Mt[r][c-1] + go, Y[r][c-1] + ge, X[r][c-1] + go)   a gap against b_j: 'D'
// with everything outside the box at -infinity.  Ties are broken by a fixed
// preference, Mt first, then the state's own extension, then the other gap
// state; the walk back from Mt at the end cell gives the columns, written
// start to end as 'M', 'I', 'D'.
//
// Not a hot-path kernel: one thread per pair runs the box row by row, keeps
// one row of the three states and one predecessor byte per cell in scratch,
// then walks back.  Batches are split so that the scratch stays bounded.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "../../include/cm.h"
#include "cm_internal.h"
#include "cm_runtime.h"

namespace cmtb {

constexpr int32_t kNegInf = -(1 << 30);
constexpr int64_t kScratchCells = int64_t(1) << 30;   // predecessor bytes per launch

struct Matrix { int32_t m[400]; };

struct TbArgs {
    const uint8_t* seqs;
    const int64_t* offsets;
    int32_t n_seqs;
    const int32_t* pairs;
    const int32_t* scores;
    const int32_t* end_a;
    const int32_t* end_b;
    const int32_t* start_a;
    const int32_t* start_b;
    const int64_t* op_offsets;
    uint8_t* ops;
    int32_t* n_ops;
    int32_t go, ge;
    uint32_t* err;
};

// box size of every pair (0: no columns to write) after checking its cells
// and its share of the column buffer
__global__ void k_tb_box(TbArgs a, int64_t n, int64_t* cells, int32_t* cols) {
    const int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (p >= n) return;
    cells[p] = 0;
    cols[p] = 0;
    if (a.scores[p] <= 0) { a.n_ops[p] = 0; return; }
    a.n_ops[p] = -1;
    const int32_t x = a.pairs[2 * p], y = a.pairs[2 * p + 1];
    if (x < 0 || y < 0 || x >= a.n_seqs || y >= a.n_seqs) { atomicOr(a.err, cmk::kErrIndex); return; }
    const int64_t lx = a.offsets[x + 1] - a.offsets[x], ly = a.offsets[y + 1] - a.offsets[y];
    const int32_t sa = a.start_a[p], sb = a.start_b[p], ea = a.end_a[p], eb = a.end_b[p];
    if (sa < 0 || sb < 0 || sa > ea || sb > eb || ea >= lx || eb >= ly) { atomicOr(a.err, cmk::kErrCell); return; }
    const int64_t R = ea - sa + 1, C = eb - sb + 1;
    if (a.op_offsets[p + 1] - a.op_offsets[p] < R + C) { atomicOr(a.err, cmk::kErrCapacity); return; }
    cells[p] = R * C;
    cols[p] = static_cast<int32_t>(C);
}

// one thread per pair of [p0, p1): the box, then the walk back
__global__ void k_tb(TbArgs a, Matrix mat, int64_t p0, int64_t p1, const int64_t* cells, const int64_t* dir_off,
                     const int64_t* row_off, uint8_t* dir_base, int32_t* row_base) {
    const int64_t p = p0 + blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (p >= p1 || cells[p] == 0) return;
    const int32_t x = a.pairs[2 * p], y = a.pairs[2 * p + 1];
    const int32_t sa = a.start_a[p], sb = a.start_b[p];
    const int32_t R = a.end_a[p] - sa + 1, C = a.end_b[p] - sb + 1;
    const uint8_t* A = a.seqs + a.offsets[x] + sa;
    const uint8_t* B = a.seqs + a.offsets[y] + sb;
    uint8_t* dir = dir_base + dir_off[p - p0];
    int32_t* rM = row_base + row_off[p - p0];
    int32_t* rX = rM + C;
    int32_t* rY = rX + C;
    const int32_t go = a.go, ge = a.ge;
    auto clamp = [](int32_t v) { return v < kNegInf ? kNegInf : v; };
    int32_t last = kNegInf;
    for (int32_t r = 0; r < R; ++r) {
        const int32_t ar = A[r];
        if (ar > 19) { atomicOr(a.err, cmk::kErrResidue); a.n_ops[p] = -1; return; }
        int32_t dM = kNegInf, dX = kNegInf, dY = kNegInf;      // previous row, column c - 1
        int32_t lM = kNegInf, lX = kNegInf, lY = kNegInf;      // this row, column c - 1
        for (int32_t c = 0; c < C; ++c) {
            const int32_t bc = B[c];
            if (bc > 19) { atomicOr(a.err, cmk::kErrResidue); a.n_ops[p] = -1; return; }
            const int32_t uM = r ? rM[c] : kNegInf, uX = r ? rX[c] : kNegInf, uY = r ? rY[c] : kNegInf;
            // aligned pair: predecessor state at the diagonal (3 = the start)
            int32_t d, pm;
            if (r == 0 && c == 0) {
                d = 0;
                pm = 3;
            } else {
                d = dM; pm = 0;
                if (dX > d) { d = dX; pm = 1; }
                if (dY > d) { d = dY; pm = 2; }
            }
            const int32_t m = d <= kNegInf ? kNegInf : d + mat.m[20 * ar + bc];
            // a_i against a gap, from the row above: 0 Mt, 1 X, 2 Y
            int32_t vx = uM + go, px = 0;
            if (uX + ge > vx) { vx = uX + ge; px = 1; }
            if (uY + go > vx) { vx = uY + go; px = 2; }
            vx = clamp(vx);
            // a gap against b_j, from the left: 0 Mt, 1 Y, 2 X
            int32_t vy = lM + go, py = 0;
            if (lY + ge > vy) { vy = lY + ge; py = 1; }
            if (lX + go > vy) { vy = lX + go; py = 2; }
            vy = clamp(vy);
            dir[static_cast<int64_t>(r) * C + c] = static_cast<uint8_t>(pm | (px << 2) | (py << 4));
            dM = uM; dX = uX; dY = uY;
            rM[c] = m; rX[c] = vx; rY[c] = vy;
            lM = m; lX = vx; lY = vy;
            last = m;
        }
    }
    if (last != a.scores[p]) { atomicOr(a.err, cmk::kErrTrace); a.n_ops[p] = -1; return; }
    // walk back twice: count the columns, then write them start to end
    int32_t len = 0;
    for (int pass = 0; pass < 2; ++pass) {
        int32_t r = R - 1, c = C - 1, state = 0, k = 0;
        uint8_t* out = a.ops + a.op_offsets[p];
        bool ok = true;
        while (true) {
            if (r < 0 || c < 0 || k >= R + C) { ok = false; break; }
            const uint8_t byte = dir[static_cast<int64_t>(r) * C + c];
            uint8_t op;
            bool done = false;
            if (state == 0) {
                op = 'M';
                const int pm = byte & 3;
                if (pm == 3) done = true;
                else { state = pm; --r; --c; }
            } else if (state == 1) {
                op = 'I';
                const int px = (byte >> 2) & 3;
                state = px;                      // 0 Mt, 1 X, 2 Y
                --r;
            } else {
                op = 'D';
                const int py = (byte >> 4) & 3;
                state = py == 0 ? 0 : (py == 1 ? 2 : 1);
                --c;
            }
            if (pass == 1) out[len - 1 - k] = op;
            ++k;
            if (done) break;
        }
        if (!ok) { atomicOr(a.err, cmk::kErrTrace); a.n_ops[p] = -1; return; }
        len = k;
    }
    a.n_ops[p] = len;
}

}  // namespace cmtb

using cmrt::fail;

extern "C" cm_status cm_sw_traceback_batch(cm_context* ctx, const uint8_t* seqs, const int64_t* offsets,
                                           int32_t n_seqs, const int32_t* pairs, int64_t n_pairs,
                                           const int32_t* matrix, int32_t gap_open, int32_t gap_extend,
                                           const int32_t* scores, const int32_t* end_a, const int32_t* end_b,
                                           const int32_t* start_a, const int32_t* start_b,
                                           const int64_t* op_offsets, uint8_t* ops, int32_t* n_ops, void* stream) {
    if (!ctx) return fail(CM_EINVAL, "ctx is NULL");
    if (n_pairs < 0 || n_seqs < 0) return fail(CM_EINVAL, "negative size");
    if (n_pairs == 0) return CM_OK;
    if (!offsets || !pairs || !matrix || !scores || !end_a || !end_b || !start_a || !start_b || !op_offsets ||
        !ops || !n_ops)
        return fail(CM_EINVAL, "NULL argument");
    cm_status s = cmrt::check_gaps(gap_open, gap_extend);
    if (s != CM_OK) return s;
    int8_t mat8[cmk::kNRes * cmk::kMatStride];
    s = cmrt::check_matrix(matrix, mat8);
    if (s != CM_OK) return s;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return cmrt::hip_fail(e, "hipSetDevice");
    hipStream_t st = static_cast<hipStream_t>(stream);
    cmtb::TbArgs a;
    a.seqs = seqs; a.offsets = offsets; a.n_seqs = n_seqs; a.pairs = pairs; a.scores = scores;
    a.end_a = end_a; a.end_b = end_b; a.start_a = start_a; a.start_b = start_b;
    a.op_offsets = op_offsets; a.ops = ops; a.n_ops = n_ops;
    a.go = gap_open; a.ge = gap_extend; a.err = ctx->err_flag;
    cmtb::Matrix mat;
    for (int k = 0; k < 400; ++k) mat.m[k] = matrix[k];
    const size_t n = static_cast<size_t>(n_pairs);
    if (!ctx->tb_meta.ensure(n * 12)) return fail(CM_ENOMEM, "traceback sizes for %lld pairs", (long long)n_pairs);
    int64_t* d_cells = static_cast<int64_t*>(ctx->tb_meta.ptr);
    int32_t* d_cols = reinterpret_cast<int32_t*>(d_cells + n);
    hipLaunchKernelGGL(cmtb::k_tb_box, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, a, n_pairs,
                       d_cells, d_cols);
    std::vector<int64_t> cells(n);
    std::vector<int32_t> cols(n);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(cells.data(), d_cells, n * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(cols.data(), d_cols, n * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return cmrt::hip_fail(e, "traceback sizes");
    // launches over runs of pairs whose predecessor bytes fit the scratch bound
    std::vector<int64_t> offs;
    size_t p0 = 0;
    while (p0 < n) {
        size_t p1 = p0;
        int64_t dir_bytes = 0, row_ints = 0;
        offs.clear();
        while (p1 < n && (p1 == p0 || dir_bytes + cells[p1] <= cmtb::kScratchCells)) {
            offs.push_back(dir_bytes);
            dir_bytes += cells[p1];
            ++p1;
        }
        const size_t m = p1 - p0;
        for (size_t q = 0; q < m; ++q) {
            offs.push_back(row_ints);
            row_ints += 3 * static_cast<int64_t>(cols[p0 + q]);
        }
        if (!ctx->tb_dir.ensure(static_cast<size_t>(std::max<int64_t>(dir_bytes, 1))) ||
            !ctx->tb_rows.ensure(static_cast<size_t>(std::max<int64_t>(row_ints, 1)) * 4) ||
            !ctx->tb_offs.ensure(offs.size() * 8))
            return fail(CM_ENOMEM, "traceback scratch (%lld cells)", static_cast<long long>(dir_bytes));
        int64_t* d_offs = static_cast<int64_t*>(ctx->tb_offs.ptr);
        e = hipMemcpyAsync(d_offs, offs.data(), offs.size() * 8, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return cmrt::hip_fail(e, "traceback offsets");
        hipLaunchKernelGGL(cmtb::k_tb, dim3(static_cast<unsigned>((m + 63) / 64)), dim3(64), 0, st, a, mat,
                           static_cast<int64_t>(p0), static_cast<int64_t>(p1), d_cells, d_offs, d_offs + m,
                           static_cast<uint8_t*>(ctx->tb_dir.ptr), static_cast<int32_t*>(ctx->tb_rows.ptr));
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);   // the host offsets and scratch are reused
        if (e != hipSuccess) return cmrt::hip_fail(e, "traceback");
        p0 = p1;
    }
    return CM_OK;
}
