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
// Not a hot-path kernel: one lane per pair, 64 pairs of like box shape per
// wavefront, the box swept in strips of columns with the row above in
// registers; each strip's left boundary column and one predecessor byte per
// cell go to scratch, then every lane walks back through its own bytes.
// Batches are split into launches so that the scratch stays bounded.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "../../include/cm.h"
#include "cm_internal.h"
#include "cm_runtime.h"

namespace cmtb {

constexpr int32_t kNegInf = -(1 << 30);
// predecessor bytes per launch: one byte per cell of every lane's share of its
// wavefront's largest box, so the bound sets how many wavefronts run at once
// (the buffer is released when the call returns)
constexpr int64_t kScratchCells = int64_t(16) << 30;

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

// One wavefront per 64 pairs of like box shape (sorted on the host), one pair
// per lane, all lanes stepping through the wavefront's largest box together.
// The box is swept in strips of kStrip columns: within a strip the three
// states of the row above live in registers, and only the strip's left
// boundary column (three values per row) goes through memory, written by the
// previous strip and read one row ahead.  Boundary columns and predecessor
// bytes are interleaved by lane ([r][lane], [r][c][lane]), so every access of
// a step is one contiguous line.  A lane outside its own box only waits; then
// each lane walks back through its own predecessor bytes.
constexpr int kStrip = 16;
struct Wave { int64_t dir_off, row_off; int32_t rmax, cmax; };

__global__ __launch_bounds__(64) void k_tb(TbArgs a, Matrix mat, const int32_t* lane_pair, const Wave* waves,
                                           uint8_t* dir_base, int32_t* row_base) {
    const int lane = threadIdx.x;
    __shared__ int32_t s_mat[400];
    for (int k = lane; k < 400; k += 64) s_mat[k] = mat.m[k];
    __syncthreads();
    const Wave w = waves[blockIdx.x];
    const int32_t p = lane_pair[static_cast<int64_t>(blockIdx.x) * 64 + lane];
    int32_t R = 0, C = 0;
    const uint8_t* A = a.seqs;
    const uint8_t* B = a.seqs;
    if (p >= 0) {
        const int32_t sa = a.start_a[p], sb = a.start_b[p];
        R = a.end_a[p] - sa + 1;
        C = a.end_b[p] - sb + 1;
        A = a.seqs + a.offsets[a.pairs[2 * p]] + sa;
        B = a.seqs + a.offsets[a.pairs[2 * p + 1]] + sb;
    }
    uint8_t* dir = dir_base + w.dir_off + lane;
    // two boundary columns (read / write), each three planes of rmax rows
    const int64_t plane = static_cast<int64_t>(w.rmax) * 64;
    int32_t* bnd[2] = {row_base + w.row_off + lane, row_base + w.row_off + 3 * plane + lane};
    const int32_t go = a.go, ge = a.ge;
    auto clamp = [](int32_t v) { return v < kNegInf ? kNegInf : v; };
    int32_t last = kNegInf;
    bool bad = false;
    int cur = 0;
    for (int32_t c0 = 0; c0 < w.cmax; c0 += kStrip) {
        const int32_t* in = bnd[cur];
        int32_t* outb = bnd[1 - cur];
        int32_t uM[kStrip], uX[kStrip], uY[kStrip];           // row above, columns c0 .. c0 + kStrip - 1
        uint32_t bcode[kStrip];
#pragma unroll
        for (int k = 0; k < kStrip; ++k) {
            uM[k] = kNegInf; uX[k] = kNegInf; uY[k] = kNegInf;
            const int32_t c = c0 + k;
            const uint32_t v = c < C ? B[c] : 0u;
            bad |= v > 19;
            bcode[k] = min(v, 19u);
        }
        // left boundary (column c0 - 1) of row 0, and of the row above (for the diagonal)
        int32_t nM = kNegInf, nX = kNegInf, nY = kNegInf;
        if (c0 > 0 && 0 < R) { nM = in[0]; nX = in[plane]; nY = in[2 * plane]; }
        int32_t pM = kNegInf, pX = kNegInf, pY = kNegInf;      // (r - 1, c0 - 1)
        for (int32_t r = 0; r < w.rmax; ++r) {
            const bool row_in = r < R;
            int32_t lM = nM, lX = nX, lY = nY;                 // (r, c0 - 1)
            // the next row's left boundary, loaded a row ahead
            nM = kNegInf; nX = kNegInf; nY = kNegInf;
            if (c0 > 0 && r + 1 < R) {
                const int64_t q = static_cast<int64_t>(r + 1) * 64;
                nM = in[q]; nX = in[plane + q]; nY = in[2 * plane + q];
            }
            const uint32_t ar = row_in ? A[r] : 0u;
            bad |= row_in && ar > 19;
            const int32_t* srow = s_mat + 20 * min(ar, 19u);
            int32_t dM = pM, dX = pX, dY = pY;                 // diagonal of column c0
            pM = lM; pX = lX; pY = lY;
#pragma unroll
            for (int k = 0; k < kStrip; ++k) {
                const int32_t c = c0 + k;
                if (!row_in || c >= C) continue;
                const int32_t oM = uM[k], oX = uX[k], oY = uY[k];   // (r - 1, c)
                int32_t d, pm;
                if (r == 0 && c == 0) {
                    d = 0;
                    pm = 3;
                } else {
                    d = dM; pm = 0;
                    if (dX > d) { d = dX; pm = 1; }
                    if (dY > d) { d = dY; pm = 2; }
                }
                const int32_t m = d <= kNegInf ? kNegInf : d + srow[bcode[k]];
                // a_i against a gap, from the row above: 0 Mt, 1 X, 2 Y
                int32_t vx = oM + go, px = 0;
                if (oX + ge > vx) { vx = oX + ge; px = 1; }
                if (oY + go > vx) { vx = oY + go; px = 2; }
                vx = clamp(vx);
                // a gap against b_j, from the left: 0 Mt, 1 Y, 2 X
                int32_t vy = lM + go, py = 0;
                if (lY + ge > vy) { vy = lY + ge; py = 1; }
                if (lX + go > vy) { vy = lX + go; py = 2; }
                vy = clamp(vy);
                dir[(static_cast<int64_t>(r) * w.cmax + c) * 64] = static_cast<uint8_t>(pm | (px << 2) | (py << 4));
                dM = oM; dX = oX; dY = oY;
                uM[k] = m; uX[k] = vx; uY[k] = vy;
                lM = m; lX = vx; lY = vy;
                last = m;
            }
            // this row's last strip column is the next strip's left boundary
            if (row_in && c0 + kStrip < C) {
                const int64_t q = static_cast<int64_t>(r) * 64;
                outb[q] = lM; outb[plane + q] = lX; outb[2 * plane + q] = lY;
            }
        }
        cur = 1 - cur;
    }
    if (p < 0) return;
    if (bad) { atomicOr(a.err, cmk::kErrResidue); a.n_ops[p] = -1; return; }
    if (last != a.scores[p]) { atomicOr(a.err, cmk::kErrTrace); a.n_ops[p] = -1; return; }
    // walk back twice: count the columns, then write them start to end
    int32_t len = 0;
    for (int pass = 0; pass < 2; ++pass) {
        int32_t r = R - 1, c = C - 1, state = 0, k = 0;
        uint8_t* out = a.ops + a.op_offsets[p];
        bool ok = true;
        while (true) {
            if (r < 0 || c < 0 || k >= R + C) { ok = false; break; }
            const uint8_t byte = dir[(static_cast<int64_t>(r) * w.cmax + c) * 64];
            uint8_t op;
            bool done = false;
            if (state == 0) {
                op = 'M';
                const int pm = byte & 3;
                if (pm == 3) done = true;
                else { state = pm; --r; --c; }
            } else if (state == 1) {
                op = 'I';
                state = (byte >> 2) & 3;         // 0 Mt, 1 X, 2 Y
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
    CM_TRY
    if (!ctx) return fail(CM_EINVAL, "ctx is NULL");
    if (n_pairs < 0 || n_seqs < 0) return fail(CM_EINVAL, "negative size");
    if (n_pairs == 0) return CM_OK;
    if (n_pairs > static_cast<int64_t>(0x7fffffff)) return fail(CM_EINVAL, "n_pairs too large");
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
    // pairs with a box, sorted by shape, 64 to a wavefront; launches over
    // runs of wavefronts whose predecessor bytes fit the scratch bound
    std::vector<int32_t> order;
    for (size_t p = 0; p < n; ++p)
        if (cells[p] > 0) order.push_back(static_cast<int32_t>(p));
    auto rows_of = [&](int32_t p) { return static_cast<int32_t>(cells[p] / cols[p]); };
    std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return cols[x] != cols[y] ? cols[x] < cols[y] : (rows_of(x) != rows_of(y) ? rows_of(x) < rows_of(y) : x < y);
    });
    const size_t n_waves = (order.size() + 63) / 64;
    // every wavefront's predecessor bytes (its largest rows x columns, 64 lanes)
    // must fit the per-launch bound; checked before anything is launched
    for (size_t w = 0; w < n_waves; ++w) {
        int32_t rmax = 0, cmax = 0;
        for (size_t k = 64 * w; k < std::min(order.size(), 64 * w + 64); ++k) {
            rmax = std::max(rmax, rows_of(order[k]));
            cmax = std::max(cmax, cols[order[k]]);
        }
        const int64_t wd = static_cast<int64_t>(rmax) * cmax * 64;
        if (wd > cmtb::kScratchCells)
            return fail(CM_EUNSUPPORTED,
                        "traceback: boxes of up to %d x %d cells in one wavefront need %lld bytes of predecessor "
                        "scratch, above the %lld-byte bound (boxes of up to 2^28 cells, e.g. 16384 x 16384)", rmax,
                        cmax, static_cast<long long>(wd), static_cast<long long>(cmtb::kScratchCells));
    }
    std::vector<cmtb::Wave> waves;
    std::vector<int32_t> lane_pair;
    size_t w0 = 0;
    while (w0 < n_waves) {
        waves.clear();
        lane_pair.clear();
        int64_t dir_bytes = 0, row_ints = 0;
        size_t w1 = w0;
        while (w1 < n_waves) {
            int32_t rmax = 0, cmax = 0;
            for (size_t k = 64 * w1; k < std::min(order.size(), 64 * w1 + 64); ++k) {
                rmax = std::max(rmax, rows_of(order[k]));
                cmax = std::max(cmax, cols[order[k]]);
            }
            const int64_t wd = static_cast<int64_t>(rmax) * cmax * 64;
            if (w1 > w0 && dir_bytes + wd > cmtb::kScratchCells) break;
            waves.push_back({dir_bytes, row_ints, rmax, cmax});
            for (size_t k = 64 * w1; k < 64 * w1 + 64; ++k) lane_pair.push_back(k < order.size() ? order[k] : -1);
            dir_bytes += wd;
            row_ints += 6 * static_cast<int64_t>(rmax) * 64;     // two boundary columns, three states
            ++w1;
        }
        const size_t m = w1 - w0;
        const size_t meta_bytes = m * sizeof(cmtb::Wave) + lane_pair.size() * 4;
        if (!ctx->tb_dir.ensure(static_cast<size_t>(std::max<int64_t>(dir_bytes, 1))) ||
            !ctx->tb_rows.ensure(static_cast<size_t>(std::max<int64_t>(row_ints, 1)) * 4) ||
            !ctx->tb_offs.ensure(meta_bytes))
            return fail(CM_ENOMEM, "traceback scratch (%lld bytes)", static_cast<long long>(dir_bytes));
        cmtb::Wave* d_waves = static_cast<cmtb::Wave*>(ctx->tb_offs.ptr);
        int32_t* d_lanes = reinterpret_cast<int32_t*>(d_waves + m);
        e = hipMemcpyAsync(d_waves, waves.data(), m * sizeof(cmtb::Wave), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_lanes, lane_pair.data(), lane_pair.size() * 4, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return cmrt::hip_fail(e, "traceback plan");
        hipLaunchKernelGGL(cmtb::k_tb, dim3(static_cast<unsigned>(m)), dim3(64), 0, st, a, mat, d_lanes, d_waves,
                           static_cast<uint8_t*>(ctx->tb_dir.ptr), static_cast<int32_t*>(ctx->tb_rows.ptr));
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);   // the host tables and scratch are reused
        if (e != hipSuccess) return cmrt::hip_fail(e, "traceback");
        w0 = w1;
    }
    ctx->tb_dir.release();
    ctx->tb_rows.release();
    return CM_OK;
    CM_CATCH
}
