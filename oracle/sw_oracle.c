/*
 * sw_oracle.c -- plain scalar Smith-Waterman with affine gaps (Gotoh).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the CPU oracle the GPU path is
 * checked against.  Only the tests, the smoke check and the benchmark's CPU
 * baseline leg load it.  It shares no code, header or table with the GPU
 * library and must never be linked into it.
 *
 * What it computes (Section 4 of the paper: the similarity f of two proteins
 * is the Smith-Waterman local-alignment score under a substitution matrix;
 * the paper does not state its gap model, so the affine model below is the
 * reading used throughout):
 *
 *   An alignment of substrings of a (length m) and b (length n) is a sequence
 *   of columns: aligned pairs (i,j), gaps in b (i,-) and gaps in a (-,j).  Its
 *   score is the sum of M[a_i][b_j] over aligned pairs plus W(k) for every
 *   maximal run of k gap columns of one kind, W(k) = go + (k-1)*ge.
 *   S(a,b) = max(0, best alignment score).
 *
 *   Gotoh recurrence over rows i in [0,m) and columns j in [0,n), borders
 *   H = 0 and E = F = -infinity (here -2^30):
 *     E[i][j] = max(E[i][j-1] + ge, H[i][j-1] + go)      gap in a (horizontal)
 *     F[i][j] = max(F[i-1][j] + ge, H[i-1][j] + go)      gap in b (vertical)
 *     H[i][j] = max(0, H[i-1][j-1] + M[a_i][b_j], E[i][j], F[i][j])
 *     S = max over all cells of H.
 *
 *   End cell: the first cell in row-major order (smallest i, then smallest j)
 *   with H = S, when S > 0; (-1,-1) when S = 0.
 *
 *   Start cell (needed by the coverage test of Section 4): the same recurrence
 *   run on a' = reverse(a[0..i*]) and b' = reverse(b[0..j*]); its maximum
 *   equals S, and with (r*, c*) its first row-major cell holding S the start
 *   is (i* - r*, j* - c*): among optimal alignments that end at the end cell,
 *   the one with the lexicographically largest start.
 *
 * Build: gcc -O2 -shared -fPIC -o liboracle_sw.so sw_oracle.c
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_NEG_INF (-(1 << 30))

static int32_t imax(int32_t x, int32_t y) { return x > y ? x : y; }

/* Full Gotoh table walk; returns S and the first row-major end cell. */
static int32_t gotoh(const uint8_t* a, int32_t m, const uint8_t* b, int32_t n,
                     const int32_t* M, int32_t go, int32_t ge,
                     int32_t* end_i, int32_t* end_j)
{
    /* Hrow[j] holds H[i-1][j] while row i is computed, then H[i][j]. */
    int32_t* Hrow = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t* Frow = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t best = 0, bi = -1, bj = -1;
    for (int32_t j = 0; j < n; ++j) { Hrow[j] = 0; Frow[j] = ORACLE_NEG_INF; }
    for (int32_t i = 0; i < m; ++i) {
        int32_t diag = 0;                 /* H[i-1][j-1]; left border is 0 */
        int32_t left = 0;                 /* H[i][j-1]   */
        int32_t E = ORACLE_NEG_INF;       /* E[i][j-1]   */
        const int32_t* row = M + 20 * (int32_t)a[i];
        for (int32_t j = 0; j < n; ++j) {
            int32_t up = Hrow[j];         /* H[i-1][j] */
            E = imax(E + ge, left + go);
            int32_t F = imax(Frow[j] + ge, up + go);
            int32_t H = imax(0, imax(diag + row[b[j]], imax(E, F)));
            Frow[j] = F;
            Hrow[j] = H;
            diag = up;
            left = H;
            if (H > best) { best = H; bi = i; bj = j; }
        }
    }
    free(Hrow);
    free(Frow);
    if (best == 0) { bi = -1; bj = -1; }
    *end_i = bi;
    *end_j = bj;
    return best;
}

int32_t oracle_sw(const uint8_t* a, int32_t m, const uint8_t* b, int32_t n,
                  const int32_t* M, int32_t go, int32_t ge,
                  int32_t* end_i, int32_t* end_j)
{
    return gotoh(a, m, b, n, M, go, ge, end_i, end_j);
}

/* Score, end cell and start cell.  Returns 0 on success, -1 if the reverse
 * pass does not reproduce S (which would mean an error in this file). */
int32_t oracle_sw_span(const uint8_t* a, int32_t m, const uint8_t* b, int32_t n,
                       const int32_t* M, int32_t go, int32_t ge, int32_t* out5)
{
    int32_t ei, ej;
    int32_t S = gotoh(a, m, b, n, M, go, ge, &ei, &ej);
    out5[0] = S; out5[1] = ei; out5[2] = ej; out5[3] = -1; out5[4] = -1;
    if (S == 0) return 0;
    int32_t mr = ei + 1, nr = ej + 1;
    uint8_t* ra = (uint8_t*)malloc((size_t)mr);
    uint8_t* rb = (uint8_t*)malloc((size_t)nr);
    for (int32_t k = 0; k < mr; ++k) ra[k] = a[ei - k];
    for (int32_t k = 0; k < nr; ++k) rb[k] = b[ej - k];
    int32_t ri, rj;
    int32_t S2 = gotoh(ra, mr, rb, nr, M, go, ge, &ri, &rj);
    free(ra);
    free(rb);
    if (S2 != S) return -1;
    out5[3] = ei - ri;
    out5[4] = ej - rj;
    return 0;
}

/* Loop over a pair list: rows come from pairs[2p], columns from pairs[2p+1].
 * end_a / end_b may be NULL. */
void oracle_sw_batch(const uint8_t* res, const int64_t* off, const int32_t* pairs, int64_t n_pairs,
                     const int32_t* M, int32_t go, int32_t ge,
                     int32_t* scores, int32_t* end_a, int32_t* end_b)
{
    for (int64_t p = 0; p < n_pairs; ++p) {
        int32_t x = pairs[2 * p], y = pairs[2 * p + 1];
        int32_t ei, ej;
        scores[p] = gotoh(res + off[x], (int32_t)(off[x + 1] - off[x]),
                          res + off[y], (int32_t)(off[y + 1] - off[y]), M, go, ge, &ei, &ej);
        if (end_a) end_a[p] = ei;
        if (end_b) end_b[p] = ej;
    }
}

/* Same, with start cells; out5 is [n_pairs][5] = score, end_a, end_b, start_a, start_b.
 * Returns the number of pairs whose reverse pass failed (0 expected). */
int64_t oracle_span_batch(const uint8_t* res, const int64_t* off, const int32_t* pairs, int64_t n_pairs,
                          const int32_t* M, int32_t go, int32_t ge, int32_t* out5)
{
    int64_t bad = 0;
    for (int64_t p = 0; p < n_pairs; ++p) {
        int32_t x = pairs[2 * p], y = pairs[2 * p + 1];
        bad += oracle_sw_span(res + off[x], (int32_t)(off[x + 1] - off[x]),
                              res + off[y], (int32_t)(off[y + 1] - off[y]), M, go, ge, out5 + 5 * p) != 0;
    }
    return bad;
}

/* Traceback of the optimal local alignment between its start cell (sa, sb)
 * and end cell (ea, eb), score S > 0 (a reading: the paper's final stage
 * records scores only and leaves alignments to later analysis).  Every optimal
 * local alignment with these ends begins and ends with an aligned pair (a
 * leading or trailing gap only lowers the score), so it is a global alignment
 * of a[sa..ea] with b[sb..eb] that starts and ends with aligned pairs, and
 * the best such global alignment scores exactly S.  Three Gotoh states over
 * the box (r = i - sa, c = j - sb):
 *   Mt[r][c] = s(a_i, b_j) + max(Mt, X, Y)[r-1][c-1]    (Mt[0][0] = s: the start)
 *   X[r][c]  = max(Mt[r-1][c] + go, X[r-1][c] + ge, Y[r-1][c] + go)   a_i against a gap ('I')
 *   Y[r][c]  = max(Mt[r][c-1] + go, Y[r][c-1] + ge, X[r][c-1] + go)   a gap against b_j ('D')
 * Cells outside the box are -infinity.  The walk starts in Mt at the end cell
 * and, where several predecessors give a state's value, takes Mt first, then
 * the state's own extension, then the other gap state.  The columns are
 * written start to end as 'M', 'I', 'D'.  Returns the number of columns, -1
 * if the end value is not S, -2 if cap is too small. */
int32_t oracle_sw_traceback(const uint8_t* a, const uint8_t* b, const int32_t* M, int32_t go, int32_t ge,
                            int32_t S, int32_t sa, int32_t sb, int32_t ea, int32_t eb, char* ops, int32_t cap)
{
    const int32_t R = ea - sa + 1, C = eb - sb + 1;
    const size_t cells = (size_t)R * (size_t)C;
    int32_t* Mt = (int32_t*)malloc(cells * sizeof(int32_t));
    int32_t* X = (int32_t*)malloc(cells * sizeof(int32_t));
    int32_t* Y = (int32_t*)malloc(cells * sizeof(int32_t));
#define AT(T, r, c) (((r) < 0 || (c) < 0) ? ORACLE_NEG_INF : (T)[(size_t)(r) * C + (c)])
    for (int32_t r = 0; r < R; ++r) {
        for (int32_t c = 0; c < C; ++c) {
            const int32_t s = M[20 * a[sa + r] + b[sb + c]];
            int32_t d;
            if (r == 0 && c == 0) d = 0;
            else d = imax(imax(AT(Mt, r - 1, c - 1), AT(X, r - 1, c - 1)), AT(Y, r - 1, c - 1));
            Mt[(size_t)r * C + c] = d <= ORACLE_NEG_INF ? ORACLE_NEG_INF : d + s;
            X[(size_t)r * C + c] = imax(imax(AT(Mt, r - 1, c) + go, AT(X, r - 1, c) + ge), AT(Y, r - 1, c) + go);
            Y[(size_t)r * C + c] = imax(imax(AT(Mt, r, c - 1) + go, AT(Y, r, c - 1) + ge), AT(X, r, c - 1) + go);
            if (X[(size_t)r * C + c] < ORACLE_NEG_INF) X[(size_t)r * C + c] = ORACLE_NEG_INF;
            if (Y[(size_t)r * C + c] < ORACLE_NEG_INF) Y[(size_t)r * C + c] = ORACLE_NEG_INF;
        }
    }
    int32_t n_ops = -1;
    if (Mt[cells - 1] == S) {
        char* rev = (char*)malloc((size_t)(R + C));
        int32_t k = 0, r = R - 1, c = C - 1, state = 0;   /* 0 = Mt, 1 = X, 2 = Y */
        for (;;) {
            if (state == 0) {
                rev[k++] = 'M';
                if (r == 0 && c == 0) break;
                const int32_t v = Mt[(size_t)r * C + c] - M[20 * a[sa + r] + b[sb + c]];
                if (AT(Mt, r - 1, c - 1) == v) state = 0;
                else if (AT(X, r - 1, c - 1) == v) state = 1;
                else state = 2;
                --r; --c;
            } else if (state == 1) {
                rev[k++] = 'I';
                const int32_t v = X[(size_t)r * C + c];
                if (AT(Mt, r - 1, c) + go == v) state = 0;
                else if (AT(X, r - 1, c) + ge == v) state = 1;
                else state = 2;
                --r;
            } else {
                rev[k++] = 'D';
                const int32_t v = Y[(size_t)r * C + c];
                if (AT(Mt, r, c - 1) + go == v) state = 0;
                else if (AT(Y, r, c - 1) + ge == v) state = 2;
                else state = 1;
                --c;
            }
        }
        if (k > cap) n_ops = -2;
        else {
            for (int32_t q = 0; q < k; ++q) ops[q] = rev[k - 1 - q];
            n_ops = k;
        }
        free(rev);
    }
#undef AT
    free(Mt);
    free(X);
    free(Y);
    return n_ops;
}

/* Batch: out5 rows are (score, end_a, end_b, start_a, start_b) as written by
 * oracle_span_batch; pair p's columns go to ops[op_off[p] ..], their number to
 * n_ops[p] (0 when the score is 0).  Returns the number of failed pairs. */
int64_t oracle_traceback_batch(const uint8_t* res, const int64_t* off, const int32_t* pairs, int64_t n_pairs,
                               const int32_t* M, int32_t go, int32_t ge, const int32_t* out5,
                               const int64_t* op_off, char* ops, int32_t* n_ops)
{
    int64_t bad = 0;
    for (int64_t p = 0; p < n_pairs; ++p) {
        const int32_t* q = out5 + 5 * p;
        if (q[0] <= 0) { n_ops[p] = 0; continue; }
        const int32_t x = pairs[2 * p], y = pairs[2 * p + 1];
        n_ops[p] = oracle_sw_traceback(res + off[x], res + off[y], M, go, ge, q[0], q[3], q[4], q[1], q[2],
                                       ops + op_off[p], (int32_t)(op_off[p + 1] - op_off[p]));
        bad += n_ops[p] < 0;
    }
    return bad;
}
