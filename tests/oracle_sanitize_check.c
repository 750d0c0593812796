/* Memory and undefined-behaviour check of the C oracle (test infrastructure):
 * built with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitized.py and run over every ordered pair of 60
 * sequences (empty, one and two residues, random 4- and 20-letter sequences,
 * near-copies of their neighbours) under five gap models.  Every entry point
 * runs; the batch calls must agree with the single-pair calls, the columns
 * buffer is sized exactly, and everything allocated is freed (leak check).
 * Prints "ok: ..." and exits 0 on success. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int32_t oracle_sw(const uint8_t*, int32_t, const uint8_t*, int32_t, const int32_t*, int32_t, int32_t, int32_t*, int32_t*);
int32_t oracle_sw_span(const uint8_t*, int32_t, const uint8_t*, int32_t, const int32_t*, int32_t, int32_t, int32_t*);
void oracle_sw_batch(const uint8_t*, const int64_t*, const int32_t*, int64_t, const int32_t*, int32_t, int32_t,
                     int32_t*, int32_t*, int32_t*);
int64_t oracle_span_batch(const uint8_t*, const int64_t*, const int32_t*, int64_t, const int32_t*, int32_t, int32_t,
                          int32_t*);
int64_t oracle_traceback_batch(const uint8_t*, const int64_t*, const int32_t*, int64_t, const int32_t*, int32_t,
                               int32_t, const int32_t*, const int64_t*, char*, int32_t*);

static uint64_t st = 88172645463325252ull;
static uint32_t rnd(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return (uint32_t)st; }

int main(void) {
    int32_t M[400];
    for (int x = 0; x < 20; ++x)
        for (int y = 0; y < 20; ++y) M[20 * x + y] = x == y ? 4 + (int)(rnd() % 8) : (int)(rnd() % 8) - 4;
    for (int x = 0; x < 20; ++x)
        for (int y = 0; y < x; ++y) M[20 * x + y] = M[20 * y + x];
    const int n = 60;
    int64_t off[61];
    off[0] = 0;
    int32_t len[60];
    for (int k = 0; k < n; ++k) {
        len[k] = k < 3 ? k : (int32_t)(rnd() % 300);     /* empty, 1, 2 residues, then random */
        off[k + 1] = off[k] + len[k];
    }
    uint8_t* res = malloc((size_t)off[n] + 1);
    for (int k = 0; k < n; ++k)
        for (int i = 0; i < len[k]; ++i) {
            /* every third sequence copies most of the previous one, others use 4 letters or all 20 */
            uint8_t v = (uint8_t)(k % 2 ? rnd() % 4 : rnd() % 20);
            if (k % 3 == 0 && k > 3 && i < len[k - 1] && rnd() % 10) v = res[off[k - 1] + i];
            res[off[k] + i] = v;
        }
    const int P = n * n;
    int32_t* pairs = malloc(sizeof(int32_t) * 2 * P);
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) { pairs[2 * (a * n + b)] = a; pairs[2 * (a * n + b) + 1] = b; }
    const int32_t gaps[5][2] = {{-11, -1}, {-5, -5}, {-3, 0}, {-1, -1}, {-2, -1}};
    int32_t* sc = malloc(4 * P); int32_t* ea = malloc(4 * P); int32_t* eb = malloc(4 * P);
    int32_t* out5 = malloc(4 * 5 * P);
    int64_t* op_off = malloc(8 * (P + 1));
    int32_t* n_ops = malloc(4 * P);
    long checks = 0;
    for (int g = 0; g < 5; ++g) {
        const int32_t go = gaps[g][0], ge = gaps[g][1];
        oracle_sw_batch(res, off, pairs, P, M, go, ge, sc, ea, eb);
        int64_t bad = oracle_span_batch(res, off, pairs, P, M, go, ge, out5);
        if (bad) { printf("span bad %lld\n", (long long)bad); return 1; }
        op_off[0] = 0;
        for (int p = 0; p < P; ++p) {
            int64_t cap = out5[5 * p] > 0 ? (out5[5 * p + 1] - out5[5 * p + 3] + 1) + (out5[5 * p + 2] - out5[5 * p + 4] + 1) : 0;
            op_off[p + 1] = op_off[p] + cap;
        }
        char* ops = malloc((size_t)op_off[P] + 1);
        bad = oracle_traceback_batch(res, off, pairs, P, M, go, ge, out5, op_off, ops, n_ops);
        if (bad) { printf("traceback bad %lld\n", (long long)bad); return 1; }
        for (int p = 0; p < P; ++p) {
            int32_t s5[5];
            const int a = pairs[2 * p], b = pairs[2 * p + 1];
            int32_t s = oracle_sw_span(res + off[a], len[a], res + off[b], len[b], M, go, ge, s5);
            int32_t ei, ej;
            int32_t s2 = oracle_sw(res + off[a], len[a], res + off[b], len[b], M, go, ge, &ei, &ej);
            if (s != 0 || s5[0] != sc[p] || s2 != sc[p] || memcmp(s5, out5 + 5 * p, sizeof s5)) { printf("mismatch %d (%d,%d) g=%d: s=%d s2=%d sc=%d s5=[%d %d %d %d %d] out5=[%d %d %d %d %d] ea/eb=%d %d\n", p, a, b, g, s, s2, sc[p], s5[0], s5[1], s5[2], s5[3], s5[4], out5[5*p], out5[5*p+1], out5[5*p+2], out5[5*p+3], out5[5*p+4], ea[p], eb[p]); return 1; }
            ++checks;
        }
        free(ops);
    }
    printf("ok: %ld pair checks, %lld residues\n", checks, (long long)off[n]);
    free(res); free(pairs); free(sc); free(ea); free(eb); free(out5); free(op_off); free(n_ops);
    return 0;
}
