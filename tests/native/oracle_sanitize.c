/*
 * Drives the CPU oracle (oracle/lw_oracle.c) through its whole interface on
 * many small inputs so that it can run under AddressSanitizer and
 * UndefinedBehaviorSanitizer: every linkage, n = 1 .. 40, random and tied
 * matrices, truncated runs (max_merges), fp64 runs, replays of valid and
 * invalid merge lists, rejected input (NaN, inf, 2^101) and bad arguments.
 * Prints "ok" and exits 0 when every call returned what it should.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int lw_oracle_f32(const float *dist, int64_t n, int link, int64_t max_merges, int32_t *out_i, int32_t *out_j,
                  float *out_h, int32_t *out_size, int nthreads, int64_t *merges_done);
int lw_oracle_f64(const double *dist, int64_t n, int link, int64_t max_merges, int32_t *out_i, int32_t *out_j,
                  double *out_h, int32_t *out_size, int nthreads, int64_t *merges_done);
int lw_replay_f64(const float *dist, int64_t n, int link, int64_t count, const int32_t *mi, const int32_t *mj,
                  double *h64, double *min64, int64_t opt_stride, int nthreads);

static uint64_t state = 88172645463325252ull;
static double next_unit(void) {  /* xorshift64 */
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) / 9007199254740992.0;
}

#define CHECK(cond, ...)                    \
    do {                                    \
        if (!(cond)) {                      \
            fprintf(stderr, __VA_ARGS__);   \
            fprintf(stderr, "\n");          \
            return 1;                       \
        }                                   \
    } while (0)

int main(void) {
    for (int n = 1; n <= 40; ++n) {
        float *d = malloc(sizeof(float) * n * n);
        double *d64 = malloc(sizeof(double) * n * n);
        int m = n > 1 ? n - 1 : 1;
        int32_t *mi = malloc(sizeof(int32_t) * m), *mj = malloc(sizeof(int32_t) * m), *ms = malloc(sizeof(int32_t) * m);
        float *mh = malloc(sizeof(float) * m);
        double *mh64 = malloc(sizeof(double) * m), *h64 = malloc(sizeof(double) * m), *min64 = malloc(sizeof(double) * m);
        for (int kind = 0; kind < 3; ++kind) {
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) {
                    double v = kind == 0 ? next_unit() * 10.0 : kind == 1 ? (double)(1 + (int)(next_unit() * 3)) : 1.0;
                    d[a * n + b] = a == b ? 0.0f : (float)v;
                    d64[a * n + b] = d[a * n + b];
                }
            for (int link = 0; link <= 5; ++link) {
                int64_t done = -1;
                int rc = lw_oracle_f32(d, n, link, -1, mi, mj, mh, ms, 2, &done);
                CHECK(rc == 0 && done == n - 1, "f32 n=%d link=%d rc=%d done=%lld", n, link, rc, (long long)done);
                for (int s = 0; s < n - 1; ++s)
                    CHECK(mi[s] >= 0 && mi[s] < mj[s] && mj[s] < n && ms[s] >= 2 && ms[s] <= n, "record n=%d", n);
                rc = lw_replay_f64(d, n, link, n - 1, mi, mj, h64, min64, 1, 2);
                CHECK(rc == 0, "replay n=%d link=%d rc=%d", n, link, rc);
                if (n > 2) {  /* a list that reuses a retired slot is rejected */
                    int32_t keep = mj[1];
                    mj[1] = mj[0];
                    if (mi[1] < mj[1]) {
                        rc = lw_replay_f64(d, n, link, 2, mi, mj, h64, min64, 0, 1);
                        CHECK(rc == -1, "bad replay accepted n=%d", n);
                    }
                    mj[1] = keep;
                }
                rc = lw_oracle_f64(d64, n, link, -1, mi, mj, mh64, ms, 1, &done);
                CHECK(rc == 0 && done == n - 1, "f64 n=%d link=%d rc=%d", n, link, rc);
                rc = lw_oracle_f32(d, n, link, n / 2, mi, mj, mh, ms, 1, &done);
                CHECK(rc == 0 && done == (n > 1 ? (n / 2 < n - 1 ? n / 2 : n - 1) : 0), "truncated n=%d", n);
                rc = lw_oracle_f32(d, n, link, 0, NULL, NULL, NULL, NULL, 1, &done);
                CHECK(rc == 0 && done == 0, "zero merges n=%d", n);
            }
        }
        if (n > 1) {
            const float bad[3] = {NAN, INFINITY, 2.5353012e30f /* 2^101 */};
            for (int t = 0; t < 3; ++t) {
                float keep = d[n - 1];
                d[n - 1] = bad[t];  /* row 0, last column: strict upper triangle */
                int64_t done = -1;
                int rc = lw_oracle_f32(d, n, 1, -1, mi, mj, mh, ms, 1, &done);
                CHECK(rc == -2 && done == 0, "bad value %d accepted n=%d rc=%d", t, n, rc);
                d[n - 1] = keep;
            }
        }
        CHECK(lw_oracle_f32(d, n, 6, -1, mi, mj, mh, ms, 1, NULL) == -1, "bad linkage accepted");
        CHECK(lw_oracle_f32(d, 0, 1, -1, mi, mj, mh, ms, 1, NULL) == -1, "n=0 accepted");
        CHECK(lw_oracle_f32(NULL, n, 1, -1, mi, mj, mh, ms, 1, NULL) == -1, "NULL dist accepted");
        free(d); free(d64); free(mi); free(mj); free(ms); free(mh); free(mh64); free(h64); free(min64);
    }
    printf("ok\n");
    return 0;
}
