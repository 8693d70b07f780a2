/*
 * CPU oracle for Lance-Williams agglomerative clustering.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or constant with the
 * GPU library.
 *
 * What it computes (Section 4, "Lance-William Algorithm", steps 1-4, and
 * Table 1):
 *   start with n singleton clusters in slots 0..n-1;
 *   repeat n-1 times:
 *     1. find the smallest distance D[i][j] over pairs of live slots i < j
 *        (first strict '<' minimum in row-major order, i.e. the
 *        lexicographically smallest (D, i, j));
 *     2. merge j into i: slot i keeps the merged cluster, slot j is retired
 *        (Section 5.3, step 6: row/column i is reused, row/column j is marked
 *        not to be used again);
 *     3. for every other live slot k, recompute D[k][i] = D[i][k] with the
 *        Lance-Williams update of step 3 using the Table 1 coefficients;
 *     4. emit the merge record (i, j, height = D[i][j], size of i after merge).
 *
 * Two precisions:
 *   - lw_oracle_f32: every distance stored and updated in fp32 with the fixed
 *     operation order below (compile with -ffp-contract=off, no fast-math);
 *   - lw_oracle_f64: the same loop in fp64, used only for error bounds.
 *
 * Coefficients (Table 1) as evaluated here:
 *   single   : alpha_i = alpha_j = 1/2, beta = 0, gamma = -1/2.  In real
 *              arithmetic this is exactly min(D_ki, D_kj); evaluated as fminf,
 *              which is exact in fp32.
 *   complete : alpha_i = alpha_j = 1/2, beta = 0, gamma = +1/2  -> max, fmaxf.
 *   average  : alpha_i = n_i/(n_i+n_j), alpha_j = n_j/(n_i+n_j), beta=gamma=0.
 *              fp32: a_i, a_j are fp64 quotients rounded once to fp32;
 *              v = (a_i*D_ki) + (a_j*D_kj), each operation rounded.
 *   ward     : T = n_i+n_j+n_k; alpha_i = (n_i+n_k)/T, alpha_j = (n_j+n_k)/T,
 *              beta = -n_k/T, gamma = 0.  fp32: coefficients are fp64
 *              quotients rounded once to fp32;
 *              v = ((a_i*D_ki) + (a_j*D_kj)) + (b*D_ij).
 *   weighted : (Table 1 row "Weighted Average") alpha_i = alpha_j = 1/2,
 *              beta = gamma = 0.  fp32: v = (0.5*D_ki) + (0.5*D_kj).
 *   centroid : (Table 1 row "Centroid") alpha_i = n_i/(n_i+n_j),
 *              alpha_j = n_j/(n_i+n_j), beta = -n_i*n_j/(n_i+n_j)^2, gamma = 0.
 *              fp32: coefficients are fp64 quotients rounded once to fp32;
 *              v = ((a_i*D_ki) + (a_j*D_kj)) + (b*D_ij).  Heights need not
 *              increase and can be negative when the input is not a matrix
 *              of squared Euclidean distances.  Values stay finite: D_ij is
 *              the minimum over live pairs, so a negative minimum never
 *              grows in magnitude and one merge adds at most |D_ij|/4 to any
 *              entry; |D| stays below 2^100 * (1 + (n-1)/4).
 * A result equal to zero is stored as +0.
 *
 * Input: the strict upper triangle of the row-major n x n matrix is
 * authoritative (Section 5.2: only the upper half is needed); diagonal and
 * lower triangle are ignored.  Values must be finite with |x| <= 2^100;
 * -0 is read as +0.  The working copy keeps only that upper half too: the
 * distance between slots a != b lives at row min(a,b), column max(a,b).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_SINGLE = 0, OR_COMPLETE = 1, OR_AVERAGE = 2, OR_WARD = 3, OR_WEIGHTED = 4, OR_CENTROID = 5 };
enum { OR_OK = 0, OR_EINVAL = -1, OR_EINPUT = -2, OR_ENOMEM = -3, OR_EINTERNAL = -4 };
#define OR_MAX_LINK 5

#define OR_MAX_ABS 1.2676506002282294e30 /* 2^100 */

/* Index of the stored distance between slots a != b (upper triangle). */
#define UPPER(a, b) ((a) < (b) ? (a) * n + (b) : (b) * n + (a))

/* ---- fp32 Lance-Williams update (Section 4 step 3, Table 1) ------------ */
static float lw_f32(int link, float dki, float dkj, float dij,
                    int64_t ni, int64_t nj, int64_t nk)
{
    float v;
    if (link == OR_SINGLE) {
        v = fminf(dki, dkj);
    } else if (link == OR_COMPLETE) {
        v = fmaxf(dki, dkj);
    } else if (link == OR_AVERAGE) {
        double s = (double)(ni + nj);
        float ai = (float)((double)ni / s);
        float aj = (float)((double)nj / s);
        float t1 = ai * dki;
        float t2 = aj * dkj;
        v = t1 + t2;
    } else if (link == OR_WEIGHTED) {
        float t1 = 0.5f * dki;
        float t2 = 0.5f * dkj;
        v = t1 + t2;
    } else if (link == OR_CENTROID) {
        double s = (double)(ni + nj);
        float ai = (float)((double)ni / s);
        float aj = (float)((double)nj / s);
        float b = (float)(-((double)ni * (double)nj) / (s * s));
        float t1 = ai * dki;
        float t2 = aj * dkj;
        float t3 = b * dij;
        float u = t1 + t2;
        v = u + t3;
    } else { /* OR_WARD */
        double t = (double)(ni + nj + nk);
        float ai = (float)((double)(ni + nk) / t);
        float aj = (float)((double)(nj + nk) / t);
        float b = (float)(-(double)nk / t);
        float t1 = ai * dki;
        float t2 = aj * dkj;
        float t3 = b * dij;
        float u = t1 + t2;
        v = u + t3;
    }
    if (v == 0.0f) v = 0.0f; /* store zero as +0 */
    return v;
}

/* ---- fp64 Lance-Williams update: same expressions, no fp32 rounding ---- */
static double lw_f64(int link, double dki, double dkj, double dij,
                     int64_t ni, int64_t nj, int64_t nk)
{
    double v;
    if (link == OR_SINGLE) {
        v = fmin(dki, dkj);
    } else if (link == OR_COMPLETE) {
        v = fmax(dki, dkj);
    } else if (link == OR_AVERAGE) {
        double s = (double)(ni + nj);
        v = ((double)ni / s) * dki + ((double)nj / s) * dkj;
    } else if (link == OR_WEIGHTED) {
        v = 0.5 * dki + 0.5 * dkj;
    } else if (link == OR_CENTROID) {
        double s = (double)(ni + nj);
        v = (((double)ni / s) * dki + ((double)nj / s) * dkj) + (-((double)ni * (double)nj) / (s * s)) * dij;
    } else {
        double t = (double)(ni + nj + nk);
        v = (((double)(ni + nk) / t) * dki + ((double)(nj + nk) / t) * dkj)
            + (-(double)nk / t) * dij;
    }
    if (v == 0.0) v = 0.0;
    return v;
}

/*
 * One clustering run, written out once per precision (T = float or double).
 *
 * Step 1 follows the paper's parallel steps 1-4 (Section 5.3): each thread
 * ("processor") takes the local minimum over the rows it is handed, then the
 * global minimum is the smallest (value, i, j) among the local ones.  The
 * comparison is a total order, so this is the same pair a serial row-major
 * scan with strict '<' finds.
 */
static int better(double v, int64_t a, int64_t b, double bv, int64_t ba, int64_t bb)
{
    if (ba < 0) return 1;
    if (v != bv) return v < bv;
    if (a != ba) return a < ba;
    return b < bb;
}

int lw_oracle_f32(const float *dist, int64_t n, int link, int64_t max_merges,
                  int32_t *out_i, int32_t *out_j, float *out_h, int32_t *out_size,
                  int nthreads, int64_t *merges_done)
{
    if (merges_done) *merges_done = 0;
    if (n < 1 || !dist || link < 0 || link > OR_MAX_LINK) return OR_EINVAL;
    int64_t want = n - 1;
    if (max_merges >= 0 && max_merges < want) want = max_merges;
    if (want > 0 && (!out_i || !out_j || !out_h || !out_size)) return OR_EINVAL;
    for (int64_t a = 0; a < n; a++)
        for (int64_t b = a + 1; b < n; b++)
            if (!(fabs((double)dist[a * n + b]) <= OR_MAX_ABS)) return OR_EINPUT;
    float *w = (float *)malloc(sizeof(float) * (size_t)n * (size_t)n);
    int64_t *sz = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    unsigned char *alive = (unsigned char *)malloc((size_t)n);
    if (!w || !sz || !alive) { free(w); free(sz); free(alive); return OR_ENOMEM; }
    /* working copy of the upper triangle (the lower one is never used) */
    for (int64_t a = 0; a < n; a++) {
        for (int64_t b = a + 1; b < n; b++) {
            float x = dist[a * n + b];
            if (x == 0.0f) x = 0.0f; /* -0 -> +0 */
            w[a * n + b] = x;
        }
        sz[a] = 1;
        alive[a] = 1;
    }
    if (nthreads <= 0) nthreads = 1;
    for (int64_t s = 0; s < want; s++) {
        /* step 1: closest live pair, smallest (D, i, j) */
        float best = 0.0f; int64_t bi = -1, bj = -1;
        #pragma omp parallel num_threads(nthreads)
        {
            float lbest = 0.0f; int64_t li = -1, lj = -1;
            #pragma omp for schedule(dynamic, 16) nowait
            for (int64_t a = 0; a < n; a++) {
                if (!alive[a]) continue;
                const float *row = w + a * n;
                for (int64_t b = a + 1; b < n; b++)
                    if (alive[b] && better(row[b], a, b, lbest, li, lj)) {
                        lbest = row[b]; li = a; lj = b;
                    }
            }
            #pragma omp critical
            if (li >= 0 && better(lbest, li, lj, best, bi, bj)) {
                best = lbest; bi = li; bj = lj;
            }
        }
        if (bi < 0) { /* no live pair although >= 2 clusters remain */
            free(w); free(sz); free(alive);
            return OR_EINTERNAL;
        }
        int64_t i = bi, j = bj;
        float h = best;
        /* step 3: Lance-Williams update of row/column i */
        for (int64_t k = 0; k < n; k++) {
            if (!alive[k] || k == i || k == j) continue;
            float v = lw_f32(link, w[UPPER(k, i)], w[UPPER(k, j)], h, sz[i], sz[j], sz[k]);
            w[UPPER(k, i)] = v;
        }
        /* step 2 bookkeeping: j retired, i holds the merged cluster */
        alive[j] = 0;
        sz[i] += sz[j];
        /* step 4: output the level */
        out_i[s] = (int32_t)i; out_j[s] = (int32_t)j;
        out_h[s] = h; out_size[s] = (int32_t)sz[i];
        if (merges_done) *merges_done = s + 1;
    }
    free(w); free(sz); free(alive);
    return OR_OK;
}

int lw_oracle_f64(const double *dist, int64_t n, int link, int64_t max_merges,
                  int32_t *out_i, int32_t *out_j, double *out_h, int32_t *out_size,
                  int nthreads, int64_t *merges_done)
{
    if (merges_done) *merges_done = 0;
    if (n < 1 || !dist || link < 0 || link > OR_MAX_LINK) return OR_EINVAL;
    int64_t want = n - 1;
    if (max_merges >= 0 && max_merges < want) want = max_merges;
    if (want > 0 && (!out_i || !out_j || !out_h || !out_size)) return OR_EINVAL;
    for (int64_t a = 0; a < n; a++)
        for (int64_t b = a + 1; b < n; b++)
            if (!(fabs(dist[a * n + b]) <= OR_MAX_ABS)) return OR_EINPUT;
    double *w = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    int64_t *sz = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    unsigned char *alive = (unsigned char *)malloc((size_t)n);
    if (!w || !sz || !alive) { free(w); free(sz); free(alive); return OR_ENOMEM; }
    for (int64_t a = 0; a < n; a++) {
        for (int64_t b = a + 1; b < n; b++) {
            double x = dist[a * n + b];
            if (x == 0.0) x = 0.0;
            w[a * n + b] = x;
        }
        sz[a] = 1;
        alive[a] = 1;
    }
    if (nthreads <= 0) nthreads = 1;
    for (int64_t s = 0; s < want; s++) {
        double best = 0.0; int64_t bi = -1, bj = -1;
        #pragma omp parallel num_threads(nthreads)
        {
            double lbest = 0.0; int64_t li = -1, lj = -1;
            #pragma omp for schedule(dynamic, 16) nowait
            for (int64_t a = 0; a < n; a++) {
                if (!alive[a]) continue;
                const double *row = w + a * n;
                for (int64_t b = a + 1; b < n; b++)
                    if (alive[b] && better(row[b], a, b, lbest, li, lj)) {
                        lbest = row[b]; li = a; lj = b;
                    }
            }
            #pragma omp critical
            if (li >= 0 && better(lbest, li, lj, best, bi, bj)) {
                best = lbest; bi = li; bj = lj;
            }
        }
        if (bi < 0) { /* no live pair although >= 2 clusters remain */
            free(w); free(sz); free(alive);
            return OR_EINTERNAL;
        }
        int64_t i = bi, j = bj;
        double h = best;
        for (int64_t k = 0; k < n; k++) {
            if (!alive[k] || k == i || k == j) continue;
            double v = lw_f64(link, w[UPPER(k, i)], w[UPPER(k, j)], h, sz[i], sz[j], sz[k]);
            w[UPPER(k, i)] = v;
        }
        alive[j] = 0;
        sz[i] += sz[j];
        out_i[s] = (int32_t)i; out_j[s] = (int32_t)j;
        out_h[s] = h; out_size[s] = (int32_t)sz[i];
        if (merges_done) *merges_done = s + 1;
    }
    free(w); free(sz); free(alive);
    return OR_OK;
}

/*
 * Replay a given merge list in fp64 (checker, not an oracle of its own):
 * applies the listed merges with the fp64 update and reports, per merge,
 *   h64[s]  = fp64 distance of the listed pair at that moment, and
 *   min64[s] = fp64 minimum over all live pairs at that moment
 *              (computed only when s % opt_stride == 0, else NAN).
 * Returns OR_EINVAL if the list names a dead or out-of-range slot.
 */
int lw_replay_f64(const float *dist, int64_t n, int link, int64_t count,
                  const int32_t *mi, const int32_t *mj, double *h64,
                  double *min64, int64_t opt_stride, int nthreads)
{
    if (n < 1 || !dist || link < 0 || link > OR_MAX_LINK || count < 0 || count > n - 1)
        return OR_EINVAL;
    double *w = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    int64_t *sz = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    unsigned char *alive = (unsigned char *)malloc((size_t)n);
    if (!w || !sz || !alive) { free(w); free(sz); free(alive); return OR_ENOMEM; }
    for (int64_t a = 0; a < n; a++) {
        for (int64_t b = a + 1; b < n; b++) {
            double x = (double)dist[a * n + b];
            if (x == 0) x = 0;
            w[a * n + b] = x;
        }
        sz[a] = 1;
        alive[a] = 1;
    }
    if (nthreads <= 0) nthreads = 1;
    int rc = OR_OK;
    for (int64_t s = 0; s < count; s++) {
        int64_t i = mi[s], j = mj[s];
        if (i < 0 || j >= n || i >= j || !alive[i] || !alive[j]) { rc = OR_EINVAL; break; }
        h64[s] = w[i * n + j];
        min64[s] = NAN;
        if (opt_stride > 0 && s % opt_stride == 0) {
            double gmin = INFINITY;
            #pragma omp parallel for num_threads(nthreads) reduction(min:gmin) schedule(dynamic, 16)
            for (int64_t a = 0; a < n; a++) {
                if (!alive[a]) continue;
                for (int64_t b = a + 1; b < n; b++)
                    if (alive[b] && w[a * n + b] < gmin) gmin = w[a * n + b];
            }
            min64[s] = gmin;
        }
        double h = w[i * n + j];
        for (int64_t k = 0; k < n; k++) {
            if (!alive[k] || k == i || k == j) continue;
            double v = lw_f64(link, w[UPPER(k, i)], w[UPPER(k, j)], h, sz[i], sz[j], sz[k]);
            w[UPPER(k, i)] = v;
        }
        alive[j] = 0;
        sz[i] += sz[j];
    }
    free(w); free(sz); free(alive);
    return rc;
}
