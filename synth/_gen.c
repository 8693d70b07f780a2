/*
 * Fixed-order fp64 arithmetic for the synthetic inputs.
 *
 * Input generation only: points to distance matrices, random rotations.  No
 * clustering arithmetic lives here.  Every output element is computed by the
 * same sequence of correctly rounded IEEE-754 double operations (gcc -O2
 * -ffp-contract=off, no fast-math, sums taken in index order), so a matrix
 * is bit-identical on any x86-64 host whatever its vector units or thread
 * count -- unlike a BLAS product, whose summation order depends on the CPU.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

/* Squared norm of each point, summed over d = 0 .. dim-1 in order. */
static void sq_norms(const double *x, int64_t n, int dim, double *sq)
{
    #pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < n; a++) {
        const double *p = x + a * dim;
        double s = 0.0;
        for (int d = 0; d < dim; d++) {
            double t = p[d] * p[d];
            s = s + t;
        }
        sq[a] = s;
    }
}

/* sqrt(max(0, |x_a|^2 + |x_b|^2 - 2 x_a.x_b)) in fp64, the dot product summed
 * over d in order, evaluated as ((-2 g) + sq_a) + sq_b. */
static inline double gram_dist(const double *pa, const double *pb, int dim, double sa, double sb)
{
    double g = 0.0;
    for (int d = 0; d < dim; d++) {
        double t = pa[d] * pb[d];
        g = g + t;
    }
    double v = -2.0 * g;
    v = v + sa;
    v = v + sb;
    if (!(v > 0.0)) v = 0.0;
    return sqrt(v);
}

/*
 * Full symmetric n x n fp32 Euclidean matrix of fp64 points x (n x dim,
 * row-major).  The strict upper triangle is computed, optionally multiplied
 * by scale_to / (largest distance) and rounded half-to-even to round_dec
 * decimals (round_dec < 0: no rounding), rounded once to fp32 and mirrored;
 * the diagonal is 0.  Returns 0, or -1 if scratch memory is missing.
 */
int synth_euclid(const double *x, int64_t n, int dim, float *out, double scale_to, int round_dec)
{
    double *sq = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!sq) return -1;
    sq_norms(x, n, dim, sq);
    double factor = 1.0;
    int scale = scale_to > 0.0;
    if (scale) {
        double dmax = 0.0;
        #pragma omp parallel for schedule(dynamic, 16) reduction(max : dmax)
        for (int64_t a = 0; a < n; a++)
            for (int64_t b = a + 1; b < n; b++) {
                double v = gram_dist(x + a * dim, x + b * dim, dim, sq[a], sq[b]);
                if (v > dmax) dmax = v;
            }
        factor = dmax > 0.0 ? scale_to / dmax : 1.0;
    }
    const double p = round_dec >= 0 ? pow(10.0, (double)round_dec) : 1.0;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t a = 0; a < n; a++) {
        out[a * n + a] = 0.0f;
        for (int64_t b = a + 1; b < n; b++) {
            double v = gram_dist(x + a * dim, x + b * dim, dim, sq[a], sq[b]);
            if (scale) v = v * factor;
            if (round_dec >= 0) {
                v = v * p;
                v = nearbyint(v); /* default rounding mode: half to even */
                v = v / p;
            }
            out[a * n + b] = (float)v;
        }
    }
    /* mirror, in tiles so that the column writes stay in cache */
    const int64_t T = 64;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t bb = 0; bb < n; bb += T)
        for (int64_t aa = 0; aa <= bb; aa += T)
            for (int64_t b = bb; b < bb + T && b < n; b++)
                for (int64_t a = aa; a < aa + T && a < b; a++)
                    out[b * n + a] = out[a * n + b];
    free(sq);
    return 0;
}

/*
 * Orthonormalise the columns of the dim x dim matrix g (row-major) by
 * modified Gram-Schmidt, in column order, into q: the Q factor of g = QR with
 * a positive diagonal of R.  Returns -1 if g is numerically singular.
 */
int synth_orthonormal(const double *g, int dim, double *q)
{
    for (int i = 0; i < dim * dim; i++) q[i] = g[i];
    for (int j = 0; j < dim; j++) {
        for (int k = 0; k < j; k++) {
            double r = 0.0;
            for (int i = 0; i < dim; i++) {
                double t = q[i * dim + k] * q[i * dim + j];
                r = r + t;
            }
            for (int i = 0; i < dim; i++) {
                double t = r * q[i * dim + k];
                q[i * dim + j] = q[i * dim + j] - t;
            }
        }
        double s = 0.0;
        for (int i = 0; i < dim; i++) {
            double t = q[i * dim + j] * q[i * dim + j];
            s = s + t;
        }
        double nrm = sqrt(s);
        if (!(nrm > 0.0)) return -1;
        for (int i = 0; i < dim; i++) q[i * dim + j] = q[i * dim + j] / nrm;
    }
    return 0;
}

/*
 * Anisotropic cluster points: pts[a][e] = c[e] + sum_f (z[a][f] * s[f]) q[e][f]
 * (sum over f in order) for the `count` points whose rows are listed in
 * rows[], with one cluster's centre c (dim), scales s (dim) and rotation q
 * (dim x dim, row-major).  z and pts are n x dim.
 */
void synth_rotate(const double *z, const int64_t *rows, int64_t count, int dim, const double *c,
                  const double *s, const double *q, double *pts)
{
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < count; r++) {
        const int64_t a = rows[r];
        for (int e = 0; e < dim; e++) {
            double acc = 0.0;
            for (int f = 0; f < dim; f++) {
                double zs = z[a * dim + f] * s[f];
                double t = zs * q[e * dim + f];
                acc = acc + t;
            }
            pts[a * dim + e] = c[e] + acc;
        }
    }
}
