// hac_qcp.h -- superposed RMSD of one pair of conformations from its 3 x 3
// cross-covariance, in fp64: the per-pair epilogue of the RMSD producer.
//
// For centred conformations A, B of m atoms with squared norms ga, gb and
// cross-covariance M[p][q] = sum_i a_ip * b_iq, the best proper rotation
// attains lambda_max, the largest eigenvalue of the symmetric traceless 4 x 4
// quaternion key matrix K(M) (Horn, J. Opt. Soc. Am. A 4 (1987)), and
//     RMSD^2 = (ga + gb - 2 * lambda_max) / m.
// lambda_max is the largest root of det(K - x I) = x^4 + c2 x^2 + c1 x + c0,
// with c2 = -2 |M|_F^2, c1 = -8 det M and c0 = det K, found by Newton's
// method from x0 = (ga + gb) / 2, which bounds lambda_max from above (the
// quaternion characteristic polynomial method of Theobald, Acta Cryst. A 61
// (2005)).  Above its largest root the quartic is increasing and convex, so
// the iterates decrease monotonically to it; multiple roots (collinear or
// planar conformations) converge linearly, hence the iteration cap.
//
// Shared by the device kernel and a host-side check, so it is plain C++
// marked for both sides.
#ifndef HAC_QCP_H
#define HAC_QCP_H

#include <math.h>

#ifdef __HIPCC__
#define HAC_QCP_FN __host__ __device__ inline
#else
#define HAC_QCP_FN inline
#endif

namespace hac {

constexpr int kQcpMaxIter = 128;

// m9: M row-major (Sxx, Sxy, Sxz, Syx, Syy, Syz, Szx, Szy, Szz).
HAC_QCP_FN double qcp_lambda_max(const double *m9, double ga, double gb) {
    const double sxx = m9[0], sxy = m9[1], sxz = m9[2];
    const double syx = m9[3], syy = m9[4], syz = m9[5];
    const double szx = m9[6], szy = m9[7], szz = m9[8];
    // K(M), symmetric
    const double k00 = sxx + syy + szz, k01 = syz - szy, k02 = szx - sxz, k03 = sxy - syx;
    const double k11 = sxx - syy - szz, k12 = sxy + syx, k13 = szx + sxz;
    const double k22 = -sxx + syy - szz, k23 = syz + szy;
    const double k33 = -sxx - syy + szz;
    // det K by Laplace expansion along rows 0-1 (2 x 2 minors of rows 0-1
    // times complementary minors of rows 2-3)
    const double a01 = k00 * k11 - k01 * k01, a02 = k00 * k12 - k02 * k01, a03 = k00 * k13 - k03 * k01;
    const double a12 = k01 * k12 - k02 * k11, a13 = k01 * k13 - k03 * k11, a23 = k02 * k13 - k03 * k12;
    const double b01 = k02 * k13 - k12 * k03, b02 = k02 * k23 - k22 * k03, b03 = k02 * k33 - k23 * k03;
    const double b12 = k12 * k23 - k22 * k13, b13 = k12 * k33 - k23 * k13, b23 = k22 * k33 - k23 * k23;
    const double c0 = a01 * b23 - a02 * b13 + a03 * b12 + a12 * b03 - a13 * b02 + a23 * b01;
    const double detm = sxx * (syy * szz - syz * szy) - sxy * (syx * szz - syz * szx) + sxz * (syx * szy - syy * szx);
    const double c1 = -8.0 * detm;
    const double c2 = -2.0 * (sxx * sxx + sxy * sxy + sxz * sxz + syx * syx + syy * syy + syz * syz +
                              szx * szx + szy * szy + szz * szz);
    double x = 0.5 * (ga + gb);
    for (int it = 0; it < kQcpMaxIter; ++it) {
        const double x2 = x * x;
        const double p = (x2 + c2) * x2 + c1 * x + c0;
        const double dp = (4.0 * x2 + 2.0 * c2) * x + c1;
        if (!(dp > 0.0)) break;  // at (or, by rounding, just past) the root
        const double d = p / dp;
        x -= d;
        if (fabs(d) <= 1e-11 * fabs(x)) break;
    }
    return x;
}

// Superposed RMSD of the pair, rounded once to fp32.
HAC_QCP_FN float qcp_rmsd(const double *m9, double ga, double gb, int atoms) {
    const double lam = qcp_lambda_max(m9, ga, gb);
    const double r2 = (ga + gb - 2.0 * lam) / (double)atoms;
    return r2 > 0.0 ? (float)sqrt(r2) : 0.0f;
}

}  // namespace hac

#endif  // HAC_QCP_H
