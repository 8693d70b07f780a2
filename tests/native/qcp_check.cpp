// Host build of the RMSD producer's per-pair epilogue (hac_qcp.h): reads
// "atoms ga gb m0 .. m8" per line, prints lambda_max and the fp32 RMSD.
#include <cstdio>

#include "hac_qcp.h"

int main() {
    int atoms;
    double ga, gb, m[9];
    while (std::scanf("%d %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf", &atoms, &ga, &gb, &m[0], &m[1], &m[2],
                      &m[3], &m[4], &m[5], &m[6], &m[7], &m[8]) == 12) {
        const double lam = hac::qcp_lambda_max(m, ga, gb);
        const float r = hac::qcp_rmsd(m, ga, gb, atoms);
        std::printf("%.17g %.9g\n", lam, (double)r);
    }
    return 0;
}
