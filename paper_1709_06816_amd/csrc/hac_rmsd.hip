// hac_rmsd.hip -- the input producer: the n x n matrix of superposed RMSDs
// between n conformations of one chain (the paper's input is such a matrix,
// computed by a parallel RMSD step before the clustering: Section 2.1's
// protein example, Section 5.1).
//
// Two kernels:
//   k_rmsd_prep   one wave per conformation: centroid (fp64), centred
//                 coordinates rounded to fp32 into three coordinate planes
//                 laid out for the matrix cores, squared norm (fp64 sum of the
//                 rounded coordinates), input check.
//   k_rmsd_tiles  one 256-thread workgroup per 64 x 64 block of pairs on or
//                 above the diagonal; each wave owns a 32 x 32 pair tile and
//                 accumulates the nine cross-covariance sums
//                 M_pq(s, t) = sum_i a_p(s, i) * a_q(t, i) with nine fp32
//                 32x32x2 MFMA accumulators, two atoms per instruction; lane
//                 l of every accumulator holds the same 16 pairs, so each lane
//                 finishes its pairs in registers (hac_qcp.h, fp64) and
//                 writes the strict upper triangle (diagonal 0).
//
// Plane layout (device workspace): planes[((p * half + k) * npad + s) * 2 + h]
// is coordinate p of atom 2k + h of conformation s (zero for the padding atom
// of odd m and for the padding conformations s >= n), npad = n rounded up to
// 64.  For the MFMA operand, lanes 0-31 read atom 2k and lanes 32-63 atom
// 2k + 1 of 32 consecutive conformations: 256 contiguous bytes per plane.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hac_qcp.h"
#include "hac_rmsd.h"

namespace hac {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kPairBlock = 64;  // conformations per workgroup block side
constexpr float kMaxCoord = (float)kRmsdMaxCoord;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void k_rmsd_clear(uint32_t *status) {
    if (threadIdx.x == 0) *status = 0u;
}

__global__ __launch_bounds__(256) void k_rmsd_prep(const float *__restrict__ xyz, int n, int npad, int atoms,
                                                   int half, float *__restrict__ planes, double *__restrict__ sq,
                                                   uint32_t *__restrict__ status) {
    const int lane = threadIdx.x & 63;
    const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (s >= npad) return;
    const size_t pstride = (size_t)half * npad * 2;
    if (s >= n) {  // padding conformation: zeros
        for (int i = lane; i < 2 * half; i += 64) {
            const size_t o = ((size_t)(i >> 1) * npad + s) * 2 + (i & 1);
            planes[o] = 0.0f;
            planes[o + pstride] = 0.0f;
            planes[o + 2 * pstride] = 0.0f;
        }
        if (lane == 0) sq[s] = 0.0;
        return;
    }
    const float *x = xyz + (size_t)s * atoms * 3;
    double c0 = 0.0, c1 = 0.0, c2 = 0.0;
    bool bad = false;
    for (int i = lane; i < atoms; i += 64) {
        const float u = x[3 * i], v = x[3 * i + 1], w = x[3 * i + 2];
        bad |= !(fabsf(u) <= kMaxCoord) || !(fabsf(v) <= kMaxCoord) || !(fabsf(w) <= kMaxCoord);
        c0 += u;
        c1 += v;
        c2 += w;
    }
    if (__ballot(bad) != 0ull) {
        if (lane == 0) atomicOr(status, 1u);
        return;
    }
    c0 = wave_sum(c0) / atoms;
    c1 = wave_sum(c1) / atoms;
    c2 = wave_sum(c2) / atoms;
    double g = 0.0;
    for (int i = lane; i < 2 * half; i += 64) {
        float u = 0.0f, v = 0.0f, w = 0.0f;
        if (i < atoms) {
            u = (float)((double)x[3 * i] - c0);
            v = (float)((double)x[3 * i + 1] - c1);
            w = (float)((double)x[3 * i + 2] - c2);
            g += (double)u * u + (double)v * v + (double)w * w;
        }
        const size_t o = ((size_t)(i >> 1) * npad + s) * 2 + (i & 1);
        planes[o] = u;
        planes[o + pstride] = v;
        planes[o + 2 * pstride] = w;
    }
    g = wave_sum(g);
    if (lane == 0) sq[s] = g;
}

__global__ __launch_bounds__(256) void k_rmsd_tiles(const float *__restrict__ planes, const double *__restrict__ sq,
                                                    const uint32_t *__restrict__ status, int n, int npad, int atoms,
                                                    int half, int64_t nblocks, float *__restrict__ out, int64_t ld) {
    if (*status != 0u) return;  // rejected input: the output stays untouched

    // Blocks are handed to the 8 XCDs round-robin; renumber them so that each
    // XCD takes one contiguous run of pair blocks (shared conformations stay
    // in that XCD's L2).
    const int64_t bid = blockIdx.x;
    const int64_t q = nblocks / 8, r = nblocks % 8;
    const int64_t xcd = bid % 8, j = bid / 8;
    const int64_t idx = xcd * q + (xcd < r ? xcd : r) + j;
    // Column-major enumeration of the upper triangle: idx = bt (bt + 1) / 2 + bs.
    int64_t bt = (int64_t)((sqrt(8.0 * (double)idx + 1.0) - 1.0) * 0.5);
    while (bt * (bt + 1) / 2 > idx) --bt;
    while ((bt + 1) * (bt + 2) / 2 <= idx) ++bt;
    const int64_t bs = idx - bt * (bt + 1) / 2;

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int s0 = (int)bs * kPairBlock + (wave >> 1) * 32;
    const int t0 = (int)bt * kPairBlock + (wave & 1) * 32;
    if (s0 >= n || t0 >= n || s0 > t0 + 31) return;  // no pair of this tile is wanted

    const int rr = lane & 31, hh = lane >> 5;
    const size_t pstride = (size_t)half * npad * 2, kstride = (size_t)npad * 2;
    const float *pa = planes + (size_t)(s0 + rr) * 2 + hh;
    const float *pb = planes + (size_t)(t0 + rr) * 2 + hh;
    v16f acc[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) acc[u] = v16f{0.0f};
    // Atom pairs in chunks of kChunk: the next chunk's loads are issued
    // before the current chunk's 9 * kChunk matrix instructions.
    constexpr int kChunk = 4;
    float ca[3][kChunk], cb[3][kChunk], na[3][kChunk], nb[3][kChunk];
    auto load = [&](int k0, float (&xa)[3][kChunk], float (&xb)[3][kChunk]) {
#pragma unroll
        for (int c = 0; c < kChunk; ++c) {
            const bool in = k0 + c < half;
            const size_t o = (size_t)(in ? k0 + c : 0) * kstride;
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                xa[p][c] = in ? pa[o + p * pstride] : 0.0f;
                xb[p][c] = in ? pb[o + p * pstride] : 0.0f;
            }
        }
    };
    load(0, ca, cb);
    for (int k0 = 0; k0 < half; k0 += kChunk) {
        if (k0 + kChunk < half) load(k0 + kChunk, na, nb);
#pragma unroll
        for (int c = 0; c < kChunk; ++c) {
#pragma unroll
            for (int p = 0; p < 3; ++p) {
#pragma unroll
                for (int qq = 0; qq < 3; ++qq)
                    acc[3 * p + qq] = __builtin_amdgcn_mfma_f32_32x32x2f32(ca[p][c], cb[qq][c], acc[3 * p + qq], 0, 0, 0);
            }
        }
#pragma unroll
        for (int p = 0; p < 3; ++p) {
#pragma unroll
            for (int c = 0; c < kChunk; ++c) {
                ca[p][c] = na[p][c];
                cb[p][c] = nb[p][c];
            }
        }
    }
    // Accumulator element e of lane l: row 8 (e / 4) + 4 (l / 32) + e % 4 of
    // the tile (conformation s), column l % 32 (conformation t).
    const int t = t0 + rr;
    const double gt = t < n ? sq[t] : 0.0;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int s = s0 + 8 * (e >> 2) + 4 * hh + (e & 3);
        if (s < n && t < n && s <= t) {
            float v = 0.0f;
            if (s != t) {
                const double m9[9] = {acc[0][e], acc[1][e], acc[2][e], acc[3][e], acc[4][e],
                                      acc[5][e], acc[6][e], acc[7][e], acc[8][e]};
                v = qcp_rmsd(m9, sq[s], gt, atoms);
            }
            out[(size_t)s * ld + t] = v;
        }
    }
}

}  // namespace

RmsdLayout rmsd_layout(int n, int atoms) {
    RmsdLayout L;
    L.npad = (n + kPairBlock - 1) / kPairBlock * kPairBlock;
    L.half = (atoms + 1) / 2;
    L.planes_bytes = (size_t)3 * L.half * L.npad * 2 * sizeof(float);
    L.sq_offset = L.planes_bytes;
    L.status_offset = L.sq_offset + (size_t)L.npad * sizeof(double);
    L.bytes = L.status_offset + 256;
    const int64_t side = L.npad / kPairBlock;
    L.blocks = side * (side + 1) / 2;
    return L;
}

hipError_t launch_rmsd(const float *xyz, int n, int atoms, float *out, void *ws, hipStream_t stream) {
    const RmsdLayout L = rmsd_layout(n, atoms);
    char *base = static_cast<char *>(ws);
    float *planes = reinterpret_cast<float *>(base);
    double *sq = reinterpret_cast<double *>(base + L.sq_offset);
    uint32_t *status = reinterpret_cast<uint32_t *>(base + L.status_offset);
    hipLaunchKernelGGL(k_rmsd_clear, dim3(1), dim3(64), 0, stream, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rmsd_prep, dim3((unsigned)(L.npad / 4)), dim3(256), 0, stream, xyz, n, L.npad, atoms,
                       L.half, planes, sq, status);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rmsd_tiles, dim3((unsigned)L.blocks), dim3(256), 0, stream, planes, sq, status, n, L.npad,
                       atoms, L.half, L.blocks, out, (int64_t)n);
    return hipGetLastError();
}

}  // namespace hac
