// hac_rmsd.hip -- the input producer: the n x n matrix of superposed RMSDs
// between n conformations of one chain (the paper's input is such a matrix,
// computed by a parallel RMSD step before the clustering: Section 2.1's
// protein example, Section 5.1).
//
// Two kernels:
//   k_rmsd_prep   one wave per conformation: centroid (fp64), centred
//                 coordinates rounded to fp32 into the tiled layout below,
//                 squared norm (fp64 sum of the rounded coordinates), input
//                 check.
//   k_rmsd_tiles  one 256-thread workgroup per 32 x 32 block of pairs on or
//                 above the diagonal; each wave owns a 16 x 16 pair tile and
//                 accumulates the nine cross-covariance sums
//                 M_pq(s, t) = sum_i a_p(s, i) * a_q(t, i) with nine fp32
//                 16x16x4 MFMA accumulators (four registers each), four atoms
//                 per instruction; lane l of every accumulator holds the same
//                 4 pairs, so each lane finishes its pairs in registers
//                 (hac_qcp.h, fp64) and writes the strict upper triangle
//                 (diagonal 0).  The small accumulator footprint leaves room
//                 for three waves per SIMD, so one wave's fp64 epilogue
//                 runs beside another's matrix instructions.
//
// Coordinate layout (device workspace): conformations in tiles of 16, atoms
// in groups of 4 (one MFMA's k), groups in chunks of kChunk = 4.  Within
// tile T and chunk C, coordinate p of atom h of group c = 4 g + j of
// conformation r of the tile is at (G = kChunk / 4 = 1, so g = 0)
//     coords[(T * chunks + C) * 3 * 64 * kChunk + (((p * G + g) * 4 + h) * 16 + r) * 4 + j]
// (zero for padding atoms and padding conformations).  MFMA lane l = 16 h + r
// needs, for groups 4 g .. 4 g + 3, the four floats j = 0..3 at one 16-byte
// aligned address: one 16-byte load per (p, g), consecutive lanes at
// consecutive addresses (1 KiB per wave and load), 3 G loads per operand and
// chunk at immediate offsets from one pointer per lane.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hac_qcp.h"
#include "hac_rmsd.h"

namespace hac {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kPad = 64;        // conformations are padded to a multiple of this
constexpr int kPairBlock = 32;  // conformations per workgroup block side
constexpr int kGroup = 4;       // atoms per matrix instruction
constexpr int kSuper = 8;       // pair blocks per super-block side (L2 reuse)
constexpr int kChunk = 4;       // atom groups per chunk; groups are padded to a multiple of it
constexpr int kTile = 16;       // conformations per tile (an MFMA operand's rows)
constexpr int kBlockFloats = kTile * kGroup;            // one (p, c) block
static_assert(kChunk % 4 == 0, "a lane loads four atom groups at once");
constexpr int kChunkFloats = 3 * kChunk * kBlockFloats;  // one chunk of a tile
constexpr float kMaxCoord = (float)kRmsdMaxCoord;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void k_rmsd_clear(uint32_t *status) {
    if (threadIdx.x == 0) *status = 0u;
}

// Offset of coordinate 0 of atom i of conformation s; coordinate p is at
// + p * kPlaneStep.
__device__ __forceinline__ size_t coord_at(int i, int s, int chunks) {
    const int k = i / kGroup, c = k % kChunk;
    return ((size_t)(s / kTile) * chunks + k / kChunk) * kChunkFloats +
           ((((c / 4) * kGroup + i % kGroup) * kTile + s % kTile) * 4 + c % 4);
}
constexpr int kPlaneStep = kChunk * kBlockFloats;  // between coordinates p and p + 1

__global__ __launch_bounds__(256) void k_rmsd_prep(const float *__restrict__ xyz, int n, int npad, int atoms,
                                                   int quads, float *__restrict__ planes, double *__restrict__ sq,
                                                   uint32_t *__restrict__ status) {
    const int lane = threadIdx.x & 63;
    const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (s >= npad) return;
    const int chunks = quads / kChunk;
    if (s >= n) {  // padding conformation: zeros
        for (int i = lane; i < kGroup * quads; i += 64) {
            const size_t o = coord_at(i, s, chunks);
            planes[o] = 0.0f;
            planes[o + kPlaneStep] = 0.0f;
            planes[o + 2 * kPlaneStep] = 0.0f;
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
    for (int i = lane; i < kGroup * quads; i += 64) {
        float u = 0.0f, v = 0.0f, w = 0.0f;
        if (i < atoms) {
            u = (float)((double)x[3 * i] - c0);
            v = (float)((double)x[3 * i + 1] - c1);
            w = (float)((double)x[3 * i + 2] - c2);
            g += (double)u * u + (double)v * v + (double)w * w;
        }
        const size_t o = coord_at(i, s, chunks);
        planes[o] = u;
        planes[o + kPlaneStep] = v;
        planes[o + 2 * kPlaneStep] = w;
    }
    g = wave_sum(g);
    if (lane == 0) sq[s] = g;
}

// Three waves per SIMD (at most 170 VGPRs, no spills): one wave's fp64
// epilogue and loads run beside the others' matrix instructions (measured
// 15.3 -> 13.6 ms at n = 32768, m = 128 against two waves).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_rmsd_tiles(const float *__restrict__ planes, const double *__restrict__ sq,
                                                    const uint32_t *__restrict__ status, int n, int npad, int atoms,
                                                    int quads, int64_t nblocks, float *__restrict__ out, int64_t ld) {
    if (*status != 0u) return;  // rejected input: the output stays untouched

    // Blocks are handed to the 8 XCDs round-robin; renumber them so that each
    // XCD takes one contiguous run of pair blocks.
    const int64_t bid = blockIdx.x;
    const int64_t q = nblocks / 8, r = nblocks % 8;
    const int64_t xcd = bid % 8, j = bid / 8;
    const int64_t idx = xcd * q + (xcd < r ? xcd : r) + j;
    // The run walks super-blocks of kSuper x kSuper pair blocks on or above
    // the diagonal (column-major: sb = st (st + 1) / 2 + ss), each one whole:
    // its 2 kSuper conformation tiles stay in the XCD's L2 while its
    // kSuper^2 blocks use them.  Blocks below the diagonal or past the last
    // conformation exit at once.
    const int64_t sb = idx / (kSuper * kSuper), within = idx % (kSuper * kSuper);
    int64_t st = (int64_t)((sqrt(8.0 * (double)sb + 1.0) - 1.0) * 0.5);
    while (st * (st + 1) / 2 > sb) --st;
    while ((st + 1) * (st + 2) / 2 <= sb) ++st;
    const int64_t ss = sb - st * (st + 1) / 2;
    const int64_t bs = ss * kSuper + within / kSuper, bt = st * kSuper + within % kSuper;
    if (bs > bt) return;

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int s0 = (int)bs * kPairBlock + (wave >> 1) * 16;
    const int t0 = (int)bt * kPairBlock + (wave & 1) * 16;
    if (s0 >= n || t0 >= n || s0 > t0 + 15) return;  // no pair of this tile is wanted

    const int rr = lane & 15, hh = lane >> 4;
    const int chunks = quads / kChunk;
    const float *pa = planes + (size_t)(s0 / kTile) * chunks * kChunkFloats + lane * 4;
    const float *pb = planes + (size_t)(t0 / kTile) * chunks * kChunkFloats + lane * 4;
    v4f acc[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) acc[u] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    // Two register buffers of kChunk atom groups, used in turn: the loads of
    // one are in flight while the matrix instructions consume the other (no
    // copies between them, so the wait before a chunk leaves the other
    // chunk's loads outstanding).  quads is a multiple of kChunk.
    float a0[3][kChunk], b0[3][kChunk], a1[3][kChunk], b1[3][kChunk];
    auto load = [&](int chunk, float (&xa)[3][kChunk], float (&xb)[3][kChunk]) {
        const float *qa = pa + (size_t)chunk * kChunkFloats;
        const float *qb = pb + (size_t)chunk * kChunkFloats;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
#pragma unroll
            for (int g = 0; g < kChunk / 4; ++g) {
                const float4 va = *reinterpret_cast<const float4 *>(qa + (p * (kChunk / 4) + g) * 256);
                const float4 vb = *reinterpret_cast<const float4 *>(qb + (p * (kChunk / 4) + g) * 256);
                xa[p][4 * g] = va.x;
                xa[p][4 * g + 1] = va.y;
                xa[p][4 * g + 2] = va.z;
                xa[p][4 * g + 3] = va.w;
                xb[p][4 * g] = vb.x;
                xb[p][4 * g + 1] = vb.y;
                xb[p][4 * g + 2] = vb.z;
                xb[p][4 * g + 3] = vb.w;
            }
        }
    };
    auto mma = [&](const float (&xa)[3][kChunk], const float (&xb)[3][kChunk]) {
#pragma unroll
        for (int c = 0; c < kChunk; ++c) {
#pragma unroll
            for (int p = 0; p < 3; ++p) {
#pragma unroll
                for (int qq = 0; qq < 3; ++qq)
                    acc[3 * p + qq] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[p][c], xb[qq][c], acc[3 * p + qq], 0, 0, 0);
            }
        }
    };
    load(0, a0, b0);
    for (int ch = 0; ch < chunks; ch += 2) {
        const bool second = ch + 1 < chunks;
        if (second) load(ch + 1, a1, b1);
        mma(a0, b0);
        if (!second) break;
        if (ch + 2 < chunks) load(ch + 2, a0, b0);
        mma(a1, b1);
    }
    // Accumulator element e of lane l: row 4 (l / 16) + e of the tile
    // (conformation s), column l % 16 (conformation t).
    const int t = t0 + rr;
    const double gt = t < n ? sq[t] : 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int s = s0 + 4 * hh + e;
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
    L.npad = (n + kPad - 1) / kPad * kPad;
    L.quads = ((atoms + kGroup - 1) / kGroup + kChunk - 1) / kChunk * kChunk;
    L.planes_bytes = (size_t)3 * L.quads * L.npad * kGroup * sizeof(float);
    L.sq_offset = L.planes_bytes;
    L.status_offset = L.sq_offset + (size_t)L.npad * sizeof(double);
    L.bytes = L.status_offset + 256;
    const int64_t side = L.npad / kPairBlock;
    const int64_t supers = (side + kSuper - 1) / kSuper;
    L.blocks = supers * (supers + 1) / 2 * kSuper * kSuper;
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
                       L.quads, planes, sq, status);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rmsd_tiles, dim3((unsigned)L.blocks), dim3(256), 0, stream, planes, sq, status, n, L.npad,
                       atoms, L.quads, L.blocks, out, (int64_t)n);
    return hipGetLastError();
}

}  // namespace hac
