// Scan engine: the paper's own closest-pair step (Section 5.3 step 1) -- a
// scan of the whole live upper triangle before every merge -- spread over
// every CU of the GPU.  Same merge list as every other path (Section 4, steps
// 1-4; lexicographic ties; Table 1 updates).
//
// One grid barrier per merge.  After it every workgroup reduces the G
// published candidates to the merge (i, j) and then, for merge s:
//   update  the Lance-Williams update of row and column i, one column per
//           thread over the whole grid; every new entry's key (v, min, max)
//           is folded into the workgroup's candidate for merge s+1;
//   scan    its share of the live upper triangle, without row and column i
//           (their new entries are the update's keys) and without j (retired),
//           folded into the same candidate, which is then published.
// Nothing the scan of merge s reads is written during merge s, and what the
// update writes is read only after the next barrier.
//
// Layout: the live items are kept compact.  The working matrix is copied at
// the start into a spare buffer with its leading dimension padded to a
// multiple of 4 (16-byte aligned rows), and whenever fewer than ~90% of the
// current width are live the live rows and columns are copied, in order,
// into the other buffer (an extra grid barrier on each side).  Keys use the
// compact indices, whose order is the slots' order, so ties resolve as on
// the original slots; records name the original slots (idx[]).  The upper
// triangle is cut into units of 2048 columns of one row (float4 aligned),
// balanced over the workgroups; a wave loads a unit's 8 KB at once.
#include <hip/hip_runtime.h>

#include "hac_dev.h"
#include "hac_scan.h"

namespace hac {
namespace {

constexpr uint64_t kNone = ~0ull;
constexpr int B = kScanBlock;
constexpr int W = B / 64;
constexpr int kSegF4 = 8;                // 16-byte loads per lane per unit
constexpr int kSeg = 64 * 4 * kSegF4;    // columns per unit
constexpr int kCompactNum = 9, kCompactDen = 10;  // compact below 9/10 live
constexpr int kMinCompactW = 64;

__shared__ uint64_t s_red[W];
__shared__ uint64_t s_cand;
__shared__ int s_row0, s_k0;

__device__ uint64_t block_min(uint64_t v) {
    v = wave_min(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) s_red[wv] = v;
    __syncthreads();
    uint64_t r = s_red[0];
#pragma unroll
    for (int q = 1; q < W; ++q) r = umin64(r, s_red[q]);
    return r;
}

__device__ unsigned long long block_sum(unsigned long long v) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) s_red[wv] = v;
    __syncthreads();
    unsigned long long r = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) r += s_red[q];
    return r;
}

// Fold every lane's v into s_cand (one LDS atomic per wave).
__device__ void fold(uint64_t v) {
    v = wave_min(v);
    if ((threadIdx.x & 63) == 0 && v != kNone) atomicMin(reinterpret_cast<unsigned long long *>(&s_cand), v);
}

struct Lds {
    uint16_t *size1;  // size - 1 of every compact slot
    uint32_t *live;   // live bitmask of the compact slots
    uint32_t *wpre;   // live slots before each mask word (compaction)
};

__device__ __forceinline__ bool live_at(const Lds &L, int c) { return (L.live[c >> 5] >> (c & 31)) & 1u; }

// Compact index of live slot c (slots before it that are live).
__device__ __forceinline__ int new_index(const Lds &L, int c) {
    return (int)L.wpre[c >> 5] + __popc(L.live[c >> 5] & ((1u << (c & 31)) - 1u));
}

// Units of row r (0 <= r <= w-2) of a w-wide compact matrix: its columns
// from 4*floor((r+1)/4) to w-1 in pieces of kSeg.
__device__ __forceinline__ int row_units(int r, int w) {
    const int cs = ((r + 1) >> 2) << 2;
    return (w - cs + kSeg - 1) / kSeg;
}

struct Part {
    int u0, u1;  // this workgroup's units [u0, u1)
};

// Split the units of a w-wide matrix evenly over the G workgroups; leaves
// the row and in-row unit of u0 in s_row0 / s_k0.
__device__ Part partition(int w, int G, int g) {
    // Units per thread's block of rows, then an exclusive block scan.
    const int rows = w - 1;
    const int per = (rows + B - 1) / B;
    const int ra = min(rows, (int)threadIdx.x * per), rb = min(rows, ra + per);
    unsigned long long mine = 0;
    for (int r = ra; r < rb; ++r) mine += row_units(r, w);
    const unsigned long long total = block_sum(mine);
    // Exclusive prefix of `mine` over the threads (simple two-level scan).
    __shared__ unsigned long long s_pre[B];
    s_pre[threadIdx.x] = mine;
    __syncthreads();
    for (int d = 1; d < B; d <<= 1) {
        const unsigned long long add = threadIdx.x >= (unsigned)d ? s_pre[threadIdx.x - d] : 0ull;
        __syncthreads();
        s_pre[threadIdx.x] += add;
        __syncthreads();
    }
    const unsigned long long before = s_pre[threadIdx.x] - mine;
    Part p;
    p.u0 = (int)(total * (unsigned long long)g / (unsigned long long)G);
    p.u1 = (int)(total * (unsigned long long)(g + 1) / (unsigned long long)G);
    if (threadIdx.x == 0) {
        s_row0 = rows;
        s_k0 = 0;
    }
    __syncthreads();
    if ((unsigned long long)p.u0 >= before && (unsigned long long)p.u0 < before + mine) {
        unsigned long long acc = before;
        for (int r = ra; r < rb; ++r) {
            const int ur = row_units(r, w);
            if ((unsigned long long)p.u0 < acc + ur) {
                s_row0 = r;
                s_k0 = (int)((unsigned long long)p.u0 - acc);
                break;
            }
            acc += ur;
        }
    }
    __syncthreads();
    return p;
}

__device__ __forceinline__ void advance(int &r, int &k, int w) {
    while (r < w - 1 && k >= row_units(r, w)) {
        k -= row_units(r, w);
        ++r;
    }
}

// This wave's part of the scan of the live upper triangle without row and
// column `skip`, folded into s_cand.
__device__ void scan_units(const float *__restrict__ C, int w, int ld, const Lds &L, const Part &P, int skip,
                           unsigned long long &elems) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int r = s_row0, k = s_k0 + wv;
    advance(r, k, w);
    uint64_t best = kNone;
    for (int u = P.u0 + wv; u < P.u1 && r < w - 1; u += W) {
        if (live_at(L, r) && r != skip) {
            const int c0 = (((r + 1) >> 2) << 2) + k * kSeg;
            const float *row = C + (size_t)r * ld;
            float4 x[kSegF4];
#pragma unroll
            for (int f = 0; f < kSegF4; ++f) {
                const int c = c0 + 4 * (f * 64 + lane);
                x[f] = c < w ? *reinterpret_cast<const float4 *>(row + c) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int f = 0; f < kSegF4; ++f) {
                const int c = c0 + 4 * (f * 64 + lane);
                if (c >= w) continue;
                uint32_t m = (L.live[c >> 5] >> (c & 31)) & 0xFu;
                if (c + 4 > w) m &= (1u << (w - c)) - 1u;
                const int below = r + 1 - c;  // columns <= r
                if (below > 0) m &= below >= 4 ? 0u : (0xFu << below) & 0xFu;
                if ((skip >> 2) == (c >> 2)) m &= ~(1u << (skip & 3));
                elems += __popc(m);
                const float v[4] = {x[f].x, x[f].y, x[f].z, x[f].w};
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if ((m >> t) & 1u)
                        best = umin64(best, ((uint64_t)ord32(v[t]) << 32) | ((uint64_t)r << 16) | (uint64_t)(c + t));
            }
        }
        k += W;
        advance(r, k, w);
    }
    fold(best);
}

struct Args {
    float *buf[2];          // working matrix (leading dimension n), spare
    int n, link, flags;
    const uint32_t *status;
    Control *ctl;
    ScanCtl *sc;
    uint64_t *cand;         // 2 x G published candidates (by merge parity)
    int32_t *idx;           // 2 x n original slot of each compact index
    hac_merge *out;
    uint64_t timeout;
};

// Copy the live rows and columns of `src` (w wide, leading dimension ld) in
// order into `dst` (leading dimension nld); idx goes along.  Every live slot
// c moves to new_index(c); L.wpre must be up to date.
__device__ void compact_copy(const float *__restrict__ src, int w, int ld, float *__restrict__ dst, int nld,
                             const int32_t *idx_src, int32_t *idx_dst, const Lds &L) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int gw = (int)blockIdx.x * W + wv, NW = (int)gridDim.x * W;
    for (int r = gw; r < w; r += NW) {
        if (!live_at(L, r)) continue;
        const int a = new_index(L, r);
        if (lane == 0) idx_dst[a] = idx_src[r];
        const float *sr = src + (size_t)r * ld;
        float *dr = dst + (size_t)a * nld;
        for (int c0 = 0; c0 < w; c0 += 64 * 8) {
            float x[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int c = c0 + t * 64 + lane;
                x[t] = c < w ? sr[c] : 0.0f;
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int c = c0 + t * 64 + lane;
                if (c < w && live_at(L, c)) dr[new_index(L, c)] = x[t];
            }
        }
    }
}

// Word prefix of the live mask (live slots before each word), and the live
// count, for a w-wide mask.
__device__ int live_prefix(const Lds &L, int w) {
    const int nw = (w + 31) >> 5;
    __shared__ uint32_t s_tot;
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int q = 0; q < nw; ++q) {
            L.wpre[q] = acc;
            acc += __popc(L.live[q]);
        }
        s_tot = acc;
    }
    __syncthreads();
    return (int)s_tot;
}

// Move the LDS sizes of the live slots to their compact indices, in place
// (a slot never moves up, so chunk by chunk, reading a whole chunk before
// writing it, never overwrites an entry still to be read).
__device__ void compact_sizes(const Lds &L, int w) {
    for (int c0 = 0; c0 < w; c0 += B) {
        const int c = c0 + (int)threadIdx.x;
        const bool mv = c < w && live_at(L, c);
        const uint16_t v = mv ? L.size1[c] : 0;
        const int to = mv ? new_index(L, c) : 0;
        __syncthreads();
        if (mv) L.size1[to] = v;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan(Args A) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int n = A.n, link = A.link, G = (int)gridDim.x, g = (int)blockIdx.x, tid = (int)threadIdx.x;
    if (__hip_atomic_load(A.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrInput) return;
    const int nwords = (n + 31) >> 5;
    Lds L;
    L.size1 = reinterpret_cast<uint16_t *>(smem);
    L.live = reinterpret_cast<uint32_t *>(smem + (((size_t)n * 2 + 15) & ~(size_t)15));
    L.wpre = L.live + nwords;
    unsigned long long st_scan = 0, st_upd = 0;
    uint32_t gen = 0;
    auto sync = [&]() {
        return grid_sync(&A.sc->bar, &A.sc->abort, &A.ctl->error, kErrTimeout, gen, (uint32_t)G, A.timeout,
                         (A.flags & kFlagStall) && g == 0 && gen == 0);
    };

    // Start: everything live, sizes 1, identity slots; copy into the spare
    // buffer with a padded leading dimension.
    for (int q = tid; q < nwords; q += B) {
        const int rem = n - q * 32;
        L.live[q] = rem >= 32 ? 0xFFFFFFFFu : ((1u << rem) - 1u);
    }
    for (int k = tid; k < n; k += B) L.size1[k] = 0;
    for (int k = g * B + tid; k < n; k += G * B) A.idx[k] = k;
    __syncthreads();
    int w = n, ld = n, cur = 0, m = live_prefix(L, n);
    if (!sync()) return;
    int nld = (n + 3) & ~3;
    compact_copy(A.buf[0], w, ld, A.buf[1], nld, A.idx, A.idx + n, L);
    if (!sync()) return;
    cur = 1;
    ld = nld;
    const int32_t *idx = A.idx + n;
    int idx_half = 1;

    // First candidate: the whole upper triangle.
    Part P = partition(w, G, g);
    if (tid == 0) s_cand = kNone;
    __syncthreads();
    scan_units(A.buf[1], w, ld, L, P, -1, st_scan);
    __syncthreads();
    if (tid == 0) A.cand[g] = s_cand;

    for (int s = 0; s < n - 1; ++s) {
        if (!sync()) return;
        // ---- the merge: smallest published candidate --------------------
        uint64_t best = kNone;
        const uint64_t *cs = A.cand + (size_t)(s & 1) * G;
        for (int t = tid; t < G; t += B) best = umin64(best, cs[t]);
        best = block_min(best);
        if (best == kNone) {
            if (tid == 0) {
                atomicOr(&A.ctl->error, kErrInternal);
                __hip_atomic_store(&A.sc->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            return;
        }
        int ci = (int)((best >> 16) & 0xFFFFull), cj = (int)(best & 0xFFFFull);
        const float h = unord32((uint32_t)(best >> 32));
        const int ni = (int)L.size1[ci] + 1, nj = (int)L.size1[cj] + 1;
        float *C = cur ? A.buf[1] : A.buf[0];
        if (g == 0 && tid == 0) {
            int4 rec;
            rec.x = idx[ci];
            rec.y = idx[cj];
            rec.z = __float_as_int(h);
            rec.w = ni + nj;
            reinterpret_cast<int4 *>(A.out)[s] = rec;
        }
        if (s == n - 2) break;

        // ---- Lance-Williams update of row/column i (Section 4 step 3) -----
        float ai = 0.0f, aj = 0.0f, bij = 0.0f;
        if (link == HAC_AVERAGE || link == HAC_CENTROID) {
            const double sum = (double)(ni + nj);
            ai = (float)((double)ni / sum);
            aj = (float)((double)nj / sum);
            bij = (float)(-((double)ni * (double)nj) / (sum * sum));
        }
        if (tid == 0) s_cand = kNone;
        __syncthreads();
        uint64_t key = kNone;
        for (int k = g * B + tid; k < w; k += G * B) {
            if (k == ci || k == cj || !live_at(L, k)) continue;
            const float a = C[(size_t)ci * ld + k], b = C[(size_t)cj * ld + k];
            const float v = lw_update(link, a, b, h, ni, nj, (int)L.size1[k] + 1, ai, aj, bij);
            C[(size_t)ci * ld + k] = v;
            C[(size_t)k * ld + ci] = v;
            ++st_upd;
            key = umin64(key, ((uint64_t)ord32(v) << 32) | ((uint64_t)min(ci, k) << 16) | (uint64_t)max(ci, k));
        }
        fold(key);
        __syncthreads();
        // ---- retire j, grow i (Section 4 steps 2, 4; Section 5.3 step 6) ---
        if (tid == 0) {
            L.live[cj >> 5] &= ~(1u << (cj & 31));
            L.size1[ci] = (uint16_t)(ni + nj - 1);
        }
        --m;
        __syncthreads();

        // ---- compaction of the live slots --------------------------------
        if (m >= kMinCompactW && (long long)m * kCompactDen < (long long)w * kCompactNum) {
            if (!sync()) return;  // every update is in place
            live_prefix(L, w);
            const int nw2 = m, nld2 = (m + 3) & ~3;
            compact_copy(C, w, ld, cur ? A.buf[0] : A.buf[1], nld2, idx, A.idx + (size_t)(idx_half ^ 1) * n, L);
            // This workgroup's candidate (new entries of row/column i) in
            // the new indices.
            if (tid == 0 && s_cand != kNone) {
                const uint64_t c = s_cand;
                const int a = new_index(L, (int)((c >> 16) & 0xFFFFull)), b = new_index(L, (int)(c & 0xFFFFull));
                s_cand = (c & 0xFFFFFFFF00000000ull) | ((uint64_t)a << 16) | (uint64_t)b;
            }
            ci = new_index(L, ci);
            compact_sizes(L, w);
            if (!sync()) return;  // the copy is complete
            for (int q = tid; q < ((w + 31) >> 5); q += B) {
                const int rem = nw2 - q * 32;
                L.live[q] = rem >= 32 ? 0xFFFFFFFFu : rem > 0 ? ((1u << rem) - 1u) : 0u;
            }
            w = nw2;
            ld = nld2;
            cur ^= 1;
            idx_half ^= 1;
            idx = A.idx + (size_t)idx_half * n;
            C = cur ? A.buf[1] : A.buf[0];
            if (g == 0 && tid == 0) A.sc->compactions++;
            __syncthreads();
            P = partition(w, G, g);
        }

        // ---- the paper's step 1 for the next merge ------------------------
        scan_units(C, w, ld, L, P, ci, st_scan);
        __syncthreads();
        if (tid == 0) A.cand[(size_t)((s + 1) & 1) * G + g] = s_cand;
    }
    const unsigned long long sc = wave_sum(st_scan), up = wave_sum(st_upd);
    if ((tid & 63) == 0) {
        atomicAdd(&A.ctl->rescan_elems, sc);
        atomicAdd(&A.ctl->update_elems, up);
    }
    if (g == 0 && tid == 0) A.ctl->rounds = A.sc->compactions;
}

}  // namespace

ScanLayout scan_layout(int n, int G) {
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    ScanLayout L{};
    size_t off = 0;
    L.ctl = off;  off += al(sizeof(ScanCtl));
    L.cand = off; off += al((size_t)2 * G * 8);
    L.idx = off;  off += al((size_t)2 * n * 4);
    L.bytes = off;
    return L;
}

size_t scan_spare_floats(int n) { return (size_t)n * (size_t)((n + 3) & ~3); }

size_t scan_lds_bytes(int n) {
    const size_t nw = (size_t)(n + 31) / 32;
    return (((size_t)n * 2 + 15) & ~(size_t)15) + nw * 4 + (nw + 1) * 4;
}

int scan_occupancy(int n) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void *>(&k_scan), kScanBlock,
                                                     scan_lds_bytes(n)) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return blocks < 1 ? 1 : blocks;
}

hipError_t launch_scan(float *D, float *spare, int n, int link, hac_merge *out, const uint32_t *status, Control *ctl,
                       void *ws, int G, uint64_t timeout_ticks, int flags, hipStream_t stream) {
    const ScanLayout Lo = scan_layout(n, G);
    char *b = static_cast<char *>(ws);
    Args a;
    a.buf[0] = D;
    a.buf[1] = spare;
    a.n = n;
    a.link = link;
    a.flags = flags;
    a.status = status;
    a.ctl = ctl;
    a.sc = reinterpret_cast<ScanCtl *>(b + Lo.ctl);
    a.cand = reinterpret_cast<uint64_t *>(b + Lo.cand);
    a.idx = reinterpret_cast<int32_t *>(b + Lo.idx);
    a.out = out;
    a.timeout = timeout_ticks;
    void *args[] = {&a};
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_scan),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)scan_lds_bytes(HAC_MAX_N));
        if (e != hipSuccess) return e;
        attr = true;
    }
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_scan), dim3(G), dim3(kScanBlock), args,
                                      (unsigned)scan_lds_bytes(n), stream);
}

}  // namespace hac
