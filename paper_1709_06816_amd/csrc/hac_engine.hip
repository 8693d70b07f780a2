// Device engine: Lance-Williams agglomerative clustering on gfx950.
//
// One instance is run by a group of g workgroups (g = 1 for small and batched
// instances; g up to the number of co-resident workgroups for large ones).
// All n-1 merges of an instance happen inside one launch.
//
// Work split (one GPU, the whole matrix in HBM):
//   * The n x n fp32 matrix is kept fully symmetric, row-major.  Rows are
//     owned in chunks of 64 by the group's workgroups (boustrophedon order so
//     that the triangular set-up work is balanced).
//   * Each workgroup keeps, in LDS, a cache entry per owned row k:
//     (ord(min_{l>k live} D[k][l]) : 32 | argmin l : 16 | size(k)-1 : 16),
//     i.e. the row's closest live partner to its right with ties to the
//     smallest l, plus the cluster size.
//   * Merge step (Section 4 steps 1-4; Section 5.3 steps 1-6):
//       argmin   every workgroup publishes the smallest cached key of its
//                rows and the smallest new entry of row i (see below); the
//                group minimum is the lexicographically smallest (D, i, j),
//                the same on every workgroup, so no second broadcast is
//                needed (Section 5.3, steps 2-5).
//       update   the owner of column k reads D[i][k], D[j][k] (coalesced row
//                reads), applies the Table 1 update, writes D[i][k] (row) and
//                D[k][i] (column, through symmetric storage), refreshes its
//                cache entry for row k and queues a rescan of row k when the
//                cached partner was i or j and can no longer be trusted
//                (Section 5.3, step 6).
//       row i    its new minimum over l > i is reduced from the updated
//                values themselves and carried in the next exchange.
//   * Exchange between workgroups: each workgroup writes three 64-bit words
//     tagged with a 16-bit generation into its own slot (double-buffered by
//     parity) after an agent-scope release fence; every workgroup polls all
//     slots of the group and takes an agent-scope acquire fence.  One
//     exchange per merge, no atomic counter.
#include <hip/hip_runtime.h>

#include "hac_engine.h"

namespace hac {
namespace {

constexpr uint64_t kEmpty = ~0ull;                     // "no candidate"
constexpr uint32_t kEmptyOrd = 0xFFFFFFFFu;             // above ord(+inf)
constexpr uint64_t kEmptyRow = 0xFFFFFFFFFFFF0000ull;   // cache entry without partner
constexpr uint64_t kHi32 = 0xFFFFFFFF00000000ull;
constexpr int kUpdBatch = 8;                           // chunks per wave per load batch
constexpr int kScanUnroll = 8;                         // loads in flight per thread in a rescan

// Order-preserving map of fp32 onto u32 (zeros are canonical +0 here).
__device__ __forceinline__ uint32_t ord32(float x) {
    uint32_t u = __float_as_uint(x);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord32(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

// Table 1 update, fp32, fixed order, no contraction.  Coefficients are fp64
// quotients rounded once to fp32.  Single/complete use the exact closed forms
// min/max of the Table 1 rows (1/2, 1/2, 0, -+1/2).
__device__ __forceinline__ float lw_update(int link, float dki, float dkj, float dij, int ni,
                                           int nj, int nk, float ai, float aj) {
    float v;
    if (link == HAC_SINGLE) {
        v = fminf(dki, dkj);
    } else if (link == HAC_COMPLETE) {
        v = fmaxf(dki, dkj);
    } else if (link == HAC_AVERAGE) {
        v = __fadd_rn(__fmul_rn(ai, dki), __fmul_rn(aj, dkj));
    } else {
        double t = (double)(ni + nj + nk);
        float wi = (float)((double)(ni + nk) / t);
        float wj = (float)((double)(nj + nk) / t);
        float wb = (float)(-(double)nk / t);
        v = __fadd_rn(__fadd_rn(__fmul_rn(wi, dki), __fmul_rn(wj, dkj)), __fmul_rn(wb, dij));
    }
    return v == 0.0f ? 0.0f : v;
}

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

__device__ __forceinline__ uint64_t wave_min(uint64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = umin64(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ bool is_live(const uint32_t *amask, int l) {
    return (amask[l >> 5] >> (l & 31)) & 1u;
}

// Chunk ownership (boustrophedon over rounds of g chunks).
__device__ __forceinline__ int chunk_of(int lq, int g, int w) {
    return lq * g + ((lq & 1) ? (g - 1 - w) : w);
}
__device__ __forceinline__ int owner_of_row(int k, int g) {
    int q = k >> 6, lq = q / g, r = q - lq * g;
    return (lq & 1) ? (g - 1 - r) : r;
}
__device__ __forceinline__ int local_of_row(int k, int g) { return ((k >> 6) / g) * 64 + (k & 63); }
__device__ __forceinline__ int own_chunks(int n, int g, int w) {
    int nch = (n + 63) >> 6, full = nch / g, rem = nch - full * g;
    int last = (full & 1) ? (g - 1 - w) : w;
    return full + (last < rem ? 1 : 0);
}

struct Lds {
    uint64_t *cache;    // own_cap entries
    uint16_t *rlist;    // own_cap entries: rows queued for a rescan (local index)
    uint32_t *amask;    // live bitmask of all n slots
    float *tile;        // kTile x (kTile + 1), set-up only
};

__shared__ uint64_t s_red[2][kWaves];
__shared__ uint32_t s_nresc;
__shared__ int s_inst;
__shared__ uint32_t s_fail;

// Minimum of (a, b) over the workgroup, returned to every thread.
__device__ void block_min2(uint64_t &a, uint64_t &b) {
    a = wave_min(a);
    b = wave_min(b);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        s_red[0][wv] = a;
        s_red[1][wv] = b;
    }
    __syncthreads();
    a = s_red[0][0];
    b = s_red[1][0];
#pragma unroll
    for (int q = 1; q < kWaves; ++q) {
        a = umin64(a, s_red[0][q]);
        b = umin64(b, s_red[1][q]);
    }
}

__device__ unsigned long long block_sum(unsigned long long v) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) s_red[0][wv] = v;
    __syncthreads();
    unsigned long long r = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) r += s_red[0][q];
    return r;
}

// Smallest (D[k][l], l) over live l > k; kEmpty if none.  Whole workgroup.
// `elems` counts the live entries this thread compared.  Rows are read with
// 16-byte loads when n is a multiple of 4 (row starts are then aligned).
__device__ uint64_t rescan_row(const float *__restrict__ D, int n, int k, const uint32_t *amask,
                               unsigned long long &elems) {
    const float *row = D + (size_t)k * n;
    uint64_t best = kEmpty;
    if ((n & 3) == 0) {
        const float4 *r4 = reinterpret_cast<const float4 *>(row);
        const int nq = n >> 2;
        for (int q0 = ((k + 1) >> 2) + (int)threadIdx.x; q0 < nq; q0 += kScanUnroll * kBlock) {
            float4 x[kScanUnroll];
#pragma unroll
            for (int u = 0; u < kScanUnroll; ++u) {
                const int q = q0 + u * kBlock;
                x[u] = q < nq ? r4[q] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
#pragma unroll
            for (int u = 0; u < kScanUnroll; ++u) {
                const int q = q0 + u * kBlock;
                if (q >= nq) continue;
                // live bits of l = 4q .. 4q+3, restricted to l > k
                uint32_t m = (amask[q >> 3] >> ((q & 7) * 4)) & 0xFu;
                const int below = k + 1 - 4 * q;  // entries l < k+1 inside this quad
                if (below > 0) m &= (0xFu << below) & 0xFu;
                if (!m) continue;
                elems += __popc(m);
                const float v[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if ((m >> c) & 1u)
                        best = umin64(best, ((uint64_t)ord32(v[c]) << 32) | ((uint64_t)(4 * q + c) << 16));
            }
        }
    } else {
        for (int l0 = k + 1 + (int)threadIdx.x; l0 < n; l0 += kScanUnroll * kBlock) {
            float x[kScanUnroll];
#pragma unroll
            for (int u = 0; u < kScanUnroll; ++u) {
                int l = l0 + u * kBlock;
                x[u] = l < n ? row[l] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kScanUnroll; ++u) {
                int l = l0 + u * kBlock;
                if (l < n && is_live(amask, l)) {
                    best = umin64(best, ((uint64_t)ord32(x[u]) << 32) | ((uint64_t)l << 16));
                    ++elems;
                }
            }
        }
    }
    uint64_t dummy = kEmpty;
    block_min2(best, dummy);
    return best;
}

// Set-up (plays the part of the paper's initial distribution of the matrix):
// validate and canonicalise the strict upper triangle, mirror it into the
// lower triangle, and compute each owned row's first cache entry.  The owner
// of row block R handles every tile (R, C >= R), so row minima stay in LDS.
__device__ void setup_rows(const Instance &I, int g, int w, Lds &L) {
    const int n = I.n, T = (n + 63) >> 6;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float *D = I.D;
    uint32_t bad = 0;
    for (int lq = 0;; ++lq) {
        const int R = chunk_of(lq, g, w);
        if (R >= T) break;
        uint64_t run[16];
#pragma unroll
        for (int p = 0; p < 16; ++p) run[p] = kEmpty;
        for (int C = R; C < T; ++C) {
            float x[16];
            const int col = C * 64 + lane;
#pragma unroll
            for (int p = 0; p < 16; ++p) {
                const int row = R * 64 + wv + 4 * p;
                x[p] = (row < n && col < n && col > row) ? D[(size_t)row * n + col] : 0.0f;
            }
#pragma unroll
            for (int p = 0; p < 16; ++p) {
                const int rr = wv + 4 * p, row = R * 64 + rr;
                if (row < n && col < n && col > row) {
                    if (!(fabsf(x[p]) <= 0x1p100f)) bad = 1;
                    if (__float_as_uint(x[p]) == 0x80000000u) {
                        x[p] = 0.0f;
                        D[(size_t)row * n + col] = 0.0f;
                    }
                    run[p] = umin64(run[p], ((uint64_t)ord32(x[p]) << 32) | ((uint64_t)col << 16));
                }
                L.tile[rr * (kTile + 1) + lane] = x[p];
            }
            __syncthreads();
#pragma unroll
            for (int p = 0; p < 16; ++p) {
                const int a = wv + 4 * p;  // row inside the lower tile (C, R)
                const int lrow = C * 64 + a, lcol = R * 64 + lane;
                if (lrow < n && lcol < lrow) D[(size_t)lrow * n + lcol] = L.tile[lane * (kTile + 1) + a];
            }
            __syncthreads();
        }
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            uint64_t v = wave_min(run[p]);
            if (lane == 0) L.cache[lq * 64 + wv + 4 * p] = (v == kEmpty) ? kEmptyRow : v;
        }
    }
    if (bad) atomicOr(I.status, kErrInput);
}

struct Stats {
    unsigned long long rescans = 0, rescan_elems = 0, update_elems = 0;
    unsigned long long prof[kPhases] = {0, 0, 0, 0, 0};  // thread 0 only
    uint64_t mark = 0;
    // Charge the time since the last mark to phase p (thread 0).
    __device__ __forceinline__ void lap(int p) {
        if (threadIdx.x == 0) {
            const uint64_t now = wall_clock64();
            prof[p] += now - mark;
            mark = now;
        }
    }
};

// Slot format (three u64, each carrying the 16-bit generation in its low
// bits so that a reader can tell a fresh word from an old one):
//   w0 = (p1 with its low 16 bits cleared) | gen      p1 = ord:32 | row:16 | partner:16
//   w1 = (partner of p1) << 16 | gen
//   w2 = (p2 with its low 16 bits cleared) | gen      p2 = ord:32 | column:16 | 0
__device__ __forceinline__ void put_slot(uint64_t *s, uint64_t p1, uint64_t p2, uint64_t gen) {
    __hip_atomic_store(s + 0, (p1 & ~0xFFFFull) | gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(s + 1, ((p1 & 0xFFFFull) << 16) | gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(s + 2, (p2 & ~0xFFFFull) | gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until slot s holds generation gen.  Returns false if the launch was
// aborted or the watchdog expired (then the abort flag is raised for all).
__device__ bool get_slot(const uint64_t *s, uint64_t gen, uint64_t &p1, uint64_t &p2,
                         const Instance &I, Control *ctl, uint64_t timeout) {
    const uint64_t t0 = wall_clock64();
    for (uint32_t it = 1;; ++it) {
        const uint64_t a = __hip_atomic_load(s + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t b = __hip_atomic_load(s + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t c = __hip_atomic_load(s + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((a & 0xFFFFull) == gen && (b & 0xFFFFull) == gen && (c & 0xFFFFull) == gen) {
            p1 = (a & ~0xFFFFull) | ((b >> 16) & 0xFFFFull);
            p2 = c & ~0xFFFFull;
            return true;
        }
        if ((it & 63u) == 0) {
            if (__hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
            if (wall_clock64() - t0 > timeout) {
                atomicOr(&ctl->error, kErrTimeout);
                atomicOr(I.status, kErrTimeout);
                __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
        }
    }
}

// Publish this workgroup's candidates for generation `epoch`, wait for the
// rest of the group, and return the group-wide minima (Section 5.3 steps
// 2-4: every processor ends up with the same global minimum).  Returns false
// if the wait was abandoned; the decision is the same for every thread.
__device__ bool group_exchange(const Instance &I, int g, int w, uint32_t epoch, uint64_t &p1,
                               uint64_t &p2, Control *ctl, uint64_t timeout) {
    if (threadIdx.x == 0) s_fail = 0;
    block_min2(p1, p2);
    const uint64_t gen = epoch & 0xFFFFu;
    uint64_t *base = I.slots + (size_t)(epoch & 1u) * (g + 1) * kSlotStride;
    if (threadIdx.x == 0) {
        // Everything this workgroup wrote before the barrier in block_min2
        // becomes visible to whoever observes the slot.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        put_slot(base + (size_t)w * kSlotStride, p1, p2, gen);
    }
    uint64_t m1 = kEmpty, m2 = kEmpty;
    if (I.exchange == kExchAllToAll || w == 0) {
        for (int t = threadIdx.x; t < g; t += kBlock) {
            uint64_t a1, a2;
            if (!get_slot(base + (size_t)t * kSlotStride, gen, a1, a2, I, ctl, timeout)) {
                atomicOr(&s_fail, 1u);
                break;
            }
            m1 = umin64(m1, a1);
            m2 = umin64(m2, a2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        block_min2(m1, m2);
        if (I.exchange == kExchReducer && threadIdx.x == 0 && !s_fail) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            put_slot(base + (size_t)g * kSlotStride, m1, m2, gen);
        }
    } else {
        if (threadIdx.x == 0) {
            if (!get_slot(base + (size_t)g * kSlotStride, gen, m1, m2, I, ctl, timeout)) s_fail = 1;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        block_min2(m1, m2);
    }
    p1 = m1;
    p2 = m2;
    return s_fail == 0;
}

// Run one instance on workgroup w of a group of g.
__device__ void run_instance(const Instance &I, int g, int w, uint8_t *smem, Control *ctl,
                             uint64_t timeout, Stats &st) {
    const int n = I.n, link = I.link;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, tid = threadIdx.x;
    const int own_ch = own_chunks(n, g, w);
    const int own_cap = ((((n + 63) >> 6) + g - 1) / g) * 64;
    const int mask_words = (n + 31) >> 5;
    Lds L;
    L.cache = reinterpret_cast<uint64_t *>(smem);
    L.rlist = reinterpret_cast<uint16_t *>(L.cache + own_cap);
    L.amask = reinterpret_cast<uint32_t *>(L.rlist + own_cap);
    L.tile = reinterpret_cast<float *>(L.amask + mask_words);
    float *D = I.D;

    if (tid == 0) st.mark = wall_clock64();
    for (int li = tid; li < own_cap; li += kBlock) L.cache[li] = kEmptyRow;
    for (int q = tid; q < mask_words; q += kBlock) {
        int rem = n - q * 32;
        L.amask[q] = rem >= 32 ? 0xFFFFFFFFu : ((1u << rem) - 1u);
    }
    __syncthreads();
    setup_rows(I, g, w, L);
    if (g > 1) {
        for (int li = tid; li < own_ch * 64; li += kBlock) {
            int k = chunk_of(li >> 6, g, w) * 64 + (li & 63);
            if (k < n) I.gsize[k] = 1;
        }
    }
    __syncthreads();

    // Local candidates: smallest cached key of the owned rows, none for row i.
    uint64_t p1 = kEmpty, p2 = kEmpty;
    for (int li = tid; li < own_ch * 64; li += kBlock) {
        int k = chunk_of(li >> 6, g, w) * 64 + (li & 63);
        uint64_t c = L.cache[li];
        if (k < n && (c >> 32) != kEmptyOrd)
            p1 = umin64(p1, (c & kHi32) | ((uint64_t)k << 16) | ((c >> 16) & 0xFFFFull));
    }

    st.lap(kPhSetup);
    int i_prev = -1;
    // Size of the cluster formed by the previous merge.  Every workgroup
    // carries it in a register; its owner writes it to gsize one merge later,
    // when no workgroup can still be reading the old value.
    int last_size = 0;
    for (int s = 0; s < n - 1; ++s) {
        // ---- argmin over the group (Section 5.3 steps 1-5) ---------------
        if (g > 1) {
            if (!group_exchange(I, g, w, (uint32_t)s + 1u, p1, p2, ctl, timeout)) return;
        } else {
            block_min2(p1, p2);
        }
        st.lap(s == 0 ? kPhSetup : kPhWait);
        if (s == 0) {
            // Set-up results (input check) are visible to everyone now; thread 0
            // reads the status word and the decision is shared through LDS so
            // that every thread leaves together.
            uint64_t ok = kEmpty, dummy = kEmpty;
            if (tid == 0 &&
                (__hip_atomic_load(I.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrInput))
                ok = 0;
            block_min2(ok, dummy);
            if (ok == 0) return;
        }
        uint64_t key_ip = kEmpty;
        if (i_prev >= 0 && (uint32_t)(p2 >> 32) != kEmptyOrd)
            key_ip = (p2 & kHi32) | ((uint64_t)i_prev << 16) | ((p2 >> 16) & 0xFFFFull);
        if (i_prev >= 0 && owner_of_row(i_prev, g) == w && tid == 0) {
            const int li = local_of_row(i_prev, g);
            const uint64_t c = L.cache[li];
            L.cache[li] = (((uint32_t)(p2 >> 32) != kEmptyOrd) ? (p2 & ~0xFFFFull) : kEmptyRow) |
                          (c & 0xFFFFull);
        }
        const uint64_t win = umin64(p1, key_ip);
        if ((uint32_t)(win >> 32) == kEmptyOrd) {
            if (tid == 0) {
                atomicOr(&ctl->error, kErrInternal);
                atomicOr(I.status, kErrInternal);
                if (g > 1) __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            return;
        }
        const int i = (int)((win >> 16) & 0xFFFFull);
        const int j = (int)(win & 0xFFFFull);
        const float h = unord32((uint32_t)(win >> 32));
        int ni, nj;
        if (g == 1) {
            // The size bits of row i may have just been rewritten by thread 0.
            __syncthreads();
            ni = (int)(L.cache[i] & 0xFFFFull) + 1;
            nj = (int)(L.cache[j] & 0xFFFFull) + 1;
        } else {
            ni = i == i_prev ? last_size
                             : __hip_atomic_load(I.gsize + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            nj = j == i_prev ? last_size
                             : __hip_atomic_load(I.gsize + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // ---- output the level (Section 4 step 4) -------------------------
        if (w == 0 && tid == 0) {
            int4 rec;
            rec.x = i;
            rec.y = j;
            rec.z = __float_as_int(h);
            rec.w = ni + nj;
            reinterpret_cast<int4 *>(I.out)[s] = rec;
        }
        if (s == n - 2) break;

        // ---- bookkeeping: j retired, i grows (Section 5.3 step 6) ---------
        if (tid == 0) {
            L.amask[j >> 5] &= ~(1u << (j & 31));
            s_nresc = 0;
            if (owner_of_row(j, g) == w) L.cache[local_of_row(j, g)] = kEmptyRow;
            if (owner_of_row(i, g) == w) {
                const int li = local_of_row(i, g);
                L.cache[li] = (L.cache[li] & ~0xFFFFull) | (uint64_t)(ni + nj - 1);
            }
            // Other workgroups read gsize[i] for this merge; the new size of i
            // is published during the next one (they use last_size meanwhile).
            if (g > 1 && i_prev >= 0 && owner_of_row(i_prev, g) == w) I.gsize[i_prev] = last_size;
        }
        __syncthreads();

        // ---- Lance-Williams update of row/column i (Section 4 step 3) -----
        float ai = 0.0f, aj = 0.0f;
        if (link == HAC_AVERAGE) {
            const double sum = (double)(ni + nj);
            ai = (float)((double)ni / sum);
            aj = (float)((double)nj / sum);
        }
        float *Di = D + (size_t)i * n;
        const float *Dj = D + (size_t)j * n;
        p2 = kEmpty;
        for (int lq0 = wv; lq0 < own_ch; lq0 += kWaves * kUpdBatch) {
            float a[kUpdBatch], b[kUpdBatch];
#pragma unroll
            for (int u = 0; u < kUpdBatch; ++u) {
                const int lq = lq0 + u * kWaves;
                const int k = lq < own_ch ? chunk_of(lq, g, w) * 64 + lane : n;
                const bool ok = k < n;
                a[u] = ok ? Di[k] : 0.0f;
                b[u] = ok ? Dj[k] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kUpdBatch; ++u) {
                const int lq = lq0 + u * kWaves;
                if (lq >= own_ch) break;
                const int k = chunk_of(lq, g, w) * 64 + lane;
                if (k >= n || k == i || k == j || !is_live(L.amask, k)) continue;
                const int li = lq * 64 + lane;
                const uint64_t c = L.cache[li];
                const int nk = (int)(c & 0xFFFFull) + 1;
                const float v = lw_update(link, a[u], b[u], h, ni, nj, nk, ai, aj);
                Di[k] = v;
                D[(size_t)k * n + i] = v;
                st.update_elems++;
                const uint32_t ov = ord32(v);
                if (k > i) p2 = umin64(p2, ((uint64_t)ov << 32) | ((uint64_t)k << 16));
                const int nn = (int)((c >> 16) & 0xFFFFull);
                if (k < i) {
                    const uint32_t oc = (uint32_t)(c >> 32);
                    if (nn == i || nn == j) {
                        if (ov <= oc)
                            L.cache[li] = ((uint64_t)ov << 32) | ((uint64_t)i << 16) | (c & 0xFFFFull);
                        else
                            L.rlist[atomicAdd(&s_nresc, 1u)] = (uint16_t)li;
                    } else if (ov < oc || (ov == oc && i < nn)) {
                        L.cache[li] = ((uint64_t)ov << 32) | ((uint64_t)i << 16) | (c & 0xFFFFull);
                    }
                } else if (k < j && nn == j) {
                    L.rlist[atomicAdd(&s_nresc, 1u)] = (uint16_t)li;
                }
            }
        }
        __syncthreads();

        st.lap(kPhUpdate);

        // ---- refresh rows whose cached partner is gone --------------------
        const uint32_t nresc = s_nresc;
        for (uint32_t r = 0; r < nresc; ++r) {
            const int li = L.rlist[r];
            const int k = chunk_of(li >> 6, g, w) * 64 + (li & 63);
            const uint64_t best = rescan_row(D, n, k, L.amask, st.rescan_elems);
            if (tid == 0) {
                const uint64_t c = L.cache[li];
                L.cache[li] = (best == kEmpty ? kEmptyRow : best) | (c & 0xFFFFull);
            }
        }
        if (tid == 0) st.rescans += nresc;
        __syncthreads();

        st.lap(kPhRescan);

        // ---- local candidates for the next argmin -------------------------
        p1 = kEmpty;
        for (int li = tid; li < own_ch * 64; li += kBlock) {
            const int k = chunk_of(li >> 6, g, w) * 64 + (li & 63);
            if (k >= n || k == i) continue;
            const uint64_t c = L.cache[li];
            if ((uint32_t)(c >> 32) == kEmptyOrd) continue;
            p1 = umin64(p1, (c & kHi32) | ((uint64_t)k << 16) | ((c >> 16) & 0xFFFFull));
        }
        i_prev = i;
        last_size = ni + nj;
        st.lap(kPhCand);
    }
}

__device__ void flush_stats(Control *ctl, Stats &st) {
    unsigned long long a = block_sum(st.rescans);
    unsigned long long b = block_sum(st.rescan_elems);
    unsigned long long c = block_sum(st.update_elems);
    if (threadIdx.x == 0) {
        atomicAdd(&ctl->rescans, a);
        atomicAdd(&ctl->rescan_elems, b);
        atomicAdd(&ctl->update_elems, c);
        for (int p = 0; p < kPhases; ++p) {
            atomicAdd(&ctl->prof_sum[p], st.prof[p]);
            atomicMax(&ctl->prof_max[p], st.prof[p]);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_run(Instance inst, Control *ctl, uint64_t timeout) {
    extern __shared__ __align__(16) uint8_t smem[];
    Stats st;
    run_instance(inst, (int)gridDim.x, (int)blockIdx.x, smem, ctl, timeout, st);
    flush_stats(ctl, st);
}

__global__ __launch_bounds__(kBlock) void k_batch(const Instance *__restrict__ insts,
                                                 const int32_t *__restrict__ order, int count,
                                                 Control *ctl, uint64_t timeout) {
    extern __shared__ __align__(16) uint8_t smem[];
    Stats st;
    for (;;) {
        if (threadIdx.x == 0) s_inst = (int)atomicAdd(&ctl->next, 1u);
        __syncthreads();
        const int q = s_inst;
        __syncthreads();
        if (q >= count) break;
        const Instance inst = insts[order[q]];
        if (inst.n > 1) run_instance(inst, 1, 0, smem, ctl, timeout, st);
        __syncthreads();
    }
    flush_stats(ctl, st);
}

__global__ void k_zero(uint32_t *p, size_t words) {
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < words;
         q += (size_t)gridDim.x * blockDim.x)
        p[q] = 0u;
}

}  // namespace

int own_rows(int n, int g) { return ((((n + 63) >> 6) + g - 1) / g) * 64; }

size_t lds_bytes(int n, int own) {
    const size_t mask_words = (size_t)(n + 31) / 32;
    return (size_t)own * 8 + (size_t)own * 2 + mask_words * 4 + (size_t)kTile * (kTile + 1) * 4;
}

hipError_t engine_setup(size_t max_lds, size_t *usable) {
    // Dynamic LDS may use what the static LDS of the kernels leaves free.
    size_t static_max = 0;
    for (const void *fn : {reinterpret_cast<const void *>(&k_run), reinterpret_cast<const void *>(&k_batch)}) {
        hipFuncAttributes a;
        hipError_t e = hipFuncGetAttributes(&a, fn);
        if (e != hipSuccess) return e;
        static_max = a.sharedSizeBytes > static_max ? a.sharedSizeBytes : static_max;
    }
    const size_t dyn = max_lds > static_max ? max_lds - static_max : 0;
    for (const void *fn : {reinterpret_cast<const void *>(&k_run), reinterpret_cast<const void *>(&k_batch)}) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
        if (e != hipSuccess) return e;
    }
    *usable = dyn;
    return hipSuccess;
}

int engine_occupancy(size_t lds, bool batch) {
    int blocks = 0;
    const void *fn = batch ? reinterpret_cast<const void *>(&k_batch) : reinterpret_cast<const void *>(&k_run);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, kBlock, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return blocks;
}

hipError_t launch_zero(void *p, size_t words, hipStream_t stream) {
    if (words == 0) return hipSuccess;
    int grid = (int)((words + 255) / 256);
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, stream, (uint32_t *)p, words);
    return hipGetLastError();
}

hipError_t launch_run(const Instance &inst, int g, Control *ctl, uint64_t timeout_ticks,
                      hipStream_t stream) {
    const size_t lds = lds_bytes(inst.n, own_rows(inst.n, g));
    if (g == 1) {
        hipLaunchKernelGGL(k_run, dim3(1), dim3(kBlock), lds, stream, inst, ctl, timeout_ticks);
        return hipGetLastError();
    }
    Instance a0 = inst;
    Control *a1 = ctl;
    uint64_t a2 = timeout_ticks;
    void *args[] = {&a0, &a1, &a2};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_run), dim3(g), dim3(kBlock),
                                      args, (unsigned)lds, stream);
}

hipError_t launch_batch(const Instance *insts, const int32_t *order, int count, int grid,
                        size_t lds, Control *ctl, uint64_t timeout_ticks, hipStream_t stream) {
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kBlock), lds, stream, insts, order, count, ctl,
                       timeout_ticks);
    return hipGetLastError();
}

}  // namespace hac
