// Device engine: Lance-Williams agglomerative clustering on gfx950.
//
// Kernels:
//   k_setup   (single-instance path) validates and canonicalises the strict
//             upper triangle, mirrors it into the lower triangle (or writes
//             both triangles of a working copy) and computes each row's first
//             cached minimum; it spreads the O(n^2) pass over the whole device.
//   k_run     runs all n-1 merges of one instance on a group of g co-resident
//             workgroups of 1024 threads (g = 1 for small n); template
//             variants rescan rows at once, defer rescans behind lower bounds,
//             or rescan everything every merge (Section 5.3 step 1).
//   k_batch   runs many independent instances in one launch: the largest
//             may each get a fixed group of workgroups (exchanging through
//             their own slots), the rest take one workgroup each, largest
//             first, from a queue; each workgroup does its instance's set-up
//             itself (deferred rescans, lazy mirror).
//   k_serve   a persistent server: workgroups take jobs that the host
//             publishes in a ring in host memory, one workgroup or a group per
//             job, until the host stops it (deferred rescans, lazy mirror where
//             the job's step table fits the LDS).
//
// Data layout (one GPU, the whole matrix in HBM):
//   * The n x n fp32 matrix is made fully symmetric, row-major, by the set-up,
//     so that both D[i][k] and D[k][i] of the merged row/column are reachable
//     with coalesced row accesses (Section 5.2 stores only the upper half,
//     split over processors; here both halves live in one HBM).  k_run keeps
//     it symmetric; the batch and serving kernels write only the survivor's
//     row (lazy mirror: a pair is read from whichever of its two rows was
//     written later, see pair_at).
//   * Rows are owned in chunks of 64 by the group's workgroups (boustrophedon
//     order over rounds of g chunks).  Each workgroup keeps, in LDS, a cache
//     entry per owned row k: ord(min_{l>k live} D[k][l]) : 32 | argmin l : 16
//     (ties to the smallest l), a live bitmask of all slots and the size of
//     every cluster (every workgroup applies the same size updates).
//
// One merge (Section 4 steps 1-4; Section 5.3 steps 1-6):
//   argmin   every workgroup publishes the smallest cached key of its rows and
//            the smallest new entry of the previous survivor's row; the group
//            minimum is the lexicographically smallest (D, i, j) and is the
//            same on every workgroup, so no second broadcast is needed
//            (steps 2-5 of Section 5.3).
//   update   the owner of column k reads D[i][k], D[j][k] (row reads),
//            applies the Table 1 update, writes D[i][k] (row) and, without
//            the lazy mirror, D[k][i] (column, through symmetric storage),
//            and refreshes its cache entry for row k; a row whose cached
//            partner was i or j is rescanned at once or, deferred, keeps a
//            lower bound (step 6; see merge_loop).
//   row i    its new minimum over l > i is reduced from the new values
//            themselves and carried in the next exchange.
// Exchange between workgroups: each workgroup writes three 64-bit words
// tagged with a 16-bit generation into its own slot (double-buffered by
// parity) after an agent-scope release fence; readers poll the slots and take
// an agent-scope acquire fence.  One exchange per merge (plus one per forced
// round of the deferred mode).
#include <hip/hip_runtime.h>

#include "hac_dev.h"
#include "hac_engine.h"

namespace hac {
namespace {

constexpr uint64_t kEmpty = ~0ull;                     // "no candidate"
constexpr uint32_t kEmptyOrd = 0xFFFFFFFFu;             // above ord(+inf)
constexpr uint64_t kEmptyRow = 0xFFFFFFFFFFFF0000ull;   // cache entry without partner
constexpr uint64_t kHi32 = 0xFFFFFFFF00000000ull;
// Low bit of a row's cache entry: the row's partner merged and the entry
// holds only a lower bound of its minimum (partner field 0; deferred mode).
constexpr uint64_t kStale = 1ull;
constexpr int kMaxWaves = 16;
// Loads in flight per thread: chunks per wave per update batch, and 16-byte
// loads per rescan step.  Large workgroups need fewer per thread for the same
// bytes in flight and have only 128 VGPRs per thread.
template <int B> constexpr int upd_batch() { return B >= 1024 ? 2 : 8; }
template <int B> constexpr int seg_unroll() { return B >= 1024 ? 4 : 8; }

// 64-bit value of the lane picked by DPP control CTRL; lanes of rows outside
// ROW_MASK keep their own value.  All lanes must be active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
    const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
    const int plo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROW_MASK, 0xF, false);
    const int phi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROW_MASK, 0xF, false);
    return ((uint64_t)(uint32_t)phi << 32) | (uint32_t)plo;
}

// Minimum over the wave, valid in lane 63: within quads (quad_perm xor 1,
// xor 2), half rows (row_half_mirror), rows (row_mirror), then across rows
// (row_bcast:15 into rows 1 and 3, row_bcast:31 into rows 2 and 3).
__device__ __forceinline__ uint64_t wave_min_last(uint64_t v) {
    v = umin64(v, dpp_u64<0xB1, 0xF>(v));
    v = umin64(v, dpp_u64<0x4E, 0xF>(v));
    v = umin64(v, dpp_u64<0x141, 0xF>(v));
    v = umin64(v, dpp_u64<0x140, 0xF>(v));
    v = umin64(v, dpp_u64<0x142, 0xA>(v));
    return umin64(v, dpp_u64<0x143, 0xC>(v));
}

// Fold every lane's v into the LDS word *acc with one atomic minimum per
// wave.  Call with every lane of the wave active.
__device__ __forceinline__ void lds_min(uint64_t *acc, uint64_t v) {
    v = wave_min_last(v);
    if ((threadIdx.x & 63) == 63 && v != ~0ull)
        atomicMin(reinterpret_cast<unsigned long long *>(acc), (unsigned long long)v);
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
__device__ __forceinline__ int row_of_local(int li, int g, int w) {
    return chunk_of(li >> 6, g, w) * 64 + (li & 63);
}

__shared__ uint64_t s_red[2][kMaxWaves];
// Per-epoch accumulators, double-buffered by epoch parity:
// [0] smallest cached key of this workgroup's rows, [1] smallest new entry of
// the survivor's row, [2] and [3] the same minima over the whole group.
__shared__ uint64_t s_acc[2][4];
__shared__ uint32_t s_nresc;
__shared__ uint64_t s_lim;
__shared__ uint32_t s_fail;
__shared__ int s_inst;

// Minimum of (a, b) over the workgroup, returned to every thread.
template <int B>
__device__ void block_min2(uint64_t &a, uint64_t &b) {
    constexpr int W = B / 64;
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
    for (int q = 1; q < W; ++q) {
        a = umin64(a, s_red[0][q]);
        b = umin64(b, s_red[1][q]);
    }
}

template <int B>
__device__ unsigned long long block_sum(unsigned long long v) {
    constexpr int W = B / 64;
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) s_red[0][wv] = v;
    __syncthreads();
    unsigned long long r = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) r += s_red[0][q];
    return r;
}

// Set-up of row block R (rows 64R .. 64R+63) over tile columns
// c_begin .. c_end-1 (c_begin >= R), playing the part of the paper's initial
// distribution of the matrix: for every tile (R, C) read the strict-upper
// entries from src, validate and canonicalise them,
// store them in D (when D is not src, or to canonicalise -0), mirror them
// into tile (C, R) of D, and keep each row's running minimum.  Hands the
// minimum key (ord : 32 | column : 16) of row 64R + r over those columns to
// `sink(r, key)` (lane 0 of the wave holding that row; kEmpty if the row has
// no entry there).  The diagonal of D is never written (nor read later).
template <int B, class Sink>
__device__ void setup_block(const float *src, float *D, int n, int R, int c_begin, int c_end, float *tile,
                            uint32_t &bad, Sink sink) {
    constexpr int W = B / 64, P = 64 / W;  // rows of a tile per wave
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint64_t run[P];
#pragma unroll
    for (int p = 0; p < P; ++p) run[p] = kEmpty;
    for (int C = c_begin; C < c_end; ++C) {
        float x[P];
        const int col = C * 64 + lane;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int row = R * 64 + wv + W * p;
            x[p] = (row < n && col < n && col > row) ? src[(size_t)row * n + col] : 0.0f;
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int rr = wv + W * p, row = R * 64 + rr;
            if (row < n && col < n && col > row) {
                if (!(fabsf(x[p]) <= 0x1p100f)) bad = 1;
                const bool neg0 = __float_as_uint(x[p]) == 0x80000000u;
                if (neg0) x[p] = 0.0f;
                if (neg0 || src != D) D[(size_t)row * n + col] = x[p];
                run[p] = umin64(run[p], ((uint64_t)ord32(x[p]) << 32) | ((uint64_t)col << 16));
            }
            tile[rr * (kTile + 1) + lane] = x[p];
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int a = wv + W * p;  // row inside the lower tile (C, R)
            const int lrow = C * 64 + a, lcol = R * 64 + lane;
            if (lrow < n && lcol < lrow) D[(size_t)lrow * n + lcol] = tile[lane * (kTile + 1) + a];
        }
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint64_t v = wave_min(run[p]);
        if (lane == 0) sink(wv + W * p, v);
    }
}

struct Stats {
    unsigned long long rescans = 0, rescan_elems = 0, update_elems = 0, forced = 0;
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

// Publish this workgroup's candidates of epoch e (s_acc[e&1][0..1]), wait for
// the rest of the group, and leave the group-wide minima in s_acc[e&1][2..3]
// (Section 5.3 steps 2-4: every processor ends up with the same global
// minimum).  The caller's last barrier before the call must be
// barrier_stores_done(), so that every wave's stores are complete.  With
// `writeback` the slot follows a release that writes this XCD's L2 back (the
// caller wrote what it publishes with plain stores); without it the caller
// wrote everything it publishes since its last exchange with agent-scope
// stores, which are at the device's point of coherence once complete, and the
// slot follows at once.  Ends with a barrier.  Returns false if the wait was
// abandoned; the decision is the same for every thread.
template <int B>
__device__ bool group_exchange(const Instance &I, int g, int w, uint32_t e, Control *ctl,
                               uint64_t timeout, bool writeback) {
    const int b = e & 1;
    const uint64_t gen = e & 0xFFFFu;
    uint64_t *base = I.slots + (size_t)b * (g + 1) * kSlotStride;
    if (threadIdx.x == 0) {
        s_fail = 0;
        // Everything this workgroup wrote before the last barrier (complete,
        // see barrier_stores_done) becomes visible to whoever observes the
        // slot.
        if (writeback) release_agent();
        if (!((I.flags & kFlagStall) && w == 0)) put_slot(base + (size_t)w * kSlotStride, s_acc[b][0], s_acc[b][1], gen);
    }
    if (I.exchange == kExchAllToAll || w == 0) {
        if (threadIdx.x < 64) {  // wave 0 polls: lane t reads slots t, t+64, ...
            uint64_t m1 = kEmpty, m2 = kEmpty;
            for (int t = threadIdx.x; t < g; t += 64) {
                uint64_t a1, a2;
                if (!get_slot(base + (size_t)t * kSlotStride, gen, a1, a2, I, ctl, timeout)) {
                    atomicOr(&s_fail, 1u);
                    break;
                }
                m1 = umin64(m1, a1);
                m2 = umin64(m2, a2);
            }
            // The barrier below orders the other waves' later loads after this.
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            lds_min(&s_acc[b][2], m1);
            lds_min(&s_acc[b][3], m2);
        }
        __syncthreads();
        if (I.exchange == kExchReducer && threadIdx.x == 0 && !s_fail) {
            if (writeback) release_agent();
            put_slot(base + (size_t)g * kSlotStride, s_acc[b][2], s_acc[b][3], gen);
        }
    } else {
        if (threadIdx.x == 0) {
            uint64_t m1 = kEmpty, m2 = kEmpty;
            if (!get_slot(base + (size_t)g * kSlotStride, gen, m1, m2, I, ctl, timeout)) s_fail = 1;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_acc[b][2] = m1;
            s_acc[b][3] = m2;
        }
        __syncthreads();
    }
    return s_fail == 0;
}

// LDS of one workgroup.
struct Lds {
    uint64_t *cache;    // own_cap entries: ord:32 | partner:16 | 0:16
    uint16_t *rlist;    // own_cap entries: rows queued for a rescan (local index)
    uint32_t *amask;    // live bitmask of all n slots
    uint16_t *size1;    // size - 1 of every slot's cluster (n entries)
    uint16_t *wstep;    // lazy mirror: merge step (from 1) that last wrote each slot's row,
                        // 0 for the input (n entries, 8-byte aligned); null otherwise
    float *tile;        // mirror tile (in-kernel set-up only; shares space with size1, wstep)
};

__device__ Lds carve(uint8_t *smem, int n, int own_cap, bool lazy) {
    Lds L;
    L.cache = reinterpret_cast<uint64_t *>(smem);
    L.rlist = reinterpret_cast<uint16_t *>(L.cache + own_cap);
    L.amask = reinterpret_cast<uint32_t *>(L.rlist + own_cap);
    L.size1 = reinterpret_cast<uint16_t *>(L.amask + (((n + 31) >> 5) + 3) / 4 * 4);
    L.wstep = lazy ? L.size1 + ((n + 3) & ~3) : nullptr;
    L.tile = reinterpret_cast<float *>(L.size1);
    return L;
}

// Lazy mirror: where pair (a, b)'s current value is.  A merge step writes the
// whole row of its survivor, so of the two rows the one written last holds
// it; rows never written hold the (mirrored) input.
__device__ __forceinline__ size_t pair_at(int a, int b, uint32_t ta, uint32_t tb, int n) {
    return tb > ta ? (size_t)b * n + a : (size_t)a * n + b;
}

template <int B>
__device__ void init_masks(const Lds &L, int n) {
    const int mask_words = (n + 31) >> 5;
    for (int q = threadIdx.x; q < mask_words; q += B) {
        const int rem = n - q * 32;
        L.amask[q] = rem >= 32 ? 0xFFFFFFFFu : ((1u << rem) - 1u);
    }
    for (int k = threadIdx.x; k < n; k += B) L.size1[k] = 0;
    if (L.wstep)
        for (int k = threadIdx.x; k < n; k += B) L.wstep[k] = 0;
}

// Minimum (D[k][l], l) over live l > k, l != skip, of row k, folded into the
// LDS word *acc: the row tail is cut into segments of one wave's loads (U
// per lane), and waves WV0 .. B/64-1 take segments round-robin starting at
// wave (WV0 + base) mod their number (so consecutive rows start on different
// waves).  Returns the number of segments.  Waves below WV0 only count.
// With `wstep` (lazy mirror) each entry is read where pair_at puts it: from
// row k, or from row l if that was written later.
template <int B, int WV0, int U = seg_unroll<B>()>
__device__ int scan_row(const float *__restrict__ D, int n, int k, const uint32_t *amask, int skip, int base,
                        uint64_t *acc, unsigned long long &elems, const uint16_t *wstep) {
    constexpr int W = B / 64 - WV0;
    static_assert(W >= 1, "no wave left to rescan");
    const int lane = threadIdx.x & 63, wv = (int)(threadIdx.x >> 6) - WV0;
    const float *row = D + (size_t)k * n;
    const int first_sg = ((wv - base) % W + W) % W;
    int nseg;
    if ((n & 3) == 0) {
        // 16-byte loads over quads q0 .. n/4-1; row starts are aligned.
        const int q0 = (k + 1) >> 2, nq = n >> 2;
        nseg = (nq - q0 + 64 * U - 1) / (64 * U);
        if (wv < 0) return nseg;
        const uint32_t tk = wstep ? wstep[k] : 0u;
        for (int sg = first_sg; sg < nseg; sg += W) {
            float4 x[U];
            if (wstep) {
                // One 4-byte load per entry; the four write steps of a quad
                // come from one 8-byte LDS read.
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int q = q0 + sg * 64 * U + u * 64 + lane;
                    float e[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                    if (q < nq) {
                        const uint64_t t4 = *reinterpret_cast<const uint64_t *>(wstep + 4 * q);
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            e[c] = D[pair_at(k, 4 * q + c, tk, (uint32_t)(t4 >> (16 * c)) & 0xFFFFu, n)];
                    }
                    x[u] = make_float4(e[0], e[1], e[2], e[3]);
                }
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int q = q0 + sg * 64 * U + u * 64 + lane;
                    x[u] = q < nq ? *reinterpret_cast<const float4 *>(row + 4 * q)
                                  : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                }
            }
            uint64_t best = kEmpty;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = q0 + sg * 64 * U + u * 64 + lane;
                if (q >= nq) continue;
                uint32_t m = (amask[q >> 3] >> ((q & 7) * 4)) & 0xFu;  // live l = 4q..4q+3
                const int below = k + 1 - 4 * q;                         // those with l <= k
                if (below > 0) m &= (0xFu << below) & 0xFu;
                if ((skip >> 2) == q) m &= ~(1u << (skip & 3));
                elems += __popc(m);
                const float v[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if ((m >> c) & 1u)
                        best = umin64(best, ((uint64_t)ord32(v[c]) << 32) | ((uint64_t)(4 * q + c) << 16));
            }
            lds_min(acc, best);
        }
    } else {
        const int l0 = k + 1;
        nseg = (n - l0 + 64 * U - 1) / (64 * U);
        if (wv < 0) return nseg;
        const uint32_t tk = wstep ? wstep[k] : 0u;
        for (int sg = first_sg; sg < nseg; sg += W) {
            float x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int l = l0 + sg * 64 * U + u * 64 + lane;
                x[u] = l >= n ? 0.0f : wstep ? D[pair_at(k, l, tk, wstep[l], n)] : row[l];
            }
            uint64_t best = kEmpty;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int l = l0 + sg * 64 * U + u * 64 + lane;
                if (l < n && l != skip && is_live(amask, l)) {
                    best = umin64(best, ((uint64_t)ord32(x[u]) << 32) | ((uint64_t)l << 16));
                    ++elems;
                }
            }
            lds_min(acc, best);
        }
    }
    return nseg;
}

// Rescan the rows queued in rlist (their entries were reset to kEmptyRow when
// queued): each entry becomes the smallest (D[k][l], l) over live l > k with
// l != skip.  All waves take segments round-robin across all queued rows and
// fold their lanes' minima into the entry with LDS atomics, so no barrier is
// needed per row.
template <int B>
__device__ void rescan_rows(const float *__restrict__ D, int n, int g, int w, const Lds &L,
                            uint32_t nresc, int skip, unsigned long long &elems) {
    int base = 0;
    for (uint32_t r = 0; r < nresc; ++r) {
        const int li = L.rlist[r];
        base += scan_row<B, 0>(D, n, row_of_local(li, g, w), L.amask, skip, base, &L.cache[li], elems, L.wstep);
    }
}

// Fold the smallest cached key (ord:32 | row:16 | partner:16) of this
// workgroup's live rows other than `skip` into *acc, using threads 0 .. NT-1
// (whole waves).  A stale row's key is (bound, row, 0), below every key the
// row can really have.
template <int NT>
__device__ void fold_candidates(const Lds &L, int n, int g, int w, int own_ch, int skip, uint64_t *acc) {
    uint64_t p = kEmpty;
    for (int li = threadIdx.x; li < own_ch * 64; li += NT) {
        const int k = row_of_local(li, g, w);
        const uint64_t c = L.cache[li];
        if (k < n && k != skip && (uint32_t)(c >> 32) != kEmptyOrd)
            p = umin64(p, (c & kHi32) | ((uint64_t)k << 16) | ((c >> 16) & 0xFFFFull));
    }
    lds_min(acc, p);
}

// All n-1 merges of one instance on workgroup w of a group of g.  On entry
// the cache holds every owned row's first minimum, the masks are initialised
// and the input is known to be valid.
//
// Cache maintenance after merging (i, j), for an owned live row k:
//   * k < i: the row gains the entry (v_k, i) and loses column j.  If its
//     partner was i or j, the new minimum is min(minimum over l != i, j,
//     (v_k, i)); otherwise min(old entry, (v_k, i)).
//   * i < k < j: the row loses column j; if its partner was j its minimum is
//     recomputed over l != j (column i lies to its left).
//   * k > j: unchanged.
// kLoopCached rescans rows whose partner was i or j right after the argmin,
// overlapping the loads of rows i and j, and folds the new (v_k, i) in
// afterwards with an atomic minimum.  Ties resolve as in the lexicographic
// order: any other column attaining the old minimum lies to the right of the
// old partner.
//
// kLoopDefer takes those rescans off the merge's critical path: such a row
// becomes stale, keeping its old minimum as a lower bound (lowered by every
// new entry it receives, so it stays a bound whatever the linkage), and
// offers (bound, k, 0) to the argmin, a key below any the row can really
// have.  A stale row is rescanned only when a stale key wins an argmin: then
// every workgroup rescans all its stale rows at once and the argmin is
// repeated (an extra exchange, a "forced round").  Most bounds never win
// before their row merges or falls behind, and the rescans that are needed
// run batched, in parallel over the workgroups.
//
// kLoopScan drops the cache: before every argmin every workgroup rescans all
// its live rows, as Section 5.3 step 1 scans the whole matrix.
enum : int { kLoopCached = 0, kLoopDefer = 1, kLoopScan = 2 };

template <int B, int kMode, int U = upd_batch<B>(), bool kSoloLimit = false>
__device__ void merge_loop(const Instance &I, int g, int w, const Lds &L, Control *ctl,
                           uint64_t timeout, Stats &st, uint32_t epoch0, int s0 = 0, uint64_t *keys = nullptr,
                           int round0 = 0) {
    constexpr int W = B / 64;
    constexpr bool scan = kMode == kLoopScan, defer = kMode == kLoopDefer;
    const int n = I.n, link = I.link;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, tid = threadIdx.x;
    const int own_ch = own_chunks(n, g, w);
    const bool prof = (I.flags & kFlagProfile) != 0;
    const bool lazy = L.wstep != nullptr;
    float *D = I.D;

    if (tid == 0) {
        for (int b = 0; b < 2; ++b)
            for (int q = 0; q < 4; ++q) s_acc[b][q] = kEmpty;
        s_nresc = 0;
    }
    __syncthreads();
    // Exchange epochs after epoch0 (used by the caller) are taken one by one:
    // one per merge, one more for each forced round (deferred mode) and for
    // the second exchange of every merge (scan mode).
    uint32_t e = epoch0;
    fold_candidates<B>(L, n, g, w, own_ch, -1, &s_acc[(e + 1) & 1][0]);
    barrier_stores_done();  // later candidates are folded inside the update loop
    int i_prev = -1;
    for (int s = s0; s < n - 1; ++s) {
        // ---- argmin over the group (Section 5.3 steps 1-5) ---------------
        ++e;
        int b = e & 1;
        if (scan) {
            // The other parity's accumulators were last read before the last
            // barrier of the previous merge; clear them for epoch e+1.
            if (tid == 0)
                for (int q = 0; q < 4; ++q) s_acc[b ^ 1][q] = kEmpty;
            barrier_stores_done();
            if (g > 1 && !group_exchange<B>(I, g, w, e, ctl, timeout, false)) return;
        } else {
            // The candidates were folded during the last update (and are
            // published at once).  Alone, a workgroup still needs a barrier
            // here: thread 0's size update of the last merge is read below.
            if (g > 1) {
                if (!group_exchange<B>(I, g, w, e, ctl, timeout, false)) return;
            } else {
                __syncthreads();
            }
            if (tid == 0)
                for (int q = 0; q < 4; ++q) s_acc[b ^ 1][q] = kEmpty;  // for epoch e+1
        }
        const uint64_t p1 = g > 1 ? s_acc[b][2] : s_acc[b][0];
        const uint64_t p2 = g > 1 ? s_acc[b][3] : s_acc[b][1];
        if (prof) st.lap(s == 0 ? kPhSetup : kPhWait);
        // Row i_prev's new cache entry: its smallest new value to the right.
        const uint64_t ip_entry = ((uint32_t)(p2 >> 32) != kEmptyOrd) ? p2 : kEmptyRow;
        uint64_t key_ip = kEmpty;
        if (i_prev >= 0 && (uint32_t)(p2 >> 32) != kEmptyOrd)
            key_ip = (p2 & kHi32) | ((uint64_t)i_prev << 16) | ((p2 >> 16) & 0xFFFFull);
        uint64_t win = umin64(p1, key_ip);
        // A stale row's bound won (partner field 0; a real partner is > 0):
        // settle every stale row and take the argmin again.
        while (defer && (uint32_t)(win >> 32) != kEmptyOrd && (win & 0xFFFFull) == 0) {
            __syncthreads();  // p1, p2 are read; s_acc[b ^ 1] is clear; s_nresc is 0
            if (tid == 0 && i_prev >= 0 && owner_of_row(i_prev, g) == w) L.cache[local_of_row(i_prev, g)] = ip_entry;
            // In the batch and serving kernels (kSoloLimit) a workgroup alone
            // settles only the stale rows whose bound key is not above its
            // smallest exact key: the others cannot win the argmin that
            // follows (that exact key is still there), and a forced round
            // costs it no exchange, so later ones are cheap.  Groups settle
            // every stale row: fewer rows per round there meant many more
            // forced rounds, each an exchange (measured slower).
            uint64_t lim = kEmpty;
            if (kSoloLimit && g == 1) {
                if (tid == 0) s_lim = kEmpty;
                __syncthreads();  // also orders row i_prev's entry above before the pass
                uint64_t ex = kEmpty;
                for (int li = tid; li < own_ch * 64; li += B) {
                    const int k = row_of_local(li, g, w);
                    const uint64_t c = L.cache[li];
                    if (k < n && !(c & kStale) && (uint32_t)(c >> 32) != kEmptyOrd)
                        ex = umin64(ex, (c & kHi32) | ((uint64_t)k << 16) | ((c >> 16) & 0xFFFFull));
                }
                lds_min(&s_lim, ex);
                __syncthreads();
                lim = s_lim;
            }
            for (int li = tid; li < own_ch * 64; li += B) {
                const int k = row_of_local(li, g, w);
                if (k < n && k != i_prev && (L.cache[li] & kStale) &&
                    (((L.cache[li] & kHi32) | ((uint64_t)k << 16)) <= lim)) {
                    L.cache[li] = kEmptyRow;
                    L.rlist[atomicAdd(&s_nresc, 1u)] = (uint16_t)li;
                }
            }
            __syncthreads();
            const uint32_t nf = s_nresc;
            if (nf) rescan_rows<B>(D, n, g, w, L, nf, -1, st.rescan_elems);
            __syncthreads();
            if (tid == 0) {
                st.rescans += nf;
                st.forced += w == 0;
                s_nresc = 0;
                for (int q = 0; q < 4; ++q) s_acc[b][q] = kEmpty;  // for the epoch after the next
            }
            // s_acc[b ^ 1] has stayed clear since the exchange above.
            ++e;
            b = e & 1;
            fold_candidates<B>(L, n, g, w, own_ch, -1, &s_acc[b][0]);
            barrier_stores_done();
            if (g > 1) {
                if (!group_exchange<B>(I, g, w, e, ctl, timeout, false)) return;
                win = s_acc[b][2];
            } else {
                win = s_acc[b][0];
            }
        }
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
        const int ni = (int)L.size1[i] + 1, nj = (int)L.size1[j] + 1;
        // ---- output the level (Section 4 step 4) -------------------------
        if (w == 0 && tid == 0) {
            int4 rec;
            rec.x = i;
            rec.y = j;
            rec.z = __float_as_int(h);
            rec.w = ni + nj;
            reinterpret_cast<int4 *>(I.out)[s] = rec;
            // After a hand-over each merge is the global minimum of its state,
            // like one round of the round engine: its sort key continues the
            // round count.
            if (keys) keys[s] = ((uint64_t)ord32(h) << 32) | ((uint64_t)i << 16) | (uint64_t)(round0 + (s - s0));
        }
        if (s == n - 2) break;

        // ---- loads of rows i and j for the first batch of owned columns ---
        // (lazy mirror: D_ik from row i or from row k, whichever was written
        // last; without it both steps are 0 and the row is read)
        float *Di = D + (size_t)i * n;
        const uint32_t ti = lazy ? L.wstep[i] : 0u, tj = lazy ? L.wstep[j] : 0u;
        float a[U], bv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int lq = wv + u * W;
            const int k = lq < own_ch ? chunk_of(lq, g, w) * 64 + lane : n;
            const uint32_t tk = lazy && k < n ? L.wstep[k] : 0u;
            a[u] = k < n ? D[pair_at(i, k, ti, tk, n)] : 0.0f;
            bv[u] = k < n ? D[pair_at(j, k, tj, tk, n)] : 0.0f;
        }
        // ---- retire j (Section 5.3 step 6); queue rows whose partner is i or j
        if (tid == 0) {
            atomicAnd(&L.amask[j >> 5], ~(1u << (j & 31)));
            if (owner_of_row(j, g) == w) L.cache[local_of_row(j, g)] = kEmptyRow;
        }
        for (int li = tid; li < (scan ? 0 : own_ch * 64); li += B) {
            const int k = row_of_local(li, g, w);
            if (k >= n || k == i || k == j) continue;
            uint64_t c = L.cache[li];
            if (k == i_prev) {
                c = ip_entry;
                L.cache[li] = c;
            }
            if (defer) {
                const int nn = (int)((c >> 16) & 0xFFFFull);
                if (!(c & kStale) && (uint32_t)(c >> 32) != kEmptyOrd && (nn == i || nn == j))
                    L.cache[li] = (c & kHi32) | kStale;  // keeps its old minimum as a bound
                continue;
            }
            const int nn = (int)((c >> 16) & 0xFFFFull);
            if ((uint32_t)(c >> 32) != kEmptyOrd && (nn == i || nn == j)) {
                L.cache[li] = kEmptyRow;  // rebuilt by the rescan below
                L.rlist[atomicAdd(&s_nresc, 1u)] = (uint16_t)li;
            }
        }
        __syncthreads();
        if (prof) st.lap(kPhUpdate);
        const uint32_t nresc = defer ? 0u : s_nresc;
        if (nresc) {
            rescan_rows<B>(D, n, g, w, L, nresc, i, st.rescan_elems);
            if (!scan) __syncthreads();  // rescanned entries are final before the update folds them
        }
        if (prof) st.lap(kPhRescan);

        // ---- Lance-Williams update of row/column i (Section 4 step 3) -----
        float ai = 0.0f, aj = 0.0f, bij = 0.0f;
        if (link == HAC_AVERAGE || link == HAC_CENTROID) {
            const double sum = (double)(ni + nj);
            ai = (float)((double)ni / sum);
            aj = (float)((double)nj / sum);
            bij = (float)(-((double)ni * (double)nj) / (sum * sum));
        }
        uint64_t q2 = kEmpty;
        uint64_t pc = kEmpty;  // this workgroup's candidates for epoch e+1
        for (int lq0 = wv; lq0 < own_ch; lq0 += W * U) {
            if (lq0 != wv) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int lq = lq0 + u * W;
                    const int k = lq < own_ch ? chunk_of(lq, g, w) * 64 + lane : n;
                    const uint32_t tk = lazy && k < n ? L.wstep[k] : 0u;
                    a[u] = k < n ? D[pair_at(i, k, ti, tk, n)] : 0.0f;
                    bv[u] = k < n ? D[pair_at(j, k, tj, tk, n)] : 0.0f;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int lq = lq0 + u * W;
                if (lq >= own_ch) break;
                const int k = chunk_of(lq, g, w) * 64 + lane;
                if (k >= n || k == i || k == j || !is_live(L.amask, k)) continue;
                const int nk = link == HAC_WARD ? (int)L.size1[k] + 1 : 1;
                const float v = lw_update(link, a[u], bv[u], h, ni, nj, nk, ai, aj, bij);
                // The column half D[k][i] is written only without the lazy
                // mirror (with it, row i is now the later-written copy).
                if (g > 1) {
                    // Other workgroups read these entries after the next
                    // exchange: agent-scope stores put them at the device's
                    // point of coherence, so the exchange needs no L2 write
                    // back (which would wait for every dirty line of the XCD).
                    __hip_atomic_store(reinterpret_cast<uint32_t *>(Di + k), __float_as_uint(v), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    if (!lazy)
                        __hip_atomic_store(reinterpret_cast<uint32_t *>(D + (size_t)k * n + i), __float_as_uint(v),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    Di[k] = v;
                    if (!lazy) D[(size_t)k * n + i] = v;
                }
                st.update_elems++;
                const uint64_t key = ((uint64_t)ord32(v) << 32) | ((uint64_t)i << 16);
                if (scan) continue;  // every row is scanned again below
                if (k > i) q2 = umin64(q2, ((uint64_t)ord32(v) << 32) | ((uint64_t)k << 16));
                if (defer) {
                    // This lane is the only one touching the row's entry now;
                    // it also folds the final entry into the candidates, so
                    // no separate pass over the cache is needed.
                    uint64_t *ce = &L.cache[(lq * 64) + lane];
                    uint64_t c = *ce;
                    if (k < i) {  // the row's new entry at column i (see above)
                        c = umin64(c, (c & kStale) ? (((uint64_t)ord32(v) << 32) | kStale) : key);
                        *ce = c;
                    }
                    if ((uint32_t)(c >> 32) != kEmptyOrd)
                        pc = umin64(pc, (c & kHi32) | ((uint64_t)k << 16) | ((c >> 16) & 0xFFFFull));
                } else {
                    uint64_t *ce = &L.cache[(lq * 64) + lane];
                    uint64_t c;
                    if (k < i)  // the row's new entry at column i (see above)
                        c = umin64(atomicMin(reinterpret_cast<unsigned long long *>(ce), (unsigned long long)key),
                                   key);
                    else
                        c = *ce;
                    if ((uint32_t)(c >> 32) != kEmptyOrd)
                        pc = umin64(pc, (c & kHi32) | ((uint64_t)k << 16) | ((c >> 16) & 0xFFFFull));
                }
            }
        }
        lds_min(&s_acc[b ^ 1][1], q2);  // row i's candidates for epoch e+1
        if (!scan) lds_min(&s_acc[b ^ 1][0], pc);
        // The update's stores (both halves) are complete before the next
        // exchange publishes them.
        barrier_stores_done();
        // Cluster i grows; every thread has read size1[i] and size1[j] for
        // this merge, and nothing reads them again before the next one.
        if (tid == 0) {
            L.size1[i] = (uint16_t)(ni + nj - 1);
            if (lazy) L.wstep[i] = (uint16_t)(s + 1);  // read again only after the next barrier
            st.rescans += nresc;
            s_nresc = 0;
        }
        if (prof) st.lap(kPhCand);

        if (scan) {
            // ---- the paper's step 1 literally: every workgroup scans the
            // live upper part of all its rows for the next argmin ---------
            if (tid == 0)
                for (int q = 0; q < 4; ++q) s_acc[b][q] = s_acc[b ^ 1][q] = kEmpty;
            barrier_stores_done();
            // Every workgroup's updated entries are in place (epoch e+1).
            ++e;
            b = e & 1;
            if (g > 1 && !group_exchange<B>(I, g, w, e, ctl, timeout, false)) return;
            for (int li = tid; li < own_ch * 64; li += B) {
                const int k = row_of_local(li, g, w);
                L.cache[li] = kEmptyRow;
                if (k < n && is_live(L.amask, k)) L.rlist[atomicAdd(&s_nresc, 1u)] = (uint16_t)li;
            }
            __syncthreads();
            const uint32_t nscan = s_nresc;
            rescan_rows<B>(D, n, g, w, L, nscan, -1, st.rescan_elems);
            __syncthreads();
            if (tid == 0) {
                st.rescans += nscan;
                s_nresc = 0;
            }
            fold_candidates<B>(L, n, g, w, own_ch, -1, &s_acc[b ^ 1][0]);
        }
        i_prev = i;
    }
}

template <int B>
__device__ void flush_stats(Control *ctl, Stats &st) {
    unsigned long long a = block_sum<B>(st.rescans);
    unsigned long long b = block_sum<B>(st.rescan_elems);
    unsigned long long c = block_sum<B>(st.update_elems);
    if (threadIdx.x == 0) {
        atomicAdd(&ctl->rescans, a);
        atomicAdd(&ctl->rescan_elems, b);
        atomicAdd(&ctl->update_elems, c);
        if (st.forced) atomicAdd(&ctl->forced, st.forced);
        for (int p = 0; p < kPhases; ++p) {
            atomicAdd(&ctl->prof_sum[p], st.prof[p]);
            atomicMax(&ctl->prof_max[p], st.prof[p]);
        }
    }
}

// Set-up for the single-instance path: workgroup (x, R) handles the strip of
// up to kSetupStrip tiles (R, R + x*kSetupStrip ...) of row block R, so that
// the pass over the upper triangle has many workgroups per CU; each row's
// first minimum is the atomic minimum of its strips' minima in rowkey
// (filled with kEmpty beforehand).
__global__ __launch_bounds__(kSetupBlock) void k_setup(Instance I, const float *src) {
    __shared__ float tile[kTile * (kTile + 1)];
    const int n = I.n, T = (n + 63) >> 6;
    const int R = (int)blockIdx.y;
    const int c0 = R + (int)blockIdx.x * kSetupStrip;
    if (c0 >= T) return;
    const int c1 = c0 + kSetupStrip < T ? c0 + kSetupStrip : T;
    uint32_t bad = 0;
    setup_block<kSetupBlock>(src, I.D, n, R, c0, c1, tile, bad, [&](int r, uint64_t v) {
        const int row = R * 64 + r;
        if (row < n && v != kEmpty)
            atomicMin(reinterpret_cast<unsigned long long *>(I.rowkey + row), (unsigned long long)v);
    });
    if (bad) atomicOr(I.status, kErrInput);
}

template <int B, int kMode>
__global__ __launch_bounds__(B) void k_run(Instance I, Control *ctl, uint64_t timeout, Resume rs) {
    extern __shared__ __align__(16) uint8_t smem[];
    Stats st;
    if (threadIdx.x == 0 && (I.flags & kFlagProfile)) st.mark = wall_clock64();
    const int g = (int)gridDim.x, w = (int)blockIdx.x, n = I.n;
    const int own_cap = ((((n + 63) >> 6) + g - 1) / g) * 64;
    const Lds L = carve(smem, n, own_cap, false);
    // The set-up kernel (and the round engine, if queued behind it) has
    // finished: the status word is final and the same for every thread of
    // every workgroup.
    const uint32_t st0 = __hip_atomic_load(I.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (st0 & kErrInput) return;
    if ((I.flags & kFlagAfterRounds) && !(st0 & kHandover)) return;
    const int own_ch = own_chunks(n, g, w);
    if (!(I.flags & kFlagAfterRounds)) {
        init_masks<B>(L, n);
        for (int li = threadIdx.x; li < own_cap; li += B) {
            const int k = row_of_local(li, g, w);
            const uint64_t v = (li < own_ch * 64 && k < n) ? I.rowkey[k] : kEmpty;
            L.cache[li] = v == kEmpty ? kEmptyRow : v;
        }
        __syncthreads();
        merge_loop<B, kMode>(I, g, w, L, ctl, timeout, st, 0u);
    } else {
        // Resume where the round engine stopped: its live slots and sizes,
        // and every own live row's minimum over the live columns to its
        // right, rescanned from the current matrix.
        const int s0 = (int)rs.state[0], round0 = (int)rs.state[1];
        const int mask_words = (n + 31) >> 5;
        for (int q = threadIdx.x; q < mask_words; q += B) L.amask[q] = rs.live[q];
        for (int k = threadIdx.x; k < n; k += B) L.size1[k] = (uint16_t)(rs.size[k] - 1);
        if (threadIdx.x == 0) s_nresc = 0;
        __syncthreads();
        for (int li = threadIdx.x; li < own_cap; li += B) {
            const int k = row_of_local(li, g, w);
            L.cache[li] = kEmptyRow;
            if (li < own_ch * 64 && k < n && is_live(L.amask, k)) L.rlist[atomicAdd(&s_nresc, 1u)] = (uint16_t)li;
        }
        __syncthreads();
        rescan_rows<B>(I.D, n, g, w, L, s_nresc, -1, st.rescan_elems);
        __syncthreads();
        if (threadIdx.x == 0) {
            st.rescans += s_nresc;
            s_nresc = 0;
        }
        __syncthreads();
        merge_loop<B, kMode>(I, g, w, L, ctl, timeout, st, 0u, s0, rs.keys, round0);
    }
    flush_stats<B>(ctl, st);
}

// One batch instance on workgroup w of a group of g (g = 1: the whole
// instance on this workgroup), including its set-up.  Returns when done.
// Deferred rescans: with the lazy mirror a rescan reads scattered entries, and
// stale rows settled together in forced rounds cost less than rescanning at
// every merge.  U: update batch depth (chunks per wave loaded at once).
template <int B, int U = upd_batch<B>()>
__device__ void batch_instance(const Instance &I, int g, int w, uint8_t *smem, Control *ctl,
                               uint64_t timeout, Stats &st, uint32_t epoch_base = 0) {
    const int n = I.n;
    if (threadIdx.x == 0 && (I.flags & kFlagProfile)) st.mark = wall_clock64();
    const int own_ch = own_chunks(n, g, w);
    const int own_cap = ((((n + 63) >> 6) + g - 1) / g) * 64;
    const Lds L = carve(smem, n, own_cap, (I.flags & kFlagLazy) != 0);
    for (int li = threadIdx.x; li < own_cap; li += B) L.cache[li] = kEmptyRow;
    __syncthreads();
    uint32_t bad = 0;
    for (int lq = 0; lq < own_ch; ++lq) {
        const int R = chunk_of(lq, g, w);
        setup_block<B>(I.D, I.D, n, R, R, (n + 63) >> 6, L.tile, bad, [&](int r, uint64_t v) {
            L.cache[lq * 64 + r] = v == kEmpty ? kEmptyRow : v;
        });
    }
    // This workgroup's verdict on its part of the input, shared through LDS.
    uint64_t okv = bad ? 0 : kEmpty, dummy = kEmpty;
    block_min2<B>(okv, dummy);
    if (okv == 0 && threadIdx.x == 0) atomicOr(I.status, kErrInput);
    uint32_t epoch0 = 0;
    if (g > 1) {
        // The group's set-up (mirror, input check) must be complete and
        // visible before any merge: one exchange with empty candidates, after
        // which every thread reads the final status word.
        const uint32_t e = epoch_base + 1u;
        if (threadIdx.x == 0) s_acc[e & 1][0] = s_acc[e & 1][1] = s_acc[e & 1][2] = s_acc[e & 1][3] = kEmpty;
        barrier_stores_done();  // the mirror (and a served job's copy-in) stores are complete
        if (!group_exchange<B>(I, g, w, e, ctl, timeout, true)) return;
        epoch0 = e;
        if (__hip_atomic_load(I.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrInput) return;
    } else if (okv == 0) {
        return;
    }
    init_masks<B>(L, n);  // size1 shares space with the tile
    __syncthreads();
    merge_loop<B, kLoopDefer, U, true>(I, g, w, L, ctl, timeout, st, epoch0);
}

// Batch: the first `ngroups` entries of `order` are run by fixed groups of
// workgroups (task t on workgroups gbase[t] .. gbase[t]+gsize[t]-1); every
// workgroup then takes the remaining entries one at a time from a queue
// (largest instances first).  Launched cooperatively when ngroups > 0 so that
// the members of a group are co-resident.  U: chunks per wave in each update
// batch (a plan parameter).
template <int B, int U>
__global__ __launch_bounds__(B) void k_batch(const Instance *__restrict__ insts,
                                             const int32_t *__restrict__ order, int count,
                                             const int32_t *__restrict__ gbase,
                                             const int32_t *__restrict__ gsize, int ngroups,
                                             Control *ctl, uint64_t timeout) {
    extern __shared__ __align__(16) uint8_t smem[];
    Stats st;
    const int wg = (int)blockIdx.x;
    for (int t = 0; t < ngroups; ++t) {
        const int base = gbase[t], g = gsize[t];
        if (wg >= base && wg < base + g) {
            const Instance I = insts[order[t]];
            if (I.n > 1) batch_instance<B, U>(I, g, wg - base, smem, ctl, timeout, st);
            __syncthreads();
        }
    }
    for (;;) {
        if (threadIdx.x == 0) s_inst = ngroups + (int)atomicAdd(&ctl->next, 1u);
        __syncthreads();
        const int q = s_inst;
        __syncthreads();
        if (q >= count) break;
        const Instance I = insts[order[q]];
        if (I.n > 1) batch_instance<B, U>(I, 1, 0, smem, ctl, timeout, st);
        __syncthreads();
    }
    flush_stats<B>(ctl, st);
}

// Serving: claim the next published entry (thread 0 only).  One workgroup
// at a time holds the token and polls the host's tail, mirroring it into
// device memory where the others poll it cheaply.  Returns false once the
// host has asked to stop and no entry is left.
__device__ bool serve_claim(ServeHost *host, const ServeEntry *ring, uint32_t cap, ServeDev *dev,
                            ServeEntry *out, uint64_t idle_ticks) {
    // Idle workgroups poll rarely, with relaxed loads only (an acquire would
    // invalidate their XCD's L2 on every poll), and try for the poller token
    // only when it looks free.  Ordering is taken once, after a claim or a
    // stop.
    bool poller = false;
    const uint64_t t0 = wall_clock64();
    for (uint32_t it = 1;; ++it) {
        const uint32_t stop = __hip_atomic_load(&dev->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (stop) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        // stop is read before tail: the poller raises stop only after it has
        // mirrored the final tail, so a stopped reader sees every entry.
        const unsigned long long t = __hip_atomic_load(&dev->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long h = __hip_atomic_load(&dev->head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (h < t) {
            if (__hip_atomic_compare_exchange_strong(&dev->head, &h, h + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)) {
                if (poller) __hip_atomic_store(&dev->token, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&dev->claims, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                // The entry lives in host memory: read it word by word with
                // system-scope loads (never through a cache).
                const unsigned long long *src =
                    reinterpret_cast<const unsigned long long *>(ring + (size_t)(h % cap));
                unsigned long long *dst = reinterpret_cast<unsigned long long *>(out);
                for (int q = 0; q < (int)(sizeof(ServeEntry) / 8); ++q)
                    dst[q] = __hip_atomic_load(src + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                return true;
            }
            continue;
        }
        if (stop) {
            if (poller) __hip_atomic_store(&dev->token, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        if (!poller && __hip_atomic_load(&dev->token, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
            uint32_t z = 0;
            poller = __hip_atomic_compare_exchange_strong(&dev->token, &z, 1u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
        }
        if (poller) {
            const unsigned long long ht = __hip_atomic_load(&host->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            if (ht > t) {
                __hip_atomic_fetch_max(&dev->tail, ht, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                continue;
            }
            if (__hip_atomic_load(&host->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) {
                // The host publishes nothing after asking to stop; re-read
                // its tail once more so that the mirror is final.
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                const unsigned long long hf =
                    __hip_atomic_load(&host->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_fetch_max(&dev->tail, hf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                release_agent();
                __hip_atomic_store(&dev->stop, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                continue;
            }
            __builtin_amdgcn_s_sleep(8);
        } else {
            // ~14 us between polls: a crowd of idle workgroups polling the
            // queue words (and trying for the token) every microsecond only
            // adds memory traffic beside the running jobs; a claim waits at
            // most this long.  Results do not depend on the interval.
            for (int z = 0; z < 4; ++z) __builtin_amdgcn_s_sleep(127);
        }
        // Safety net: the host stops an idle kernel long before this; if it
        // never does, stop as if it had (entries are still taken first).
        if ((it & 255u) == 0 && wall_clock64() - t0 > idle_ticks) {
            __hip_atomic_fetch_add(&dev->self_stops, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            release_agent();
            __hip_atomic_store(&dev->stop, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Host memory is read with system-scope loads: the same host buffer may hold
// another job's matrix than when this XCD's L2 last cached it.
__device__ __forceinline__ float ld_host(const float *p) {
    return __uint_as_float(__hip_atomic_load(reinterpret_cast<const uint32_t *>(p), __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_SYSTEM));
}

// Serving: workgroup w of a job's g copies from the job's host matrix
// (page-locked memory read over the bus; leading dimension ld) the strict
// upper triangle of the rows it owns, one wave per row with up to 16 loads in
// flight per lane.  Its set-up reads only these rows; the entries of other
// rows that its merge loop reads in its own columns are read after the
// set-up exchange with device-scope loads (multi-workgroup paths).
template <int B>
__device__ void copy_in_upper(const float *src, int64_t ld, float *D, int n, int g, int w) {
    constexpr int W = B / 64;
    constexpr int U = 16;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = wv; i < n - 1; i += W) {
        if (owner_of_row(i, g) != w) continue;
        const float *sr = src + (size_t)i * (size_t)ld;
        float *dr = D + (size_t)i * (size_t)n;
        for (int c0 = i + 1; c0 < n; c0 += 64 * U) {
            float v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = c0 + lane + 64 * u;
                v[u] = c < n ? ld_host(sr + c) : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = c0 + lane + 64 * u;
                if (c < n) dr[c] = v[u];
            }
        }
    }
}

// Serving kernel: every workgroup takes entries until the host stops it.
// A job on g workgroups has g consecutive entries; members are taken in
// publication order, so the earliest incomplete job always gets its members
// as workgroups free up.  Member 0 (the writer of the merge records) waits
// until every member has passed the last exchange, clears the job slot's
// device words and publishes seq << 32 | status in host memory after a
// system-scope release.
template <int B>
__global__ __launch_bounds__(B) void k_serve(ServeHost *host, const ServeEntry *ring, uint32_t cap,
                                             unsigned long long *done, ServeDev *dev, Control *ctl,
                                             uint64_t timeout, uint64_t idle_ticks) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ ServeEntry s_job;
    __shared__ uint32_t s_status;
    Stats st;
    for (;;) {
        if (threadIdx.x == 0) s_inst = serve_claim(host, ring, cap, dev, &s_job, idle_ticks) ? 1 : 0;
        __syncthreads();
        if (s_inst == 0) break;
        // The entry is the same for the whole workgroup: keep it in scalar
        // registers.  s_job stays unchanged until the next claim.
        ServeEntry e;
        {
            const uint32_t *src = reinterpret_cast<const uint32_t *>(&s_job);
            uint32_t *dst = reinterpret_cast<uint32_t *>(&e);
            for (int q = 0; q < (int)(sizeof(ServeEntry) / 4); ++q)
                dst[q] = (uint32_t)__builtin_amdgcn_readfirstlane((int)src[q]);
        }
        // Host memory may have changed since this kernel last read it: drop
        // cached lines before reading the job's matrix.
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        if (e.inst.n > 1) {
            copy_in_upper<B>(e.src, e.ld, e.inst.D, e.inst.n, e.g, e.rank);
            __syncthreads();
            batch_instance<B>(e.inst, e.g, e.rank, smem, ctl, timeout, st);
        }
        // Every wave's stores to the job's matrix are complete before thread
        // 0's release below: the arena region is reused by later jobs, which
        // may run on other XCDs, so no dirty line of this job may be left
        // behind in this XCD's L2 to be written back over them.
        barrier_stores_done();
        uint32_t *words = e.inst.status;  // [0] status, [1] members done
        if (threadIdx.x == 0) {
            release_system();
            __hip_atomic_fetch_add(words + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_inst = 1;
            if (e.rank == 0) {
                // Member 0 wrote the merge records, so it publishes the
                // completion: its own earlier writes to host memory are
                // ordered before its completion word, which another
                // member's would not be.  The others are at most one
                // exchange behind.
                const uint64_t t0 = wall_clock64();
                while (__hip_atomic_load(words + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (uint32_t)e.g) {
                    if (wall_clock64() - t0 > timeout) {
                        atomicOr(words, kErrTimeout);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                s_status = __hip_atomic_load(words, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_inst = 2;
            }
        }
        __syncthreads();
        if (s_inst == 2) {
            // Every member is past its last exchange: clear the slots for the
            // job slot's next use, then the words, then publish.
            if (e.g > 1) {
                const int words64 = 2 * (e.g + 1) * kSlotStride;
                for (int q = threadIdx.x; q < words64; q += B) {
                    if ((q % kSlotStride) < 3)
                        __hip_atomic_store(e.inst.slots + q, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            barrier_stores_done();  // the cleared slots are in place before the job slot is handed back
            if (threadIdx.x == 0) {
                __hip_atomic_store(words, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(words + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                release_system();
                __hip_atomic_store(done + e.job, ((unsigned long long)e.seq << 32) | s_status, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
    }
    if (threadIdx.x == 0) __hip_atomic_fetch_add(&dev->exits, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    flush_stats<B>(ctl, st);
}

__global__ void k_zero(uint32_t *p, size_t words) {
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < words;
         q += (size_t)gridDim.x * blockDim.x)
        p[q] = 0u;
}

__global__ void k_fill_ones(uint32_t *p, size_t words) {
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < words;
         q += (size_t)gridDim.x * blockDim.x)
        p[q] = 0xFFFFFFFFu;
}

}  // namespace

// The allocation-free entry point's scratch (see engine_scratch).  In host
// code this name is only a handle for hipGetSymbolAddress: kernels receive
// the address that call returns, never the name.
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

hipError_t engine_scratch(void **ptr) { return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch)); }

int own_rows(int n, int g) { return ((((n + 63) >> 6) + g - 1) / g) * 64; }

size_t lds_bytes(int n, int own, bool in_kernel_setup, bool lazy) {
    const size_t mask = (((size_t)(n + 31) / 32 + 3) / 4 * 4) * 4;
    const size_t sizes = lazy ? (size_t)((n + 3) & ~3) * 2 + (size_t)n * 2 : (size_t)n * 2;  // size1 (+ wstep)
    const size_t tile = in_kernel_setup ? (size_t)kTile * (kTile + 1) * 4 : 0;
    return (size_t)own * 8 + (size_t)own * 2 + mask + (sizes > tile ? sizes : tile);
}

template <int B>
static const void *run_kernel_b(int mode) {
    switch (mode) {
    case kLoopDefer: return reinterpret_cast<const void *>(&k_run<B, kLoopDefer>);
    case kLoopScan: return reinterpret_cast<const void *>(&k_run<B, kLoopScan>);
    default: return reinterpret_cast<const void *>(&k_run<B, kLoopCached>);
    }
}

static const void *run_kernel(int block, int mode) {
    switch (block) {
    case 256: return run_kernel_b<256>(mode);
    case 512: return run_kernel_b<512>(mode);
    default: return run_kernel_b<1024>(mode);
    }
}

hipError_t engine_setup(size_t max_lds, size_t *usable) {
    // Dynamic LDS may use what the static LDS of the kernels leaves free.
    size_t static_max = 0;
    const void *fns[] = {run_kernel(256, kLoopCached),   run_kernel(512, kLoopCached),
                         run_kernel(1024, kLoopCached),  run_kernel(256, kLoopDefer),
                         run_kernel(512, kLoopDefer),    run_kernel(1024, kLoopDefer),
                         run_kernel(256, kLoopScan),     run_kernel(512, kLoopScan),
                         run_kernel(1024, kLoopScan),    reinterpret_cast<const void *>(&k_batch<256, 8>),
                         reinterpret_cast<const void *>(&k_batch<1024, 2>),
                         reinterpret_cast<const void *>(&k_batch<1024, 4>), reinterpret_cast<const void *>(&k_serve<256>),
                         reinterpret_cast<const void *>(&k_serve<1024>)};
    for (const void *fn : fns) {
        hipFuncAttributes a;
        hipError_t e = hipFuncGetAttributes(&a, fn);
        if (e != hipSuccess) return e;
        static_max = a.sharedSizeBytes > static_max ? a.sharedSizeBytes : static_max;
    }
    const size_t dyn = max_lds > static_max ? max_lds - static_max : 0;
    for (const void *fn : fns) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
        if (e != hipSuccess) return e;
    }
    *usable = dyn;
    return hipSuccess;
}


// Batch kernel variants: 256 threads with 8-chunk update batches; 1024
// threads with 2 or 4 (4 loads an n = 4096 instance's rows in one batch at
// the cost of some register spill; the plan search picks).
static const void *batch_kernel(int block, int upd) {
    if (block != 1024) return reinterpret_cast<const void *>(&k_batch<256, 8>);
    return upd == 2 ? reinterpret_cast<const void *>(&k_batch<1024, 2>)
                    : reinterpret_cast<const void *>(&k_batch<1024, 4>);
}

int engine_occupancy(size_t lds, int block, bool batch, int32_t run_flags) {
    int blocks = 0;
    const int mode = (run_flags & kFlagScan) ? kLoopScan : (run_flags & kFlagDefer) ? kLoopDefer : kLoopCached;
    const void *fn = batch ? batch_kernel(block, 4) : run_kernel(block, mode);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, block, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return blocks;
}

static const void *serve_kernel(int block) {
    return block == 1024 ? reinterpret_cast<const void *>(&k_serve<1024>)
                         : reinterpret_cast<const void *>(&k_serve<256>);
}

int serve_occupancy(size_t lds, int block) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, serve_kernel(block), block, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return blocks;
}

hipError_t launch_serve(const ServeLaunch &sl, Control *ctl, uint64_t timeout_ticks, hipStream_t stream) {
    ServeHost *a0 = sl.host;
    const ServeEntry *a1 = sl.ring;
    uint32_t a2 = sl.cap;
    unsigned long long *a3 = sl.done;
    ServeDev *a4 = sl.dev;
    Control *a5 = ctl;
    uint64_t a6 = timeout_ticks;
    uint64_t a7 = sl.idle_ticks;
    void *args[] = {&a0, &a1, &a2, &a3, &a4, &a5, &a6, &a7};
    return hipLaunchCooperativeKernel(serve_kernel(sl.block), dim3(sl.grid), dim3(sl.block), args,
                                      (unsigned)sl.lds, stream);
}

hipError_t launch_zero(void *p, size_t words, hipStream_t stream) {
    if (words == 0) return hipSuccess;
    int grid = (int)((words + 255) / 256);
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, stream, (uint32_t *)p, words);
    return hipGetLastError();
}

hipError_t launch_setup(const Instance &inst, const float *src, hipStream_t stream) {
    const int T = (inst.n + 63) / 64;
    {
        const size_t words = (size_t)inst.n * 2;  // rowkey: n u64 set to kEmpty
        int grid = (int)((words + 255) / 256);
        if (grid > 1024) grid = 1024;
        hipLaunchKernelGGL(k_fill_ones, dim3(grid), dim3(256), 0, stream, reinterpret_cast<uint32_t *>(inst.rowkey),
                           words);
    }
    hipLaunchKernelGGL(k_setup, dim3((T + kSetupStrip - 1) / kSetupStrip, T), dim3(kSetupBlock), 0, stream, inst,
                       src);
    return hipGetLastError();
}

hipError_t launch_run(const Instance &inst, const float *src, int g, int block, Control *ctl,
                      uint64_t timeout_ticks, hipStream_t stream, hipEvent_t setup_done) {
    hipError_t e = launch_setup(inst, src, stream);
    if (e != hipSuccess) return e;
    if (setup_done) {
        e = hipEventRecord(setup_done, stream);
        if (e != hipSuccess) return e;
    }
    return launch_merge(inst, g, block, ctl, timeout_ticks, stream);
}

hipError_t launch_merge(const Instance &inst, int g, int block, Control *ctl, uint64_t timeout_ticks,
                        hipStream_t stream, const Resume &rs) {
    const size_t lds = lds_bytes(inst.n, own_rows(inst.n, g), false);
    Instance a0 = inst;
    Control *a1 = ctl;
    uint64_t a2 = timeout_ticks;
    Resume a3 = rs;
    void *args[] = {&a0, &a1, &a2, &a3};
    const int mode = (inst.flags & kFlagScan) ? kLoopScan : (inst.flags & kFlagDefer) ? kLoopDefer : kLoopCached;
    if (g == 1) return hipLaunchKernel(run_kernel(block, mode), dim3(1), dim3(block), args, lds, stream);
    return hipLaunchCooperativeKernel(run_kernel(block, mode), dim3(g), dim3(block), args, (unsigned)lds, stream);
}

hipError_t launch_batch(const BatchLaunch &b, Control *ctl, uint64_t timeout_ticks, hipStream_t stream) {
    const Instance *a0 = b.insts;
    const int32_t *a1 = b.order;
    int a2 = b.count;
    const int32_t *a3 = b.gbase;
    const int32_t *a4 = b.gsize;
    int a5 = b.ngroups;
    Control *a6 = ctl;
    uint64_t a7 = timeout_ticks;
    void *args[] = {&a0, &a1, &a2, &a3, &a4, &a5, &a6, &a7};
    if (b.ngroups > 0)
        return hipLaunchCooperativeKernel(batch_kernel(b.block, b.upd), dim3(b.grid), dim3(b.block), args,
                                          (unsigned)b.lds, stream);
    return hipLaunchKernel(batch_kernel(b.block, b.upd), dim3(b.grid), dim3(b.block), args, b.lds, stream);
}

static hipError_t add_zero_node(hipGraph_t g, hipGraphNode_t *node, const hipGraphNode_t *dep, size_t ndep,
                                void *p, size_t words, void **argbuf) {
    uint32_t **a0 = reinterpret_cast<uint32_t **>(argbuf[0]);
    size_t *a1 = reinterpret_cast<size_t *>(argbuf[1]);
    *a0 = reinterpret_cast<uint32_t *>(p);
    *a1 = words;
    unsigned grid = (unsigned)((words + 255) / 256);
    if (grid > 1024) grid = 1024;
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void *>(&k_zero);
    kp.gridDim = dim3(grid);
    kp.blockDim = dim3(256);
    kp.sharedMemBytes = 0;
    kp.kernelParams = argbuf;
    kp.extra = nullptr;
    return hipGraphAddKernelNode(node, g, dep, ndep, &kp);
}

hipError_t build_batch_graph(const BatchLaunch &b, Control *ctl, uint64_t timeout_ticks, void *up_dst,
                             const void *up_src, size_t up_bytes, void *z0, size_t z0_words, void *z1,
                             size_t z1_words, hipGraphExec_t *exec) {
    *exec = nullptr;
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return e;
    hipGraphNode_t last = nullptr, node = nullptr;
    // Kernel arguments are copied when the node is added.
    uint32_t *zp = nullptr;
    size_t zw = 0;
    void *zargs[] = {&zp, &zw};
    e = hipGraphAddMemcpyNode1D(&node, g, nullptr, 0, up_dst, up_src, up_bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        last = node;
        if (z0_words) {
            e = add_zero_node(g, &node, &last, 1, z0, z0_words, zargs);
            if (e == hipSuccess) last = node;
        }
    }
    if (e == hipSuccess && z1_words) {
        e = add_zero_node(g, &node, &last, 1, z1, z1_words, zargs);
        if (e == hipSuccess) last = node;
    }
    if (e == hipSuccess) {
        const Instance *a0 = b.insts;
        const int32_t *a1 = b.order;
        int a2 = b.count;
        const int32_t *a3 = b.gbase;
        const int32_t *a4 = b.gsize;
        int a5 = b.ngroups;
        Control *a6 = ctl;
        uint64_t a7 = timeout_ticks;
        void *args[] = {&a0, &a1, &a2, &a3, &a4, &a5, &a6, &a7};
        hipKernelNodeParams kp{};
        kp.func = const_cast<void *>(batch_kernel(b.block, b.upd));
        kp.gridDim = dim3(b.grid);
        kp.blockDim = dim3(b.block);
        kp.sharedMemBytes = (unsigned)b.lds;
        kp.kernelParams = args;
        kp.extra = nullptr;
        e = hipGraphAddKernelNode(&node, g, &last, 1, &kp);
        if (e == hipSuccess && b.ngroups > 0) {
            hipKernelNodeAttrValue v{};
            v.cooperative = 1;
            e = hipGraphKernelNodeSetAttribute(node, hipKernelNodeAttributeCooperative, &v);
        }
    }
    if (e == hipSuccess) e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) *exec = nullptr;
    return e;
}

}  // namespace hac
