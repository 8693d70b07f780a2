// Round engine: single and complete linkage by rounds of merges.
//
// The merge list is the one of Section 4 (steps 1-4): n-1 times, merge the
// pair of live clusters with the lexicographically smallest key
// (D, i, j), i < j, keep slot i.  For single and complete linkage the
// Lance-Williams update is min / max (Table 1), exact in fp32 and independent
// of the order in which merges are applied, and Section 2.1's remark that
// single linkage is Prim's minimum spanning tree in disguise points the way:
// many merges of such a hierarchy are independent of each other and can be
// made at once.  Which ones, exactly:
//
//  * Complete linkage.  With the survivor keeping the smaller slot, the key
//    order is reducible: after merging i and j, key(i+j, k) >=
//    min(key(i, k), key(j, k)) holds exactly (the max keeps or raises the
//    value, and the pair's index part (min(i,k), max(i,k)) is that of
//    key(i, k)).  So every reciprocal-nearest-neighbour pair under the key
//    order (a's smallest key is with b and b's with a) is a merge of the
//    sequential run, with the same record, and all of them can be merged
//    in one round.  The sequential run's keys then strictly increase, so
//    sorting all records by (h, i, round) gives its order.
//  * Single linkage.  min can lower a key's index part (a tie at the same
//    value moves from column j to the smaller i), so reducibility in key
//    order fails under ties.  A round merges the global smallest key (the
//    sequential run's next merge) and every reciprocal pair whose value is
//    the only minimum of both rows (strict): such a pair is isolated at its
//    height now and later, so it is a merge of the sequential run with the
//    same record; within one height and survivor, merges appear in the run
//    in round order.  Sorting by (h, i, round) again gives the order.
//
// Per round, three phases separated by grid barriers (every workgroup is
// co-resident; cooperative launch):
//   A  detect: each workgroup reads the cached full-row minimum of its rows
//      (rk: ord(value):32 | partner:16, ties to the smallest partner) and
//      claims the reciprocal (and, for single, strict) pairs, writes their
//      merge records, and publishes its rows' smallest pair key.
//   B  update: every workgroup loads the round's pairs (plus the global
//      smallest key if it was not claimed) and takes (64 columns x up to 64
//      pairs) units over the columns of clusters not merged this round:
//      v = min/max(D[i][c], D[j][c]) written to both D[i][c] and D[c][i].
//      The entry between two clusters merged in the same round, p and q, is
//      min/max of the four entries between their members, computed once by
//      one thread per unordered pair {p, q}; no other thread of the phase
//      touches those entries.  Rows whose cached
//      partner merged: complete -> queued for a rescan; single -> the
//      partner moves to i (the value cannot change) and the count of
//      entries equal to the minimum drops when both merged entries had it.
//   C  refresh: retire the j's, rescan the survivors' rows and the queued
//      rows (full rows, counting the entries equal to the minimum).
// A last kernel writes the records in merge order (rank of each record's
// key among all keys).
#include <hip/hip_runtime.h>

#include "hac_dev.h"
#include "hac_rounds.h"

namespace hac {
namespace {

constexpr uint64_t kNone = ~0ull;
constexpr int B = kRoundsBlock;
constexpr int W = B / 64;
constexpr int kPairsPerUnit = 64;   // most pairs one wave applies to its 64 columns
constexpr int kUnroll = 4;          // pairs in flight per lane
constexpr int kMaskWords = (HAC_MAX_N + 31) / 32;

__device__ __forceinline__ int partner_of(uint64_t e) { return (int)((e >> 16) & 0xFFFFull); }
__device__ __forceinline__ uint32_t value_of(uint64_t e) { return (uint32_t)(e >> 32); }

__device__ __forceinline__ float lw_minmax(int link, float a, float b) {
    return link == HAC_SINGLE ? fminf(a, b) : fmaxf(a, b);
}

__shared__ uint32_t s_live[kMaskWords];          // live bitmask of all slots (same on every workgroup)
__shared__ int2 s_pair[kRoundsMaxPairs + 1];     // this round's pairs (i, j)
__shared__ uint64_t s_red[W];
__shared__ int s_np, s_p0;

__device__ __forceinline__ bool live_at(int c) { return (s_live[c >> 5] >> (c & 31)) & 1u; }

// Grid barrier of the round engine (see hac_dev.h).
__device__ __forceinline__ bool grid_sync(RoundsCtl *rc, Control *ctl, uint32_t &gen, uint32_t G, uint64_t timeout,
                                          bool stall = false) {
    return hac::grid_sync(&rc->bar, &rc->abort, &ctl->error, kErrTimeout, gen, G, timeout, stall);
}

template <class T>
__device__ T block_min(T v) {
    v = wave_min(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) s_red[wv] = v;
    __syncthreads();
    T r = s_red[0];
#pragma unroll
    for (int q = 1; q < W; ++q) r = r < s_red[q] ? r : s_red[q];
    return r;
}

// Rescans are cut into segments of kSeg columns, one wave each, so that a
// row is rescanned by many waves at once.  A segment folds its result into
// the row's words with atomics: rk[r] = ord(min):32 | smallest column
// attaining it:16 (atomic minimum), cw[r] = ord(min):32 | number of columns
// attaining it:32 (the smaller value wins, equal values add their counts).
// Both start from kNone / kNoCount.
constexpr int kSeg = 2048;
constexpr uint64_t kNoCount = 0xFFFFFFFF00000000ull;

__device__ void fold_count(uint64_t *cw, uint32_t v, uint32_t c) {
    unsigned long long *q = reinterpret_cast<unsigned long long *>(cw);
    unsigned long long cur = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        const uint32_t cv = (uint32_t)(cur >> 32);
        if (v > cv) return;
        const unsigned long long nv = v < cv ? (((unsigned long long)v << 32) | c) : cur + c;
        if (__hip_atomic_compare_exchange_strong(q, &cur, nv, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
    }
}

// One wave: minimum and its count over the live columns c != r of segment
// `seg` of row r, folded into rk[r] and cw[r].
__device__ void rescan_segment(const float *__restrict__ D, int n, int r, int seg, uint64_t *rk, uint64_t *cw,
                               unsigned long long &elems) {
    const int lane = threadIdx.x & 63;
    const float *row = D + (size_t)r * n;
    uint32_t mv = 0xFFFFFFFFu;
    int mc = 0, mn = 0;
    auto take = [&](float x, int col) {
        const uint32_t o = ord32(x);
        if (o < mv) {
            mv = o;
            mc = col;
            mn = 1;
        } else if (o == mv) {
            ++mn;  // columns arrive in increasing order per lane: mc stays the smallest
        }
        ++elems;
    };
    const int c0 = seg * kSeg, c1 = min(n, c0 + kSeg);
    if ((n & 3) == 0) {
        constexpr int U = kSeg / 256;  // 16-byte loads per lane
        float4 x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = c0 + 4 * (u * 64 + lane);
            x[u] = c < c1 ? *reinterpret_cast<const float4 *>(row + c) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = c0 + 4 * (u * 64 + lane);
            if (c >= c1) continue;
            const int q = c >> 2;
            uint32_t m = (s_live[q >> 3] >> ((q & 7) * 4)) & 0xFu;
            if ((r >> 2) == q) m &= ~(1u << (r & 3));
            if (!m) continue;
            if (m & 1u) take(x[u].x, c);
            if (m & 2u) take(x[u].y, c + 1);
            if (m & 4u) take(x[u].z, c + 2);
            if (m & 8u) take(x[u].w, c + 3);
        }
    } else {
        constexpr int U = 8;
        for (int b0 = c0; b0 < c1; b0 += 64 * U) {
            float x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = b0 + u * 64 + lane;
                x[u] = c < c1 ? row[c] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = b0 + u * 64 + lane;
                if (c < c1 && c != r && live_at(c)) take(x[u], c);
            }
        }
    }
    const uint64_t mine = mn ? (((uint64_t)mv << 32) | ((uint64_t)mc << 16)) : kNone;
    const uint64_t best = wave_min(mine);
    const unsigned long long ties = wave_sum((mn && mv == value_of(best)) ? (unsigned long long)mn : 0ull);
    if (lane == 0 && best != kNone) {
        atomicMin(reinterpret_cast<unsigned long long *>(rk + r), (unsigned long long)best);
        fold_count(cw + r, value_of(best), (uint32_t)ties);
    }
}

struct Views {
    RoundsCtl *rc;
    uint64_t *rk;      // n row entries ord(min):32 | partner:16
    uint64_t *cw;      // n words ord(min):32 | count of entries equal to the minimum:32
    int32_t *size;     // n cluster sizes
    int32_t *role;     // n: +(p+1) survivor of pair p this round, -(p+1) retired, 0 otherwise
    int32_t *resc;     // rows queued for a rescan this round
    int2 *pairs;       // kRoundsMaxPairs claimed pairs
    uint64_t *k1;      // G smallest pair keys (one per workgroup)
    int4 *rec;         // n-1 records in claim order
    uint64_t *key;     // their sort keys ord(h):32 | i:16 | round:16
    uint32_t *live;    // live mask left at a hand-over
};

__device__ Views views(char *ws, const RoundsLayout &Lo) {
    Views v;
    v.rc = reinterpret_cast<RoundsCtl *>(ws + Lo.ctl);
    v.rk = reinterpret_cast<uint64_t *>(ws + Lo.rk);
    v.cw = reinterpret_cast<uint64_t *>(ws + Lo.cnt);
    v.size = reinterpret_cast<int32_t *>(ws + Lo.size);
    v.role = reinterpret_cast<int32_t *>(ws + Lo.role);
    v.resc = reinterpret_cast<int32_t *>(ws + Lo.resc);
    v.pairs = reinterpret_cast<int2 *>(ws + Lo.pairs);
    v.k1 = reinterpret_cast<uint64_t *>(ws + Lo.k1);
    v.rec = reinterpret_cast<int4 *>(ws + Lo.rec);
    v.key = reinterpret_cast<uint64_t *>(ws + Lo.key);
    v.live = reinterpret_cast<uint32_t *>(ws + Lo.live);
    return v;
}

__device__ __forceinline__ uint32_t count_of(uint64_t w) { return (uint32_t)w; }

// Wall clock of thread 0 charged to phases (kFlagProfile): [0] first
// rescans, [1] waiting at grid barriers, [2] phase B, [3] phase C, [4] phase A.
struct Clock {
    bool on;
    uint64_t mark = 0;
    unsigned long long t[kPhases] = {0, 0, 0, 0, 0};
    __device__ void lap(int p) {
        if (on && threadIdx.x == 0) {
            const uint64_t now = wall_clock64();
            t[p] += now - mark;
            mark = now;
        }
    }
};

// The round engine hands the remaining merges over to the one-merge-per-step
// kernel queued behind it when the last kWindow rounds merged fewer than
// kWindow * kMinPerRound pairs: a round (three grid barriers) then costs more
// than the merges it makes would cost one exchange each.  That happens near
// the end of every run, when few clusters are left, and, for single linkage
// on input with many equal values, early: strict pairs become rare as
// clusters grow.  Each merge after the hand-over is the smallest key of its
// state, as the smallest key of a round is, so the records keep their order
// under (h, i, round).
constexpr int kWindow = 8;
constexpr int kMinPerRound = 12;

__global__ __launch_bounds__(kRoundsBlock) void k_rounds(float *D, int n, int link, uint32_t *status,
                                                         Control *ctl, char *ws, RoundsLayout Lo, uint64_t timeout,
                                                         int flags) {
    const Views V = views(ws, Lo);
    Clock clk{(flags & kFlagProfile) != 0};
    if (clk.on && threadIdx.x == 0) clk.mark = wall_clock64();
    const uint32_t G = gridDim.x;
    const int w = (int)blockIdx.x, tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int gw = w * W + wv, NW = (int)G * W;
    unsigned long long st_upd = 0, st_resc = 0, st_rows = 0;
    // The set-up kernel has finished: its verdict is final.
    if (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrInput) return;

    const int words = (n + 31) >> 5;
    for (int q = tid; q < words; q += B) {
        const int rem = n - q * 32;
        s_live[q] = rem >= 32 ? 0xFFFFFFFFu : ((1u << rem) - 1u);
    }
    for (int k = w * B + tid; k < n; k += (int)G * B) {
        V.size[k] = 1;
        V.role[k] = 0;
        V.rk[k] = kNone;
        V.cw[k] = kNoCount;
    }
    __syncthreads();
    uint32_t gen = 0;
    if (!grid_sync(V.rc, ctl, gen, G, timeout, (flags & kFlagStall) && w == 0)) return;
    const int nseg = (n + kSeg - 1) / kSeg;
    // First cache entries: every row's minimum over the whole row.
    for (int t = gw; t < n * nseg; t += NW) {
        rescan_segment(D, n, t / nseg, t % nseg, V.rk, V.cw, st_resc);
        st_rows += (t % nseg) == 0;
    }
    clk.lap(0);
    if (!grid_sync(V.rc, ctl, gen, G, timeout)) return;
    clk.lap(1);

    const int R = (n + (int)G - 1) / (int)G;  // rows per workgroup in phase A
    const int r0 = w * R, r1 = min(n, r0 + R);
    const bool may_hand_over = !(flags & kFlagNoHandover);
    int window[kWindow] = {0};  // merges of the last kWindow rounds
    const int nblocks = (n + 63) >> 6;
    int merges = 0, round = 0;
    while (merges < n - 1) {
        if (may_hand_over && round >= kWindow) {
            int recent = 0;
#pragma unroll
            for (int t = 0; t < kWindow; ++t) recent += window[t];
            if (recent < kWindow * kMinPerRound) {
                // Leave the state to the kernel queued behind this one.
                if (w == 0) {
                    for (int q = tid; q < words; q += B) V.live[q] = s_live[q];
                    if (tid == 0) {
                        V.rc->merges = (uint32_t)merges;
                        V.rc->round = (uint32_t)round;
                        atomicOr(status, kHandover);
                    }
                }
                break;
            }
        }
        // ---- A: claim reciprocal (single: and strict) pairs -------------
        if (w == 0 && tid == 0) V.rc->resc = 0;
        uint64_t kmin = kNone;
        for (int a = r0 + tid; a < r1; a += B) {
            if (!live_at(a)) continue;
            const uint64_t e = V.rk[a];
            if (e == kNone) continue;
            const int b = partner_of(e);
            const uint32_t v = value_of(e);
            kmin = umin64(kmin, ((uint64_t)v << 32) | ((uint64_t)min(a, b) << 16) | (uint64_t)max(a, b));
            if (a > b) continue;
            const uint64_t eb = V.rk[b];
            if (partner_of(eb) != a) continue;
            if (link == HAC_SINGLE && (count_of(V.cw[a]) != 1u || count_of(V.cw[b]) != 1u)) continue;
            const uint32_t slot = atomicAdd(&V.rc->pairs, 1u);
            if (slot >= (uint32_t)kRoundsMaxPairs) continue;
            V.pairs[slot] = make_int2(a, b);
            V.role[a] = (int)slot + 1;
            V.role[b] = -((int)slot + 1);
            V.rec[merges + slot] = make_int4(a, b, __float_as_int(unord32(v)), V.size[a] + V.size[b]);
            V.key[merges + slot] = ((uint64_t)v << 32) | ((uint64_t)a << 16) | (uint64_t)round;
        }
        kmin = block_min(kmin);
        if (tid == 0) V.k1[w] = kmin;
        clk.lap(4);
        if (!grid_sync(V.rc, ctl, gen, G, timeout)) return;
        clk.lap(1);

        // ---- B: Lance-Williams updates of every pair --------------------
        {
            uint64_t k1 = kNone;
            for (int t = tid; t < (int)G; t += B) k1 = umin64(k1, V.k1[t]);
            k1 = block_min(k1);
            const uint32_t claimed = __hip_atomic_load(&V.rc->pairs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int p0 = (int)min(claimed, (uint32_t)kRoundsMaxPairs);
            for (int t = tid; t < p0; t += B) s_pair[t] = V.pairs[t];
            if (tid == 0) {
                int np = p0;
                if (k1 == kNone) {
                    atomicOr(&ctl->error, kErrInternal);
                    __hip_atomic_store(&V.rc->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    np = -1;
                } else {
                    const int ka = (int)((k1 >> 16) & 0xFFFFull), kb = (int)(k1 & 0xFFFFull);
                    // The smallest key is a reciprocal pair; if no slot holds
                    // it (single: not strict; or beyond the round's cap) it is
                    // merged as an extra pair, the same on every workgroup.
                    if (V.role[ka] <= 0) {
                        s_pair[p0] = make_int2(ka, kb);
                        np = p0 + 1;
                        if (w == 0) {
                            V.rec[merges + p0] = make_int4(ka, kb, __float_as_int(unord32((uint32_t)(k1 >> 32))),
                                                           V.size[ka] + V.size[kb]);
                            V.key[merges + p0] = (k1 & 0xFFFFFFFF00000000ull) | ((uint64_t)ka << 16) | (uint64_t)round;
                        }
                    }
                }
                s_np = np;
                s_p0 = p0;
            }
            __syncthreads();
            const int np = s_np;
            if (np < 0) return;
            // The survivors' rows are rescanned in phase C: clear their words.
            if (w == 0)
                for (int t = tid; t < np; t += B) {
                    V.rk[s_pair[t].x] = kNone;
                    V.cw[s_pair[t].x] = kNoCount;
                }
            const int extra_i = np > p0 ? s_pair[p0].x : -1, extra_j = np > p0 ? s_pair[p0].y : -1;
            // Pairs per unit: as few as spread the round's (pair, 64-column
            // block) work over every wave of the grid, so that a round with
            // few pairs still keeps all waves busy and the slowest wave, which
            // every workgroup waits for at the next barrier, has no more than
            // its share.
            const int per_wave = (int)(((int64_t)np * nblocks + NW - 1) / NW);
            const int ppu = min(kPairsPerUnit, max(kUnroll, (per_wave + kUnroll - 1) / kUnroll * kUnroll));
            const int npr = (np + ppu - 1) / ppu;
            const int units = nblocks * npr;
            for (int u = gw; u < units; u += NW) {
                const int cb = u % nblocks, pr = u / nblocks;
                const int c = cb * 64 + lane;
                // Columns of the round's own clusters are left to the pass
                // below: their entries are between two merged clusters.
                bool lv = c < n && live_at(c) && c != extra_i && c != extra_j;
                if (lv && V.role[c] != 0) lv = false;
                if (__ballot(lv) == 0ull) continue;
                const uint64_t ec = lv ? V.rk[c] : kNone;
                const uint32_t valc = value_of(ec);
                const int pic = partner_of(ec);
                const int pb = pr * ppu, pe = min(np, pb + ppu);
                for (int p = pb; p < pe; p += kUnroll) {
                    float a[kUnroll], b[kUnroll];
#pragma unroll
                    for (int t = 0; t < kUnroll; ++t) {
                        const int pp = p + t;
                        const bool use = lv && pp < pe;
                        const int2 ij = s_pair[pp < pe ? pp : pb];
                        a[t] = use ? D[(size_t)ij.x * n + c] : 0.0f;
                        b[t] = use ? D[(size_t)ij.y * n + c] : 0.0f;
                    }
#pragma unroll
                    for (int t = 0; t < kUnroll; ++t) {
                        const int pp = p + t;
                        if (!lv || pp >= pe) continue;
                        const int2 ij = s_pair[pp];
                        float v = lw_minmax(link, a[t], b[t]);
                        if (v == 0.0f) v = 0.0f;
                        D[(size_t)ij.x * n + c] = v;
                        D[(size_t)c * n + ij.x] = v;
                        ++st_upd;
                        if (link == HAC_COMPLETE) {
                            if (pic == ij.x || pic == ij.y) {
                                // The row's minimum went up or away: rescan it.
                                V.rk[c] = kNone;
                                V.cw[c] = kNoCount;
                                V.resc[atomicAdd(&V.rc->resc, 1u)] = c;
                            }
                        } else {
                            if (ord32(v) == valc)
                                atomicMin(reinterpret_cast<unsigned long long *>(V.rk + c),
                                          (unsigned long long)(((uint64_t)valc << 32) | ((uint64_t)ij.x << 16)));
                            if (ord32(a[t]) == valc && ord32(b[t]) == valc)
                                atomicSub(reinterpret_cast<unsigned long long *>(V.cw + c), 1ull);
                        }
                    }
                }
            }
            // Entries between two clusters merged in this round: the new
            // distance of (i_p + j_p, i_q + j_q) is min / max of the four
            // entries between their members, exact and in any order.  One
            // thread per unordered pair of pairs reads the four and writes
            // both copies; nothing else in this phase reads or writes them.
            const int64_t ncross = (int64_t)np * (np - 1) / 2;
            for (int64_t t = (int64_t)w * B + tid; t < ncross; t += (int64_t)G * B) {
                // t -> (p, q), p < q: row q of the strict lower triangle
                // holds t in [q(q-1)/2, q(q+1)/2).
                int q = (int)((1.0 + sqrt(1.0 + 8.0 * (double)t)) * 0.5);
                while ((int64_t)q * (q - 1) / 2 > t) --q;
                while ((int64_t)(q + 1) * q / 2 <= t) ++q;
                const int p = (int)(t - (int64_t)q * (q - 1) / 2);
                const int2 P = s_pair[p], Q = s_pair[q];
                const float v = lw_minmax(link, lw_minmax(link, D[(size_t)P.x * n + Q.x], D[(size_t)P.y * n + Q.x]),
                                          lw_minmax(link, D[(size_t)P.x * n + Q.y], D[(size_t)P.y * n + Q.y]));
                const float vz = v == 0.0f ? 0.0f : v;
                D[(size_t)P.x * n + Q.x] = vz;
                D[(size_t)Q.x * n + P.x] = vz;
                ++st_upd;
            }
        }
        clk.lap(2);
        if (!grid_sync(V.rc, ctl, gen, G, timeout)) return;
        clk.lap(1);

        // ---- C: retire, rescan survivors and rows whose partner merged --
        {
            const int np = s_np;
            for (int t = tid; t < np; t += B) {
                const int j = s_pair[t].y;
                atomicAnd(&s_live[j >> 5], ~(1u << (j & 31)));
            }
            if (w == 0) {
                for (int t = tid; t < np; t += B) {
                    const int2 ij = s_pair[t];
                    V.size[ij.x] += V.size[ij.y];
                    V.rk[ij.y] = kNone;
                    V.role[ij.x] = 0;
                    V.role[ij.y] = 0;
                }
                if (tid == 0) V.rc->pairs = 0;
            }
            __syncthreads();
            const int nr = link == HAC_COMPLETE
                               ? (int)__hip_atomic_load(&V.rc->resc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                               : 0;
            const int items = (np + nr) * nseg;
            for (int t = gw; t < items; t += NW) {
                const int k = t / nseg;
                const int r = k < np ? s_pair[k].x : V.resc[k - np];
                rescan_segment(D, n, r, t % nseg, V.rk, V.cw, st_resc);
                st_rows += (t % nseg) == 0;
            }
            merges += np;
            window[round % kWindow] = np;
            ++round;
        }
        clk.lap(3);
        if (!grid_sync(V.rc, ctl, gen, G, timeout)) return;
        clk.lap(1);
    }
    // Statistics (rows rescanned are counted by the wave of their first
    // segment, so only lane 0's count).
    const unsigned long long rows = wave_sum(lane == 0 ? st_rows : 0ull);
    const unsigned long long re = wave_sum(st_resc);
    const unsigned long long up = wave_sum(st_upd);
    if (lane == 0) {
        atomicAdd(&ctl->rescans, rows);
        atomicAdd(&ctl->rescan_elems, re);
        atomicAdd(&ctl->update_elems, up);
        atomicAdd(&ctl->rounds_rescans, rows);
        atomicAdd(&ctl->rounds_rescan_elems, re);
        atomicAdd(&ctl->rounds_update_elems, up);
    }
    if (w == 0 && tid == 0) ctl->rounds = (uint32_t)round;
    if (clk.on && tid == 0) {
        for (int p = 0; p < kPhases; ++p) {
            atomicAdd(&ctl->prof_sum[p], clk.t[p]);
            atomicMax(&ctl->prof_max[p], clk.t[p]);
        }
    }
}

// Records in merge order: record r goes to the rank of its key among all
// m keys (keys are distinct: one survivor merges once per round).
__global__ __launch_bounds__(256) void k_rank(const int4 *__restrict__ rec, const uint64_t *__restrict__ key, int m,
                                              hac_merge *out, const uint32_t *status, const Control *ctl) {
    constexpr int kTileKeys = 2048;
    __shared__ uint64_t tile[kTileKeys];
    // Nothing to sort after rejected input or an abandoned launch.
    if (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & (kErrInput | kErrTimeout | kErrInternal))
        return;
    if (__hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int r = (int)blockIdx.x * 256 + (int)threadIdx.x;
    const uint64_t mine = r < m ? key[r] : kNone;
    int rank = 0;
    for (int t0 = 0; t0 < m; t0 += kTileKeys) {
        const int cnt = min(kTileKeys, m - t0);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += 256) tile[t] = key[t0 + t];
        __syncthreads();
        for (int t = 0; t < cnt; ++t) rank += tile[t] < mine;
    }
    if (r < m) reinterpret_cast<int4 *>(out)[rank] = rec[r];
}

}  // namespace

RoundsLayout rounds_layout(int n, int G) {
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    RoundsLayout L{};
    size_t off = 0;
    L.ctl = off;   off += al(sizeof(RoundsCtl));
    L.rk = off;    off += al((size_t)n * 8);
    L.cnt = off;   off += al((size_t)n * 8);
    L.size = off;  off += al((size_t)n * 4);
    L.role = off;  off += al((size_t)n * 4);
    L.resc = off;  off += al((size_t)n * 4);
    L.pairs = off; off += al((size_t)kRoundsMaxPairs * 8);
    L.k1 = off;    off += al((size_t)G * 8);
    L.rec = off;   off += al((size_t)(n > 1 ? n - 1 : 1) * 16);
    L.key = off;   off += al((size_t)(n > 1 ? n - 1 : 1) * 8);
    L.live = off;  off += al((size_t)((n + 31) / 32) * 4);
    L.bytes = off;
    return L;
}

int rounds_occupancy() {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void *>(&k_rounds), kRoundsBlock,
                                                     0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return blocks < 1 ? 1 : blocks;
}

hipError_t launch_rounds(float *D, int n, int link, uint32_t *status, Control *ctl, void *ws, int G,
                         uint64_t timeout_ticks, int flags, hipStream_t stream) {
    const RoundsLayout Lo = rounds_layout(n, G);
    float *a0 = D;
    int a1 = n;
    int a2 = link;
    uint32_t *a3 = status;
    Control *a4 = ctl;
    char *a5 = static_cast<char *>(ws);
    RoundsLayout a6 = Lo;
    uint64_t a7 = timeout_ticks;
    int a8 = flags;
    void *args[] = {&a0, &a1, &a2, &a3, &a4, &a5, &a6, &a7, &a8};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_rounds), dim3(G), dim3(kRoundsBlock), args, 0,
                                      stream);
}

hipError_t launch_rank(int n, hac_merge *out, const uint32_t *status, const Control *ctl, void *ws, int G,
                       hipStream_t stream) {
    const RoundsLayout Lo = rounds_layout(n, G);
    const int m = n - 1;
    hipLaunchKernelGGL(k_rank, dim3((m + 255) / 256), dim3(256), 0, stream,
                       reinterpret_cast<const int4 *>(static_cast<char *>(ws) + Lo.rec),
                       reinterpret_cast<const uint64_t *>(static_cast<char *>(ws) + Lo.key), m, out, status, ctl);
    return hipGetLastError();
}

Resume rounds_resume(int n, int G, void *ws) {
    const RoundsLayout Lo = rounds_layout(n, G);
    char *b = static_cast<char *>(ws);
    Resume r;
    r.live = reinterpret_cast<const uint32_t *>(b + Lo.live);
    r.size = reinterpret_cast<const int32_t *>(b + Lo.size);
    r.keys = reinterpret_cast<uint64_t *>(b + Lo.key);
    r.state = reinterpret_cast<const uint32_t *>(b + Lo.ctl + offsetof(RoundsCtl, merges));
    return r;
}

hac_merge *rounds_records(int n, int G, void *ws) {
    return reinterpret_cast<hac_merge *>(static_cast<char *>(ws) + rounds_layout(n, G).rec);
}

}  // namespace hac
