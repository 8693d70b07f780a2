// C-ABI layer of the clustering library (declared in include/hac.h):
// argument checks, device workspace, choice of launch shape, status read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <unordered_map>
#include <vector>

#include "hac.h"
#include "hac_ctx_info.h"
#include "hac_engine.h"
#include "hac_rmsd.h"
#include "hac_rounds.h"
#include "hac_scan.h"
#include "hac_validate.h"

namespace {

constexpr size_t kAlign = 256;
constexpr int kDefaultSingleWgN = 1536;
constexpr int kDeferMinGroup = 2;       // HAC_OPT_DEFER = 1: defer from this many workgroups on
constexpr int64_t kDefaultTimeoutMs = 10000;
constexpr int kRoundsMinN = 1024;       // HAC_OPT_ROUNDS = 1: rounds of merges from this n on

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// How one hac_batch call is laid out on the device.
struct BatchPlan {
    int block = 256;  // threads per workgroup
    int group = 1;    // workgroups per large instance (1 = every instance on one workgroup)
    int share = 2;    // quarters of the co-resident workgroups that groups may take
    int upd = 0;      // update tile at 1024 threads: 2 or 4 chunks per wave (0: 4)
};

// Update tile a plan runs with (the batch kernel's variants).
int plan_update(const BatchPlan &p) { return p.block != 1024 ? 8 : p.upd == 2 ? 2 : 4; }

}  // namespace

struct hac_ctx {
    int device = 0;
    hipStream_t own = nullptr;
    std::string err;
    int cus = 0;
    size_t lds_max = 0;
    int wallclock_khz = 0;
    int coop = 0;

    void *ws = nullptr;          // control block, statuses, sizes, slots, descriptors
    size_t ws_cap = 0;
    void *scratch = nullptr;     // this device's static scratch array (hac_run_noalloc)
    float *dcopy = nullptr;      // HAC_PRESERVE_INPUT copy
    size_t dcopy_cap = 0;        // bytes
    float *spare = nullptr;      // HAC_MODE_SCAN: the compacted matrix's second buffer
    size_t spare_cap = 0;        // bytes
    void *rmsd_ws = nullptr;     // RMSD producer: coordinate planes, norms, status
    size_t rmsd_cap = 0;
    hac_merge *dout = nullptr;   // device merge records when the caller's out is host memory
    size_t dout_cap = 0;         // records
    void *pinned = nullptr;      // host staging (status read-back, descriptor upload)
    size_t pinned_cap = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // [3]: end of the round engine's kernel

    hac_stats stats{};
    int64_t opt_wgs = 0, opt_single_n = 0, opt_timeout_ms = 0, opt_exchange = 0, opt_profile = 0;
    int64_t opt_block = 0, opt_batch_block = 0, opt_batch_group = 0, opt_batch_upd = 0, opt_autotune = 1;
    std::unordered_map<std::string, BatchPlan> plans;  // tuned batch plans by size mix
    int64_t opt_graph = 1;
    int64_t opt_defer = 1;
    int64_t opt_rounds = 1;
    int64_t opt_stall = 0;
    bool opt_lazy = true;  // HAC_OPT_LAZY_MIRROR
    int pending_plan_source = 0, pending_plan_share = 0, pending_plan_upd = 0;  // hac_batch: its plan
    std::unordered_map<std::string, hipGraphExec_t> graphs;  // batch graphs by layout

    // State of the last enqueued call, for hac_sync / stats.
    bool pending = false;
    hipStream_t pending_stream = nullptr;
    int pending_count = 0;           // status words to check
    int pending_wgs = 0, pending_block = 0, pending_group = 0, pending_graph = 0, pending_deferred = 0;
    bool pending_rounds = false;
    bool pending_scan = false;
    int pending_seq_wgs = 0, pending_seq_block = 0, pending_seq_deferred = 0;  // kernel queued behind the rounds
};

namespace {

// The message of a failed argument check becomes the context's last error.
int checked(hac_ctx *c, int rc, const char *msg) {
    if (rc != HAC_OK) c->err = msg;
    return rc;
}

int fail(hac_ctx *c, int code, const char *fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

int hip_fail(hac_ctx *c, hipError_t e, const char *what) {
    return fail(c, e == hipErrorOutOfMemory ? HAC_ENOMEM : HAC_EDEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

#define HIP_TRY(c, expr)                                  \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_fail((c), e_, #expr); \
    } while (0)

int ensure_dev(hac_ctx *c, void **p, size_t *cap, size_t need, const char *what) {
    if (need <= *cap) return HAC_OK;
    if (*p) {
        hipError_t e = hipStreamSynchronize(c->own);
        (void)e;
        HIP_TRY(c, hipDeviceSynchronize());
        HIP_TRY(c, hipFree(*p));
        *p = nullptr;
        *cap = 0;
    }
    size_t sz = std::max(need, *cap * 3 / 2);
    hipError_t e = hipMalloc(p, sz);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        e = hipMalloc(p, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return fail(c, HAC_ENOMEM, "cannot allocate %zu bytes of device memory for %s", need, what);
        }
        sz = need;
    }
    *cap = sz;
    return HAC_OK;
}

int ensure_pinned(hac_ctx *c, size_t need) {
    if (need <= c->pinned_cap) return HAC_OK;
    if (c->pinned) {
        HIP_TRY(c, hipDeviceSynchronize());
        HIP_TRY(c, hipHostFree(c->pinned));
        c->pinned = nullptr;
        c->pinned_cap = 0;
    }
    size_t sz = std::max(need, (size_t)4096);
    hipError_t e = hipHostMalloc(&c->pinned, sz, hipHostMallocDefault);
    if (e != hipSuccess) {
        c->pinned = nullptr;
        return hip_fail(c, e, "hipHostMalloc");
    }
    c->pinned_cap = sz;
    return HAC_OK;
}

int set_device(hac_ctx *c) {
    HIP_TRY(c, hipSetDevice(c->device));
    return HAC_OK;
}

void clear_graphs(hac_ctx *c) {
    if (c->graphs.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

uint64_t timeout_ticks(const hac_ctx *c) {
    int64_t ms = c->opt_timeout_ms > 0 ? c->opt_timeout_ms : kDefaultTimeoutMs;
    return (uint64_t)ms * (uint64_t)(c->wallclock_khz > 0 ? c->wallclock_khz : 100000);
}

// Workgroups that can be co-resident for a hac_run launch with `lds` bytes
// (merge kernel variant selected by the kFlag* bits in run_flags).
int max_coresident(hac_ctx *c, size_t lds, int block, int32_t run_flags) {
    int per_cu = hac::engine_occupancy(lds, block, false, run_flags);
    if (per_cu < 1) per_cu = 1;
    return per_cu * c->cus;
}

// Check the device status words of the last call (after the stream is idle).
int check_status(hac_ctx *c) {
    const hac::Control *ctl = reinterpret_cast<const hac::Control *>(c->pinned);
    const uint32_t *st = reinterpret_cast<const uint32_t *>(
        reinterpret_cast<const char *>(c->pinned) + align_up(sizeof(hac::Control), kAlign));
    float ms = 0.0f, ims = 0.0f;
    if (hipEventElapsedTime(&ms, c->ev[1], c->ev[2]) != hipSuccess) ms = 0.0f;
    if (hipEventElapsedTime(&ims, c->ev[0], c->ev[1]) != hipSuccess) ims = 0.0f;
    c->stats.kernel_ms = ms;
    c->stats.init_ms = ims;
    c->stats.rescans = (int64_t)ctl->rescans;
    c->stats.rescan_elems = (int64_t)ctl->rescan_elems;
    c->stats.update_elems = (int64_t)ctl->update_elems;
    c->stats.forced_rounds = (int64_t)ctl->forced;
    c->stats.deferred = c->pending_deferred;
    c->stats.rounds = c->pending_rounds ? (int32_t)ctl->rounds : 0;
    c->stats.compactions = c->pending_scan ? (int32_t)ctl->rounds : 0;
    c->stats.rounds_ms = 0.0;
    c->stats.rounds_rescan_elems = c->stats.rounds_update_elems = 0;
    if (c->pending_rounds) {
        float rms = 0.0f;
        if (hipEventElapsedTime(&rms, c->ev[1], c->ev[3]) != hipSuccess) rms = 0.0f;
        c->stats.rounds_ms = rms;
        c->stats.rounds_rescan_elems = (int64_t)ctl->rounds_rescan_elems;
        c->stats.rounds_update_elems = (int64_t)ctl->rounds_update_elems;
    }
    c->stats.workgroups = c->pending_wgs;
    c->stats.block = c->pending_block;
    c->stats.group = c->pending_group;
    c->stats.graph = c->pending_graph;
    c->stats.plan_source = c->pending_plan_source;
    c->stats.plan_share = c->pending_plan_share;
    c->stats.plan_update = c->pending_plan_upd;
    if (c->pending_rounds && c->pending_count == 1 && (st[0] & hac::kHandover)) {
        // The round engine handed the rest of the merges to the kernel
        // queued behind it.
        c->stats.handed_over = 1;
        c->stats.deferred = c->pending_seq_deferred;
    }
    const double khz = c->wallclock_khz > 0 ? c->wallclock_khz : 100000.0;
    for (int p = 0; p < 5; ++p) {
        c->stats.phase_avg_ms[p] = (double)ctl->prof_sum[p] / khz / std::max(1, c->pending_wgs);
        c->stats.phase_max_ms[p] = (double)ctl->prof_max[p] / khz;
    }
    for (int k = 0; k < c->pending_count; ++k) {
        if (st[k] & hac::kErrInput)
            return fail(c, HAC_EINPUT, "instance %d: non-finite or |x| > 2^100 value in the strict upper triangle", k);
    }
    for (int k = 0; k < c->pending_count; ++k) {
        if (st[k] & hac::kErrTimeout)
            return fail(c, HAC_ETIMEDOUT, "instance %d: watchdog expired inside the persistent kernel", k);
        if (st[k] & hac::kErrInternal)
            return fail(c, HAC_EINTERNAL, "instance %d: no live pair found on the device", k);
    }
    if (ctl->error & hac::kErrTimeout)
        return fail(c, HAC_ETIMEDOUT, "watchdog expired inside the persistent kernel");
    return HAC_OK;
}

// Enqueue the read-back of control + status words, then either return
// (device output) or wait and check.
int finish(hac_ctx *c, hipStream_t s, int nstatus, hac_merge *out, size_t nrec, uint32_t flags,
           const void *ws) {
    const size_t ctl_bytes = align_up(sizeof(hac::Control), kAlign);
    HIP_TRY(c, hipMemcpyAsync(c->pinned, ws, ctl_bytes + (size_t)nstatus * 4, hipMemcpyDeviceToHost, s));
    c->pending = true;
    c->pending_stream = s;
    c->pending_count = nstatus;
    if (flags & HAC_OUT_DEVICE) return HAC_OK;
    HIP_TRY(c, hipStreamSynchronize(s));
    c->pending = false;
    int rc = check_status(c);
    if (rc != HAC_OK) return rc;
    if (nrec) HIP_TRY(c, hipMemcpy(out, c->dout, nrec * sizeof(hac_merge), hipMemcpyDeviceToHost));
    return HAC_OK;
}

}  // namespace

namespace {

// Instances at least this large may get a group of workgroups.
constexpr int kGroupMinN = 2048;

// Signature of a batch for the plan cache: size histogram (powers of two) and
// linkage mix (linkages already checked to be 0..HAC_CENTROID).
std::string batch_signature(const int32_t *ns, const int32_t *links, int count) {
    constexpr int kLinks = HAC_CENTROID + 1;
    int hist[18] = {0}, lk[kLinks] = {0};
    for (int k = 0; k < count; ++k) {
        int b = 0;
        while ((1 << (b + 1)) <= ns[k] && b < 17) ++b;
        hist[b]++;
        lk[links[k]]++;
    }
    std::string s = std::to_string(count);
    for (int b = 0; b < 18; ++b) s += "," + std::to_string(hist[b]);
    for (int q = 0; q < kLinks; ++q) s += ";" + std::to_string(lk[q]);
    return s;
}

// Where one batch call's pieces sit in the workspace.
struct BatchLayout {
    hac::BatchLaunch L{};
    size_t st_off = 0, st_bytes = 0;   // control block + statuses: [0, st_off + st_bytes)
    size_t in_off = 0, up_bytes = 0;   // descriptors, order, groups: uploaded as one block
    size_t sl_off = 0, sl_bytes = 0;   // exchange slots of the groups
    int group = 1;
};

// Lay out a batch for `plan`, write its descriptors into the pinned staging
// buffer and fill `B`.  The caller has validated the batch.  Nothing is
// enqueued.
int batch_prepare(hac_ctx *c, float *base, const int64_t *offsets, const int32_t *ns,
                  const int32_t *links, int count, hac_merge *dev_out, const int64_t *out_offsets,
                  const BatchPlan &plan, hipStream_t s, BatchLayout *B) {
    std::vector<int32_t> ord(count);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return ns[a] > ns[b]; });

    // Groups for the largest instances, on workgroups 0, g, 2g, ... while at
    // most plan.share quarters of the co-resident workgroups are taken.
    const size_t lds1 = hac::lds_bytes(ns[ord[0]], hac::own_rows(ns[ord[0]], 1), true);
    int per_cu = std::max(1, hac::engine_occupancy(lds1, plan.block, true));
    int cap = per_cu * c->cus;
    std::vector<int32_t> gbase, gsize;
    int used = 0;
    if (plan.group > 1) {
        for (int t = 0; t < count; ++t) {
            const int n = ns[ord[t]];
            if (n < kGroupMinN || used + plan.group > cap * plan.share / 4) break;
            gbase.push_back(used);
            gsize.push_back(plan.group);
            used += plan.group;
        }
    }
    const int ngroups = (int)gbase.size();
    // An instance uses the lazy mirror if its step table fits beside the rest.
    std::vector<uint8_t> lazy(count, 0);
    size_t lds = 0;
    for (int t = 0; t < count; ++t) {
        const int n = ns[ord[t]], g = t < ngroups ? plan.group : 1, own = hac::own_rows(n, g);
        lazy[ord[t]] = c->opt_lazy && hac::lds_bytes(n, own, true, true) <= c->lds_max;
        lds = std::max(lds, hac::lds_bytes(n, own, true, lazy[ord[t]] != 0));
        if (lds > c->lds_max) return fail(c, HAC_EINVAL, "n=%d does not fit one workgroup's LDS", n);
    }
    per_cu = std::max(1, hac::engine_occupancy(lds, plan.block, true));
    cap = per_cu * c->cus;
    const int grid = std::max(used, std::min(cap, used + (count - ngroups)));
    if (grid > cap) return fail(c, HAC_EINVAL, "batch plan needs %d co-resident workgroups", grid);

    const size_t ctl_bytes = align_up(sizeof(hac::Control), kAlign);
    const size_t st_off = ctl_bytes, st_bytes = align_up((size_t)count * 4, kAlign);
    const size_t in_off = st_off + st_bytes, in_bytes = align_up((size_t)count * sizeof(hac::Instance), kAlign);
    const size_t or_off = in_off + in_bytes, or_bytes = align_up((size_t)count * 4, kAlign);
    const size_t gb_off = or_off + or_bytes, gb_bytes = align_up((size_t)std::max(ngroups, 1) * 8, kAlign);
    const size_t sl_off = gb_off + gb_bytes;
    const size_t sl_each = (size_t)2 * (plan.group + 1) * hac::kSlotStride * 8;
    const size_t sl_bytes = (size_t)ngroups * sl_each;
    int rc = ensure_dev(c, &c->ws, &c->ws_cap, sl_off + sl_bytes, "workspace");
    if (rc) return rc;
    const size_t up_bytes = in_bytes + or_bytes + gb_bytes;
    rc = ensure_pinned(c, std::max(ctl_bytes + st_bytes, up_bytes));
    if (rc) return rc;
    char *ws = reinterpret_cast<char *>(c->ws);
    // The pinned buffer may still be the source or target of an earlier copy.
    HIP_TRY(c, hipStreamSynchronize(s));
    char *pin = reinterpret_cast<char *>(c->pinned);
    hac::Instance *hin = reinterpret_cast<hac::Instance *>(pin);
    for (int k = 0; k < count; ++k) {
        hac::Instance &I = hin[k];
        I.D = base + offsets[k];
        I.out = dev_out + out_offsets[k];
        I.rowkey = nullptr;
        I.slots = nullptr;
        I.status = reinterpret_cast<uint32_t *>(ws + st_off) + k;
        I.n = ns[k];
        I.link = links[k];
        I.exchange = 0;
        I.flags = (c->opt_profile ? hac::kFlagProfile : 0) | (c->opt_stall ? hac::kFlagStall : 0) |
                  (lazy[k] ? hac::kFlagLazy : 0);
    }
    for (int t = 0; t < ngroups; ++t)
        hin[ord[t]].slots = reinterpret_cast<uint64_t *>(ws + sl_off + (size_t)t * sl_each);
    std::memcpy(pin + in_bytes, ord.data(), (size_t)count * 4);
    int32_t *hg = reinterpret_cast<int32_t *>(pin + in_bytes + or_bytes);
    for (int t = 0; t < ngroups; ++t) {
        hg[t] = gbase[t];
        hg[ngroups + t] = gsize[t];
    }

    hac::BatchLaunch &L = B->L;
    L.insts = reinterpret_cast<hac::Instance *>(ws + in_off);
    L.order = reinterpret_cast<int32_t *>(ws + or_off);
    L.count = count;
    L.gbase = reinterpret_cast<int32_t *>(ws + gb_off);
    L.gsize = reinterpret_cast<int32_t *>(ws + gb_off) + ngroups;
    L.ngroups = ngroups;
    L.block = plan.block;
    L.upd = plan_update(plan);
    L.grid = grid;
    L.lds = lds;
    B->st_off = st_off;
    B->st_bytes = st_bytes;
    B->in_off = in_off;
    B->up_bytes = up_bytes;
    B->sl_off = sl_off;
    B->sl_bytes = sl_bytes;
    B->group = ngroups ? plan.group : 1;
    return HAC_OK;
}

// Enqueue a prepared batch: descriptor upload, zero fills, then (after
// `before_kernel`, if given, is recorded) the kernel.
hipError_t batch_enqueue(hac_ctx *c, const BatchLayout &B, hipStream_t s, hipEvent_t before_kernel) {
    char *ws = reinterpret_cast<char *>(c->ws);
    hipError_t e = hipMemcpyAsync(ws + B.in_off, c->pinned, B.up_bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hac::launch_zero(ws, (B.st_off + B.st_bytes) / 4, s);
    if (e == hipSuccess && B.sl_bytes) e = hac::launch_zero(ws + B.sl_off, B.sl_bytes / 4, s);
    if (e == hipSuccess && before_kernel) e = hipEventRecord(before_kernel, s);
    if (e == hipSuccess) e = hac::launch_batch(B.L, reinterpret_cast<hac::Control *>(ws), timeout_ticks(c), s);
    return e;
}

// Run `p` once on the scratch copy and return its kernel time in ms, or a
// negative value if the plan could not be laid out or launched or if its run
// reported any error (an instance's status word or the control block); such
// a plan is never chosen.
float batch_try_plan(hac_ctx *c, float *scratch, const float *packed, int64_t extent, const int64_t *offsets,
                     const int32_t *ns, const int32_t *links, int count, hac_merge *dev_out,
                     const int64_t *out_offsets, hipStream_t s, const BatchPlan &p) {
    if (hipMemcpyAsync(scratch, packed, (size_t)extent * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        (void)hipGetLastError();
        return -1.0f;
    }
    BatchLayout B;
    if (batch_prepare(c, scratch, offsets, ns, links, count, dev_out, out_offsets, p, s, &B) != HAC_OK) return -1.0f;
    if (batch_enqueue(c, B, s, c->ev[1]) != hipSuccess || hipEventRecord(c->ev[2], s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        return -1.0f;
    }
    // The control block and the status words of this run.
    if (hipMemcpy(c->pinned, c->ws, B.st_off + (size_t)count * 4, hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        return -1.0f;
    }
    const hac::Control *ctl = reinterpret_cast<const hac::Control *>(c->pinned);
    const uint32_t *st = reinterpret_cast<const uint32_t *>(static_cast<const char *>(c->pinned) + B.st_off);
    if (ctl->error || ctl->abort) return -1.0f;
    for (int k = 0; k < count; ++k)
        if (st[k]) return -1.0f;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, c->ev[1], c->ev[2]) != hipSuccess) return -1.0f;
    return ms;
}

// Pick a launch plan by timing candidates on a scratch copy of the batch;
// results never depend on the plan.  Coordinate search: first the threads
// per workgroup with every instance on one workgroup (each block size
// carries its own tile sizes: 8-deep update batches and 8-load rescan
// segments per lane at 256 threads, 4 and 4 at 1024), then with that block
// size the workgroups per large instance (2, 4, 8) and how many of the
// co-resident workgroups groups may take (a quarter, half, three quarters),
// which decides how many of the largest instances get a group, then at 1024
// threads the other update tile (2 instead of 4 chunks per wave: fewer
// registers, two load batches for the largest rows).  Plans whose
// run reports an error are skipped; if every plan fails, the default plan is
// kept and the real run reports the error.
int batch_autotune(hac_ctx *c, float *packed, int64_t extent, const int64_t *offsets,
                   const int32_t *ns, const int32_t *links, int count, hac_merge *dev_out,
                   const int64_t *out_offsets, hipStream_t s, BatchPlan *best) {
    float *scratch = nullptr;
    size_t scratch_cap = 0;
    int rc = ensure_dev(c, reinterpret_cast<void **>(&scratch), &scratch_cap, (size_t)extent * 4, "tuning copy");
    if (rc) return rc;
    float best_ms = 1e30f;
    *best = BatchPlan{};
    auto consider = [&](const BatchPlan &p) {
        const float ms = batch_try_plan(c, scratch, packed, extent, offsets, ns, links, count, dev_out, out_offsets,
                                        s, p);
        if (ms >= 0.0f && ms < best_ms) {
            best_ms = ms;
            *best = p;
        }
    };
    for (int block : {256, 1024}) consider(BatchPlan{block, 1, 2});
    const int block = best->block;
    for (int group : {2, 4, 8})
        for (int share : {1, 2, 3}) consider(BatchPlan{block, group, share});
    if (best->block == 1024) {
        BatchPlan p = *best;
        p.upd = 2;
        consider(p);
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(scratch);
    c->err.clear();
    return HAC_OK;
}

}  // namespace

namespace hac {
void ctx_info(const hac_ctx *c, CtxInfo *out) {
    out->device = c->device;
    out->cus = c->cus;
    out->wallclock_khz = c->wallclock_khz;
    out->lds_max = c->lds_max;
    out->timeout_ms = c->opt_timeout_ms;
    out->lazy = c->opt_lazy;
}
}  // namespace hac

extern "C" {

int hac_create(int device, hac_ctx **out) {
    if (!out) return HAC_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return HAC_ENODEV;
    }
    if (device < 0 || device >= count) return HAC_ENODEV;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return HAC_ENODEV;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return HAC_ENODEV;
    hac_ctx *c = new hac_ctx();
    c->device = device;
    c->cus = prop.multiProcessorCount;
    c->lds_max = prop.sharedMemPerBlock;
    c->coop = prop.cooperativeLaunch;
    int rate = 0;
    if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, device) == hipSuccess) c->wallclock_khz = rate;
    if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return HAC_EDEVICE;
    }
    for (auto &e : c->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            hac_destroy(c);
            return HAC_EDEVICE;
        }
    }
    size_t usable = 0;
    if (hac::engine_setup(c->lds_max, &usable) != hipSuccess) {
        (void)hipGetLastError();
        hac_destroy(c);
        return HAC_EDEVICE;
    }
    c->lds_max = usable;
    // The allocation-free entry point's scratch: this device's copy of the
    // library's static array (the device is current), and the page-locked
    // word its status comes back through.
    if (hac::engine_scratch(&c->scratch) != hipSuccess || !c->scratch) {
        (void)hipGetLastError();
        hac_destroy(c);
        return HAC_EDEVICE;
    }
    if (ensure_pinned(c, 4096) != HAC_OK) {
        hac_destroy(c);
        return HAC_EDEVICE;
    }
    *out = c;
    return HAC_OK;
}

int hac_destroy(hac_ctx *c) {
    if (!c) return HAC_OK;
    (void)hipSetDevice(c->device);
    if (c->own) (void)hipStreamSynchronize(c->own);
    (void)hipDeviceSynchronize();
    clear_graphs(c);
    if (c->ws) (void)hipFree(c->ws);
    if (c->dcopy) (void)hipFree(c->dcopy);
    if (c->spare) (void)hipFree(c->spare);
    if (c->rmsd_ws) (void)hipFree(c->rmsd_ws);
    if (c->dout) (void)hipFree(c->dout);
    if (c->pinned) (void)hipHostFree(c->pinned);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->own) (void)hipStreamDestroy(c->own);
    delete c;
    return HAC_OK;
}

int hac_rmsd(hac_ctx *c, const float *coords, int32_t n, int32_t atoms, float *dist, uint32_t flags, void *stream) {
    if (!c) return HAC_EINVAL;
    c->err.clear();
    char msg[192];
    int rc = hac::check_rmsd_args(coords, n, atoms, dist, flags, hac::kRmsdMaxAtoms, msg, sizeof msg);
    if (rc) return checked(c, rc, msg);
    rc = set_device(c);
    if (rc) return rc;
    if (c->pending) (void)hac_sync(c);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const hac::RmsdLayout L = hac::rmsd_layout(n, atoms);
    rc = ensure_dev(c, &c->rmsd_ws, &c->rmsd_cap, L.bytes, "the RMSD workspace");
    if (rc) return rc;
    rc = ensure_pinned(c, 64);
    if (rc) return rc;
    HIP_TRY(c, hac::launch_rmsd(coords, n, atoms, dist, c->rmsd_ws, s));
    HIP_TRY(c, hipMemcpyAsync(c->pinned, static_cast<char *>(c->rmsd_ws) + L.status_offset, sizeof(uint32_t),
                              hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    if (*static_cast<const uint32_t *>(c->pinned) != 0u)
        return fail(c, HAC_EINPUT, "a coordinate is not finite or exceeds 2^40 in magnitude");
    return HAC_OK;
}

const char *hac_last_error(const hac_ctx *c) { return c ? c->err.c_str() : "no context"; }

int hac_set_option(hac_ctx *c, int32_t option, int64_t value) {
    if (!c) return HAC_EINVAL;
    if (value < 0) return fail(c, HAC_EINVAL, "option %d: negative value", option);
    switch (option) {
    case HAC_OPT_WORKGROUPS: c->opt_wgs = value; return HAC_OK;
    case HAC_OPT_SINGLE_WG_N: c->opt_single_n = value; return HAC_OK;
    case HAC_OPT_TIMEOUT_MS: c->opt_timeout_ms = value; return HAC_OK;
    case HAC_OPT_PROFILE: c->opt_profile = value != 0; return HAC_OK;
    case HAC_OPT_BATCH_BLOCK:
        if (value != 0 && value != 256 && value != 1024)
            return fail(c, HAC_EINVAL, "batch block size %lld is not 256 or 1024", (long long)value);
        c->opt_batch_block = value;
        return HAC_OK;
    case HAC_OPT_BATCH_GROUP:
        if (value > 64) return fail(c, HAC_EINVAL, "batch group %lld > 64", (long long)value);
        c->opt_batch_group = value;
        return HAC_OK;
    case HAC_OPT_BATCH_UPDATE:
        if (value != 0 && value != 2 && value != 4)
            return fail(c, HAC_EINVAL, "batch update tile %lld is not 0, 2 or 4", (long long)value);
        c->opt_batch_upd = value;
        return HAC_OK;
    case HAC_OPT_AUTOTUNE: c->opt_autotune = value != 0; return HAC_OK;
    case HAC_OPT_GRAPH: c->opt_graph = value != 0; return HAC_OK;
    case HAC_OPT_INJECT_STALL: c->opt_stall = value != 0; return HAC_OK;
    case HAC_OPT_LAZY_MIRROR: c->opt_lazy = value != 0; return HAC_OK;
    case HAC_OPT_ROUNDS:
        if (value > 2) return fail(c, HAC_EINVAL, "rounds mode %lld is not 0, 1 or 2", (long long)value);
        c->opt_rounds = value;
        return HAC_OK;
    case HAC_OPT_DEFER:
        if (value > 2) return fail(c, HAC_EINVAL, "defer mode %lld is not 0, 1 or 2", (long long)value);
        c->opt_defer = value;
        return HAC_OK;
    case HAC_OPT_BLOCK:
        if (value != 0 && value != 256 && value != 512 && value != 1024)
            return fail(c, HAC_EINVAL, "block size %lld is not 256, 512 or 1024", (long long)value);
        c->opt_block = value;
        return HAC_OK;
    case HAC_OPT_EXCHANGE:
        if (value > 1) return fail(c, HAC_EINVAL, "exchange mode %lld", (long long)value);
        c->opt_exchange = value;
        return HAC_OK;
    default: return fail(c, HAC_EINVAL, "unknown option %d", option);
    }
}

int hac_get_stats(const hac_ctx *c, hac_stats *out) {
    if (!c || !out) return HAC_EINVAL;
    *out = c->stats;
    return HAC_OK;
}

int hac_sync(hac_ctx *c) {
    if (!c) return HAC_EINVAL;
    if (!c->pending) return HAC_OK;
    int rc = set_device(c);
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->pending_stream));
    c->pending = false;
    return check_status(c);
}

}  // extern "C"

namespace {

// Launch plan of the one-merge-per-step kernel for hac_run: workgroups g,
// threads per workgroup and kFlag* bits.
int plan_seq(hac_ctx *c, int32_t n, uint32_t flags, bool noalloc, int *g_out, int *block_out, int32_t *flags_out) {
    // Launch shape: one workgroup for small n, else a co-resident group of
    // a few large workgroups (each merge costs every workgroup one agent-scope
    // release/acquire pair, so fewer workgroups mean a cheaper exchange).
    const int nch = (n + 63) / 64;
    const int block = c->opt_block > 0 ? (int)c->opt_block : hac::kRunBlock;
    const int single_n = c->opt_single_n > 0 ? (int)c->opt_single_n : kDefaultSingleWgN;
    int g = 1;
    int32_t run_flags = (c->opt_profile ? hac::kFlagProfile : 0) | ((flags & HAC_MODE_SCAN) ? hac::kFlagScan : 0) |
                        (c->opt_stall ? hac::kFlagStall : 0);
    if (n > single_n || hac::lds_bytes(n, hac::own_rows(n, 1), false) > c->lds_max) {
        // Co-residency is checked for the deferred variant too, which may
        // be chosen below once g is known.
        if (c->opt_defer && !(flags & HAC_MODE_SCAN)) run_flags |= hac::kFlagDefer;
        // Measured on MI355X: about one workgroup per 512 items, up to 64.
        // The paper's scan mode is bandwidth-bound: as many workgroups as fit.
        int want = c->opt_wgs > 0 ? (int)c->opt_wgs
                   : (flags & HAC_MODE_SCAN) ? nch
                                             : std::max(2, std::min(64, n / 512));
        if (noalloc) want = std::min(want, HAC_NOALLOC_MAX_WORKGROUPS);
        g = std::max(1, std::min(want, nch));
        while (g < nch && hac::lds_bytes(n, hac::own_rows(n, g), false) > c->lds_max) ++g;
        const size_t lds = hac::lds_bytes(n, hac::own_rows(n, g), false);
        if (lds > c->lds_max) return fail(c, HAC_EINVAL, "n=%d does not fit in LDS", n);
        const int cap = max_coresident(c, lds, block, run_flags);
        if (g > cap) g = cap;
        if (hac::lds_bytes(n, hac::own_rows(n, g), false) > c->lds_max)
            return fail(c, HAC_EDEVICE, "n=%d needs more co-resident workgroups than the device holds", n);
        if (noalloc && g > HAC_NOALLOC_MAX_WORKGROUPS)
            return fail(c, HAC_EINVAL, "n=%d needs more than %d workgroups", n, HAC_NOALLOC_MAX_WORKGROUPS);
        if (g > 1 && !c->coop) return fail(c, HAC_EDEVICE, "device does not support cooperative launch");
    } else if (c->opt_defer == 2 && !(flags & HAC_MODE_SCAN)) {
        run_flags |= hac::kFlagDefer;  // one workgroup, deferred rescans on request
    }

    // Deferred rescans pay on every group of workgroups (measured at n = 2048
    // … 65536); a workgroup alone does better rescanning at once.
    if (c->opt_defer == 1 && g < kDeferMinGroup) run_flags &= ~hac::kFlagDefer;
    *g_out = g;
    *block_out = block;
    *flags_out = run_flags;
    return HAC_OK;
}

// hac_run through the round engine (single and complete linkage).
int run_rounds(hac_ctx *c, float *dist, int32_t n, int32_t linkage, hac_merge *out, uint32_t flags, hipStream_t s) {
    if (!c->coop) return fail(c, HAC_EDEVICE, "device does not support cooperative launch");
    int G = c->cus * hac::rounds_occupancy();
    if (c->opt_wgs > 0) G = std::min(G, (int)c->opt_wgs);
    // Automatic mode: the one-merge-per-step kernel is queued behind the
    // round engine and makes the remaining merges if the round engine hands
    // them over (when rounds merge few pairs each, see hac_rounds.h).
    const bool handover = c->opt_rounds == 1;
    int g = 1, block = hac::kRunBlock;
    int32_t seq_flags = 0;
    int rc = HAC_OK;
    if (handover) {
        rc = plan_seq(c, n, flags, false, &g, &block, &seq_flags);
        if (rc) return rc;
    }
    // Workspace: control | status | first upper row minima (set-up kernel) |
    // round engine | exchange slots of the queued kernel.
    const size_t ctl_bytes = align_up(sizeof(hac::Control), kAlign);
    const size_t st_off = ctl_bytes, st_bytes = kAlign;
    const size_t rk_off = st_off + st_bytes, rk_bytes = align_up((size_t)n * 8, kAlign);
    const size_t ro_off = rk_off + rk_bytes;
    const hac::RoundsLayout Lo = hac::rounds_layout(n, G);
    const size_t sl_off = ro_off + Lo.bytes;
    const size_t sl_bytes = (handover && g > 1) ? (size_t)2 * (g + 1) * hac::kSlotStride * 8 : 0;
    rc = ensure_dev(c, &c->ws, &c->ws_cap, sl_off + sl_bytes, "workspace");
    if (rc) return rc;
    rc = ensure_pinned(c, ctl_bytes + kAlign);
    if (rc) return rc;
    char *ws = reinterpret_cast<char *>(c->ws);
    float *D = dist;
    if (flags & HAC_PRESERVE_INPUT) {
        const size_t bytes = (size_t)n * n * 4;
        rc = ensure_dev(c, reinterpret_cast<void **>(&c->dcopy), &c->dcopy_cap, bytes, "input copy");
        if (rc) return rc;
        D = c->dcopy;
    }
    hac_merge *dev_out = out;
    if (!(flags & HAC_OUT_DEVICE)) {
        size_t cap_bytes = c->dout_cap * sizeof(hac_merge);
        rc = ensure_dev(c, reinterpret_cast<void **>(&c->dout), &cap_bytes, (size_t)(n - 1) * sizeof(hac_merge),
                        "merge buffer");
        if (rc) return rc;
        c->dout_cap = cap_bytes / sizeof(hac_merge);
        dev_out = c->dout;
    }
    hac::Instance inst{};
    inst.D = D;
    inst.out = dev_out;
    inst.rowkey = reinterpret_cast<uint64_t *>(ws + rk_off);
    inst.status = reinterpret_cast<uint32_t *>(ws + st_off);
    inst.n = n;
    inst.link = linkage;
    HIP_TRY(c, hipEventRecord(c->ev[0], s));
    HIP_TRY(c, hac::launch_zero(ws, (st_off + st_bytes) / 4, s));
    HIP_TRY(c, hac::launch_zero(ws + ro_off + Lo.ctl, sizeof(hac::RoundsCtl) / 4, s));
    if (sl_bytes) HIP_TRY(c, hac::launch_zero(ws + sl_off, sl_bytes / 4, s));
    HIP_TRY(c, hac::launch_setup(inst, dist, s));
    HIP_TRY(c, hipEventRecord(c->ev[1], s));
    const int rflags = (c->opt_profile ? hac::kFlagProfile : 0) | (handover ? 0 : hac::kFlagNoHandover) |
                       (c->opt_stall ? hac::kFlagStall : 0);
    hac::Control *ctl = reinterpret_cast<hac::Control *>(ws);
    hipError_t e = hac::launch_rounds(D, n, linkage, inst.status, ctl, ws + ro_off, G, timeout_ticks(c), rflags, s);
    if (e != hipSuccess) return hip_fail(c, e, "round kernel launch");
    HIP_TRY(c, hipEventRecord(c->ev[3], s));
    if (handover) {
        // Resumes from the round engine's state if it hands over; its
        // records join the round engine's before they are sorted.
        hac::Instance seq = inst;
        seq.out = hac::rounds_records(n, G, ws + ro_off);
        seq.slots = reinterpret_cast<uint64_t *>(ws + sl_off);
        seq.exchange = (int32_t)c->opt_exchange;
        seq.flags = seq_flags | hac::kFlagAfterRounds;
        e = hac::launch_merge(seq, g, block, ctl, timeout_ticks(c), s, hac::rounds_resume(n, G, ws + ro_off));
        if (e != hipSuccess) return hip_fail(c, e, "merge kernel launch");
    }
    e = hac::launch_rank(n, dev_out, inst.status, ctl, ws + ro_off, G, s);
    if (e != hipSuccess) return hip_fail(c, e, "record sort launch");
    HIP_TRY(c, hipEventRecord(c->ev[2], s));
    c->pending_wgs = G;
    c->pending_block = hac::kRoundsBlock;
    c->pending_group = G;
    c->pending_graph = 0;
    c->pending_plan_source = c->pending_plan_share = c->pending_plan_upd = 0;
    c->pending_deferred = 0;
    c->pending_rounds = true;
    c->pending_seq_wgs = g;
    c->pending_seq_block = block;
    c->pending_seq_deferred = (seq_flags & hac::kFlagDefer) ? 1 : 0;
    return finish(c, s, 1, out, (flags & HAC_OUT_DEVICE) ? 0 : (size_t)(n - 1), flags, ws);
}

// hac_run with HAC_MODE_SCAN: the scan engine over every CU.
int run_scan(hac_ctx *c, float *dist, int32_t n, int32_t linkage, hac_merge *out, uint32_t flags, hipStream_t s) {
    if (!c->coop) return fail(c, HAC_EDEVICE, "device does not support cooperative launch");
    if (hac::scan_lds_bytes(n) > c->lds_max) return fail(c, HAC_EINVAL, "n=%d does not fit in LDS", n);
    int G = c->cus * hac::scan_occupancy(n);
    if (c->opt_wgs > 0) G = std::min(G, (int)c->opt_wgs);
    // Workspace: control | status | first upper row minima (set-up kernel) | scan engine.
    const size_t ctl_bytes = align_up(sizeof(hac::Control), kAlign);
    const size_t st_off = ctl_bytes, st_bytes = kAlign;
    const size_t rk_off = st_off + st_bytes, rk_bytes = align_up((size_t)n * 8, kAlign);
    const size_t sc_off = rk_off + rk_bytes;
    const hac::ScanLayout Lo = hac::scan_layout(n, G);
    int rc = ensure_dev(c, &c->ws, &c->ws_cap, sc_off + Lo.bytes, "workspace");
    if (rc) return rc;
    rc = ensure_dev(c, reinterpret_cast<void **>(&c->spare), &c->spare_cap, hac::scan_spare_floats(n) * 4,
                    "scan buffer");
    if (rc) return rc;
    rc = ensure_pinned(c, ctl_bytes + kAlign);
    if (rc) return rc;
    char *ws = reinterpret_cast<char *>(c->ws);
    float *D = dist;
    if (flags & HAC_PRESERVE_INPUT) {
        rc = ensure_dev(c, reinterpret_cast<void **>(&c->dcopy), &c->dcopy_cap, (size_t)n * n * 4, "input copy");
        if (rc) return rc;
        D = c->dcopy;
    }
    hac_merge *dev_out = out;
    if (!(flags & HAC_OUT_DEVICE)) {
        size_t cap_bytes = c->dout_cap * sizeof(hac_merge);
        rc = ensure_dev(c, reinterpret_cast<void **>(&c->dout), &cap_bytes, (size_t)(n - 1) * sizeof(hac_merge),
                        "merge buffer");
        if (rc) return rc;
        c->dout_cap = cap_bytes / sizeof(hac_merge);
        dev_out = c->dout;
    }
    hac::Instance inst{};
    inst.D = D;
    inst.out = dev_out;
    inst.rowkey = reinterpret_cast<uint64_t *>(ws + rk_off);
    inst.status = reinterpret_cast<uint32_t *>(ws + st_off);
    inst.n = n;
    inst.link = linkage;
    hac::Control *ctl = reinterpret_cast<hac::Control *>(ws);
    HIP_TRY(c, hipEventRecord(c->ev[0], s));
    HIP_TRY(c, hac::launch_zero(ws, (st_off + st_bytes) / 4, s));
    HIP_TRY(c, hac::launch_zero(ws + sc_off + Lo.ctl, sizeof(hac::ScanCtl) / 4, s));
    HIP_TRY(c, hac::launch_setup(inst, dist, s));
    HIP_TRY(c, hipEventRecord(c->ev[1], s));
    hipError_t e = hac::launch_scan(D, c->spare, n, linkage, dev_out, inst.status, ctl, ws + sc_off, G,
                                    timeout_ticks(c), c->opt_stall ? hac::kFlagStall : 0, s);
    if (e != hipSuccess) return hip_fail(c, e, "scan kernel launch");
    HIP_TRY(c, hipEventRecord(c->ev[2], s));
    c->pending_wgs = G;
    c->pending_block = hac::kScanBlock;
    c->pending_group = G;
    c->pending_graph = 0;
    c->pending_plan_source = c->pending_plan_share = c->pending_plan_upd = 0;
    c->pending_deferred = 0;
    c->pending_scan = true;
    return finish(c, s, 1, out, (flags & HAC_OUT_DEVICE) ? 0 : (size_t)(n - 1), flags, ws);
}

// hac_run and hac_run_noalloc.  noalloc: the device scratch is the static
// array (c->scratch) instead of the context's workspace, the merge kernel
// runs on at most HAC_NOALLOC_MAX_WORKGROUPS workgroups, out is device
// memory, and nothing is allocated (the caller has rejected
// HAC_PRESERVE_INPUT).
int run_impl(hac_ctx *c, float *dist, int32_t n, int32_t linkage, hac_merge *out, uint32_t flags, void *stream,
             bool noalloc) {
    int rc = set_device(c);
    if (rc) return rc;
    if (c->pending) {
        rc = hac_sync(c);
        (void)rc;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    c->stats = hac_stats{};
    c->pending_rounds = false;
    c->pending_scan = false;
    if (n == 1) return HAC_OK;
    if (!noalloc && !(flags & HAC_MODE_SCAN) && (linkage == HAC_SINGLE || linkage == HAC_COMPLETE) &&
        (c->opt_rounds == 2 || (c->opt_rounds == 1 && n >= kRoundsMinN)))
        return run_rounds(c, dist, n, linkage, out, flags, s);
    if (!noalloc && (flags & HAC_MODE_SCAN)) return run_scan(c, dist, n, linkage, out, flags, s);

    int g = 1, block = hac::kRunBlock;
    int32_t run_flags = 0;
    rc = plan_seq(c, n, flags, noalloc, &g, &block, &run_flags);
    if (rc) return rc;

    // Workspace: control | status | first row minima | slots.
    const size_t ctl_bytes = align_up(sizeof(hac::Control), kAlign);
    const size_t st_off = ctl_bytes, st_bytes = kAlign;
    const size_t rk_off = st_off + st_bytes, rk_bytes = align_up((size_t)n * 8, kAlign);
    const size_t sl_off = rk_off + rk_bytes;
    const size_t sl_bytes = g > 1 ? (size_t)2 * (g + 1) * hac::kSlotStride * 8 : 0;
    char *ws = nullptr;
    if (noalloc) {
        // Fits by construction (n <= HAC_NOALLOC_MAX_N, g <= HAC_NOALLOC_MAX_WORKGROUPS);
        // the pinned staging was allocated by hac_create.
        if (sl_off + sl_bytes > hac::kNoAllocScratchBytes || ctl_bytes + kAlign > c->pinned_cap)
            return fail(c, HAC_EINVAL, "n=%d on %d workgroups exceeds the static scratch", n, g);
        ws = static_cast<char *>(c->scratch);
    } else {
        rc = ensure_dev(c, &c->ws, &c->ws_cap, sl_off + sl_bytes, "workspace");
        if (rc) return rc;
        rc = ensure_pinned(c, ctl_bytes + kAlign);
        if (rc) return rc;
        ws = reinterpret_cast<char *>(c->ws);
    }

    // With HAC_PRESERVE_INPUT the set-up kernel reads the caller's matrix and
    // writes both triangles of the library's working copy (no separate copy).
    float *D = dist;
    if (flags & HAC_PRESERVE_INPUT) {
        const size_t bytes = (size_t)n * n * 4;
        rc = ensure_dev(c, reinterpret_cast<void **>(&c->dcopy), &c->dcopy_cap, bytes, "input copy");
        if (rc) return rc;
        D = c->dcopy;
    }
    hac_merge *dev_out = out;
    if (!noalloc && !(flags & HAC_OUT_DEVICE)) {
        size_t cap_bytes = c->dout_cap * sizeof(hac_merge);
        rc = ensure_dev(c, reinterpret_cast<void **>(&c->dout), &cap_bytes, (size_t)(n - 1) * sizeof(hac_merge), "merge buffer");
        if (rc) return rc;
        c->dout_cap = cap_bytes / sizeof(hac_merge);
        dev_out = c->dout;
    }

    hac::Instance inst;
    inst.D = D;
    inst.out = dev_out;
    inst.rowkey = reinterpret_cast<uint64_t *>(ws + rk_off);
    inst.slots = reinterpret_cast<uint64_t *>(ws + sl_off);
    inst.status = reinterpret_cast<uint32_t *>(ws + st_off);
    inst.n = n;
    inst.link = linkage;
    inst.exchange = (int32_t)c->opt_exchange;
    inst.flags = run_flags;
    hac::Control *ctl = reinterpret_cast<hac::Control *>(ws);

    // Everything that must start at zero is cleared by fill kernels (no
    // memset): control block and status, the exchange slots; the set-up
    // kernel's row minima are filled by launch_run.
    HIP_TRY(c, hipEventRecord(c->ev[0], s));
    HIP_TRY(c, hac::launch_zero(ws, (st_off + st_bytes) / 4, s));
    if (sl_bytes) HIP_TRY(c, hac::launch_zero(ws + sl_off, sl_bytes / 4, s));
    hipError_t e = hac::launch_run(inst, dist, g, block, ctl, timeout_ticks(c), s, c->ev[1]);
    if (e != hipSuccess) return hip_fail(c, e, "merge kernel launch");
    HIP_TRY(c, hipEventRecord(c->ev[2], s));
    c->pending_wgs = g;
    c->pending_block = block;
    c->pending_group = g;
    c->pending_graph = 0;
    c->pending_plan_source = c->pending_plan_share = c->pending_plan_upd = 0;
    c->pending_deferred = (run_flags & hac::kFlagDefer) ? 1 : 0;
    if (noalloc) return finish(c, s, 1, nullptr, 0, flags, ws);
    return finish(c, s, 1, out, (flags & HAC_OUT_DEVICE) ? 0 : (size_t)(n - 1), flags, ws);
}

}  // namespace

extern "C" {

int hac_run(hac_ctx *c, float *dist, int32_t n, int32_t linkage, hac_merge *out, uint32_t flags,
            void *stream) {
    if (!c) return HAC_EINVAL;
    c->err.clear();
    char msg[192];
    int rc = hac::check_run_args(dist, n, linkage, out, flags, HAC_PRESERVE_INPUT | HAC_OUT_DEVICE | HAC_MODE_SCAN,
                                 HAC_MAX_N, msg, sizeof msg);
    if (rc) return checked(c, rc, msg);
    return run_impl(c, dist, n, linkage, out, flags, stream, false);
}

int hac_run_noalloc(hac_ctx *c, float *dist, int32_t n, int32_t linkage, hac_merge *out, uint32_t flags,
                    void *stream) {
    if (!c) return HAC_EINVAL;
    c->err.clear();
    if (flags & HAC_PRESERVE_INPUT)
        return fail(c, HAC_EINVAL, "HAC_PRESERVE_INPUT needs an n*n workspace; hac_run_noalloc allocates none");
    if (n > HAC_NOALLOC_MAX_N)
        return fail(c, HAC_EINVAL, "n=%d outside 1..%d (the static scratch holds the row minima of at most %d items)",
                    n, HAC_NOALLOC_MAX_N, HAC_NOALLOC_MAX_N);
    char msg[192];
    const int rc = hac::check_run_args(dist, n, linkage, out, flags, HAC_OUT_DEVICE | HAC_MODE_SCAN,
                                       HAC_NOALLOC_MAX_N, msg, sizeof msg);
    if (rc) return checked(c, rc, msg);
    if (!c->scratch) return fail(c, HAC_EDEVICE, "no static scratch on this device");
    return run_impl(c, dist, n, linkage, out, flags, stream, true);
}

int hac_batch(hac_ctx *c, float *packed, const int64_t *offsets, const int32_t *ns,
              const int32_t *linkages, int32_t count, hac_merge *out, const int64_t *out_offsets,
              uint32_t flags, void *stream) {
    if (!c) return HAC_EINVAL;
    c->err.clear();
    if (count < 0) return fail(c, HAC_EINVAL, "count=%d", count);
    if (count == 0) return HAC_OK;
    int64_t extent = 0, rec_extent = 0;
    char msg[192];
    int rc = hac::check_batch_args(packed, offsets, ns, linkages, count, out, out_offsets, flags, &extent,
                                   &rec_extent, msg, sizeof msg);
    if (rc) return checked(c, rc, msg);
    rc = set_device(c);
    if (rc) return rc;
    if (c->pending) (void)hac_sync(c);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    c->stats = hac_stats{};

    float *base = packed;
    if (flags & HAC_PRESERVE_INPUT) {
        const size_t bytes = (size_t)extent * 4;
        rc = ensure_dev(c, reinterpret_cast<void **>(&c->dcopy), &c->dcopy_cap, bytes, "input copy");
        if (rc) return rc;
        HIP_TRY(c, hipMemcpyAsync(c->dcopy, packed, bytes, hipMemcpyDeviceToDevice, s));
        base = c->dcopy;
    }
    hac_merge *dev_out = out;
    if (!(flags & HAC_OUT_DEVICE)) {
        size_t cap_bytes = c->dout_cap * sizeof(hac_merge);
        rc = ensure_dev(c, reinterpret_cast<void **>(&c->dout), &cap_bytes,
                        (size_t)std::max<int64_t>(rec_extent, 1) * sizeof(hac_merge), "merge buffer");
        if (rc) return rc;
        c->dout_cap = cap_bytes / sizeof(hac_merge);
        dev_out = c->dout;
    }

    // Plan: forced by options, cached for this size mix, or tuned now.
    BatchPlan plan;
    int plan_source = 0;  // 0: default or forced by options, 1: tuned now, 2: tuned earlier (cached)
    if (c->opt_batch_block > 0 || c->opt_batch_group > 0 || c->opt_batch_upd > 0) {
        if (c->opt_batch_block > 0) plan.block = (int)c->opt_batch_block;
        if (c->opt_batch_group > 0) plan.group = (int)c->opt_batch_group;
        plan.upd = (int)c->opt_batch_upd;
    } else {
        const std::string sig = batch_signature(ns, linkages, count);
        auto it = c->plans.find(sig);
        if (it != c->plans.end()) {
            plan = it->second;
            plan_source = 2;
        } else if (c->opt_autotune && count >= 8) {
            rc = batch_autotune(c, base, extent, offsets, ns, linkages, count, dev_out, out_offsets, s, &plan);
            if (rc) return rc;
            c->plans[sig] = plan;
            plan_source = 1;
        }
    }

    BatchLayout B;
    rc = batch_prepare(c, base, offsets, ns, linkages, count, dev_out, out_offsets, plan, s, &B);
    if (rc) return rc;
    HIP_TRY(c, hipEventRecord(c->ev[0], s));
    int graphed = 0;
    if (c->opt_graph) {
        HIP_TRY(c, hipEventRecord(c->ev[1], s));
        // One executable graph per layout; descriptors are re-read from the
        // pinned buffer at every launch.
        char key[256];
        snprintf(key, sizeof key, "%p:%zu:%zu:%zu:%zu:%d:%d:%d:%d:%zu:%llu", c->ws, B.in_off, B.up_bytes, B.st_off + B.st_bytes,
                 B.sl_bytes, B.L.count, B.L.ngroups, B.L.block * 16 + B.L.upd, B.L.grid, B.L.lds,
                 (unsigned long long)timeout_ticks(c));
        auto it = c->graphs.find(key);
        if (it == c->graphs.end()) {
            if (c->graphs.size() >= 16) clear_graphs(c);
            char *ws = reinterpret_cast<char *>(c->ws);
            hipGraphExec_t ex = nullptr;
            hipError_t ge = hac::build_batch_graph(B.L, reinterpret_cast<hac::Control *>(ws), timeout_ticks(c),
                                                   ws + B.in_off, c->pinned, B.up_bytes, ws,
                                                   (B.st_off + B.st_bytes) / 4, ws + B.sl_off, B.sl_bytes / 4, &ex);
            if (ge != hipSuccess) return hip_fail(c, ge, "building the batch graph");
            it = c->graphs.emplace(key, ex).first;
            graphed = 2;
        } else {
            graphed = 1;
        }
        HIP_TRY(c, hipGraphLaunch(it->second, s));
    } else {
        hipError_t e = batch_enqueue(c, B, s, c->ev[1]);
        if (e != hipSuccess) return hip_fail(c, e, "batch kernel launch");
    }
    HIP_TRY(c, hipEventRecord(c->ev[2], s));
    c->pending_wgs = B.L.grid;
    c->pending_block = plan.block;
    c->pending_group = B.group;
    c->pending_plan_source = plan_source;
    c->pending_plan_share = B.group > 1 ? plan.share : 0;
    c->pending_plan_upd = plan_update(plan);
    c->pending_graph = graphed;
    c->pending_deferred = 1;
    c->pending_rounds = false;
    c->pending_scan = false;
    return finish(c, s, count, out, (flags & HAC_OUT_DEVICE) ? 0 : (size_t)rec_extent, flags, c->ws);
}

}  // extern "C"
