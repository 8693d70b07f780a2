// C-ABI layer of the clustering library (declared in include/hac.h):
// argument checks, device workspace, choice of launch shape, status read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "hac.h"
#include "hac_engine.h"

namespace {

constexpr size_t kAlign = 256;
constexpr int kDefaultSingleWgN = 1536;
constexpr int64_t kDefaultTimeoutMs = 10000;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

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
    float *dcopy = nullptr;      // HAC_PRESERVE_INPUT copy
    size_t dcopy_cap = 0;        // bytes
    hac_merge *dout = nullptr;   // device merge records when the caller's out is host memory
    size_t dout_cap = 0;         // records
    void *pinned = nullptr;      // host staging (status read-back, descriptor upload)
    size_t pinned_cap = 0;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};

    hac_stats stats{};
    int64_t opt_wgs = 0, opt_single_n = 0, opt_timeout_ms = 0, opt_exchange = 0, opt_profile = 0;
    int64_t opt_block = 0;

    // State of the last enqueued call, for hac_sync / stats.
    bool pending = false;
    hipStream_t pending_stream = nullptr;
    int pending_count = 0;           // status words to check
    int pending_wgs = 0;
};

namespace {

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

uint64_t timeout_ticks(const hac_ctx *c) {
    int64_t ms = c->opt_timeout_ms > 0 ? c->opt_timeout_ms : kDefaultTimeoutMs;
    return (uint64_t)ms * (uint64_t)(c->wallclock_khz > 0 ? c->wallclock_khz : 100000);
}

// Workgroups that can be co-resident for a hac_run launch with `lds` bytes.
int max_coresident(hac_ctx *c, size_t lds, int block) {
    int per_cu = hac::engine_occupancy(lds, block);
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
    c->stats.workgroups = c->pending_wgs;
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
int finish(hac_ctx *c, hipStream_t s, int nstatus, hac_merge *out, size_t nrec, uint32_t flags) {
    const size_t ctl_bytes = align_up(sizeof(hac::Control), kAlign);
    HIP_TRY(c, hipMemcpyAsync(c->pinned, c->ws, ctl_bytes + (size_t)nstatus * 4, hipMemcpyDeviceToHost, s));
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
    *out = c;
    return HAC_OK;
}

int hac_destroy(hac_ctx *c) {
    if (!c) return HAC_OK;
    (void)hipSetDevice(c->device);
    if (c->own) (void)hipStreamSynchronize(c->own);
    (void)hipDeviceSynchronize();
    if (c->ws) (void)hipFree(c->ws);
    if (c->dcopy) (void)hipFree(c->dcopy);
    if (c->dout) (void)hipFree(c->dout);
    if (c->pinned) (void)hipHostFree(c->pinned);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->own) (void)hipStreamDestroy(c->own);
    delete c;
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

int hac_run(hac_ctx *c, float *dist, int32_t n, int32_t linkage, hac_merge *out, uint32_t flags,
            void *stream) {
    if (!c) return HAC_EINVAL;
    c->err.clear();
    if (!dist) return fail(c, HAC_EINVAL, "dist is NULL");
    if (n < 1 || n > HAC_MAX_N) return fail(c, HAC_EINVAL, "n=%d outside 1..%d", n, HAC_MAX_N);
    if (linkage < 0 || linkage > 3) return fail(c, HAC_EINVAL, "linkage %d is not 0..3", linkage);
    if (flags & ~(HAC_PRESERVE_INPUT | HAC_OUT_DEVICE)) return fail(c, HAC_EINVAL, "unknown flags 0x%x", flags);
    if (n > 1 && !out) return fail(c, HAC_EINVAL, "out is NULL");
    int rc = set_device(c);
    if (rc) return rc;
    if (c->pending) {
        rc = hac_sync(c);
        (void)rc;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    c->stats = hac_stats{};
    if (n == 1) return HAC_OK;

    // Launch shape: one workgroup for small n, else a co-resident group of
    // a few large workgroups (each merge costs every workgroup one agent-scope
    // release/acquire pair, so fewer workgroups mean a cheaper exchange).
    const int nch = (n + 63) / 64;
    const int block = c->opt_block > 0 ? (int)c->opt_block : hac::kRunBlock;
    const int single_n = c->opt_single_n > 0 ? (int)c->opt_single_n : kDefaultSingleWgN;
    int g = 1;
    if (n > single_n || hac::lds_bytes(n, hac::own_rows(n, 1), false) > c->lds_max) {
        // Measured on MI355X: about one workgroup per 512 items, up to 64.
        int want = c->opt_wgs > 0 ? (int)c->opt_wgs : std::max(2, std::min(64, n / 512));
        g = std::max(1, std::min(want, nch));
        while (g < nch && hac::lds_bytes(n, hac::own_rows(n, g), false) > c->lds_max) ++g;
        const size_t lds = hac::lds_bytes(n, hac::own_rows(n, g), false);
        if (lds > c->lds_max) return fail(c, HAC_EINVAL, "n=%d does not fit in LDS", n);
        const int cap = max_coresident(c, lds, block);
        if (g > cap) g = cap;
        if (hac::lds_bytes(n, hac::own_rows(n, g), false) > c->lds_max)
            return fail(c, HAC_EDEVICE, "n=%d needs more co-resident workgroups than the device holds", n);
        if (g > 1 && !c->coop) return fail(c, HAC_EDEVICE, "device does not support cooperative launch");
    }

    // Workspace: control | status | first row minima | slots.
    const size_t ctl_bytes = align_up(sizeof(hac::Control), kAlign);
    const size_t st_off = ctl_bytes, st_bytes = kAlign;
    const size_t rk_off = st_off + st_bytes, rk_bytes = align_up((size_t)n * 8, kAlign);
    const size_t sl_off = rk_off + rk_bytes;
    const size_t sl_bytes = g > 1 ? (size_t)2 * (g + 1) * hac::kSlotStride * 8 : 0;
    rc = ensure_dev(c, &c->ws, &c->ws_cap, sl_off + sl_bytes, "workspace");
    if (rc) return rc;
    rc = ensure_pinned(c, ctl_bytes + kAlign);
    if (rc) return rc;

    float *D = dist;
    if (flags & HAC_PRESERVE_INPUT) {
        const size_t bytes = (size_t)n * n * 4;
        rc = ensure_dev(c, reinterpret_cast<void **>(&c->dcopy), &c->dcopy_cap, bytes, "input copy");
        if (rc) return rc;
        HIP_TRY(c, hipMemcpyAsync(c->dcopy, dist, bytes, hipMemcpyDeviceToDevice, s));
        D = c->dcopy;
    }
    hac_merge *dev_out = out;
    if (!(flags & HAC_OUT_DEVICE)) {
        size_t cap_bytes = c->dout_cap * sizeof(hac_merge);
        rc = ensure_dev(c, reinterpret_cast<void **>(&c->dout), &cap_bytes, (size_t)(n - 1) * sizeof(hac_merge), "merge buffer");
        if (rc) return rc;
        c->dout_cap = cap_bytes / sizeof(hac_merge);
        dev_out = c->dout;
    }

    char *ws = reinterpret_cast<char *>(c->ws);
    hac::Instance inst;
    inst.D = D;
    inst.out = dev_out;
    inst.rowkey = reinterpret_cast<uint64_t *>(ws + rk_off);
    inst.slots = reinterpret_cast<uint64_t *>(ws + sl_off);
    inst.status = reinterpret_cast<uint32_t *>(ws + st_off);
    inst.n = n;
    inst.link = linkage;
    inst.exchange = (int32_t)c->opt_exchange;
    inst.flags = c->opt_profile ? hac::kFlagProfile : 0;
    hac::Control *ctl = reinterpret_cast<hac::Control *>(ws);

    HIP_TRY(c, hipEventRecord(c->ev[0], s));
    HIP_TRY(c, hac::launch_zero(ws, (st_off + st_bytes) / 4, s));
    if (sl_bytes) HIP_TRY(c, hac::launch_zero(ws + sl_off, sl_bytes / 4, s));
    hipError_t e = hac::launch_run(inst, g, block, ctl, timeout_ticks(c), s, c->ev[1]);
    if (e != hipSuccess) return hip_fail(c, e, "merge kernel launch");
    HIP_TRY(c, hipEventRecord(c->ev[2], s));
    c->pending_wgs = g;
    return finish(c, s, 1, out, (flags & HAC_OUT_DEVICE) ? 0 : (size_t)(n - 1), flags);
}

int hac_batch(hac_ctx *c, float *packed, const int64_t *offsets, const int32_t *ns,
              const int32_t *linkages, int32_t count, hac_merge *out, const int64_t *out_offsets,
              uint32_t flags, void *stream) {
    if (!c) return HAC_EINVAL;
    c->err.clear();
    if (count < 0) return fail(c, HAC_EINVAL, "count=%d", count);
    if (count == 0) return HAC_OK;
    if (!packed || !offsets || !ns || !linkages || !out || !out_offsets)
        return fail(c, HAC_EINVAL, "NULL argument");
    if (flags & ~(HAC_PRESERVE_INPUT | HAC_OUT_DEVICE)) return fail(c, HAC_EINVAL, "unknown flags 0x%x", flags);
    int64_t extent = 0, rec_extent = 0;
    int nmax = 1;
    for (int k = 0; k < count; ++k) {
        if (ns[k] < 1 || ns[k] > HAC_MAX_BATCH_N)
            return fail(c, HAC_EINVAL, "instance %d: n=%d outside 1..%d", k, ns[k], HAC_MAX_BATCH_N);
        if (linkages[k] < 0 || linkages[k] > 3) return fail(c, HAC_EINVAL, "instance %d: linkage %d", k, linkages[k]);
        if (offsets[k] < 0 || out_offsets[k] < 0) return fail(c, HAC_EINVAL, "instance %d: negative offset", k);
        extent = std::max(extent, offsets[k] + (int64_t)ns[k] * ns[k]);
        rec_extent = std::max(rec_extent, out_offsets[k] + (int64_t)ns[k] - 1);
        nmax = std::max(nmax, (int)ns[k]);
    }
    const size_t lds = hac::lds_bytes(nmax, hac::own_rows(nmax, 1), true);
    if (lds > c->lds_max) return fail(c, HAC_EINVAL, "n=%d does not fit one workgroup's LDS", nmax);
    int rc = set_device(c);
    if (rc) return rc;
    if (c->pending) (void)hac_sync(c);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    c->stats = hac_stats{};

    const size_t ctl_bytes = align_up(sizeof(hac::Control), kAlign);
    const size_t st_off = ctl_bytes, st_bytes = align_up((size_t)count * 4, kAlign);
    const size_t in_off = st_off + st_bytes, in_bytes = align_up((size_t)count * sizeof(hac::Instance), kAlign);
    const size_t or_off = in_off + in_bytes, or_bytes = align_up((size_t)count * 4, kAlign);
    rc = ensure_dev(c, &c->ws, &c->ws_cap, or_off + or_bytes, "workspace");
    if (rc) return rc;
    rc = ensure_pinned(c, std::max(ctl_bytes + st_bytes, in_bytes + or_bytes));
    if (rc) return rc;

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

    // Descriptors, and the longest-processing-time-first order (largest n first).
    char *ws = reinterpret_cast<char *>(c->ws);
    // The pinned buffer is reused below for the read-back; make sure no
    // earlier copy out of it is still pending.
    HIP_TRY(c, hipStreamSynchronize(s));
    hac::Instance *hin = reinterpret_cast<hac::Instance *>(c->pinned);
    int32_t *hord = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(c->pinned) + in_bytes);
    for (int k = 0; k < count; ++k) {
        hac::Instance &I = hin[k];
        I.D = base + offsets[k];
        I.out = dev_out + out_offsets[k];
        I.rowkey = nullptr;
        I.slots = nullptr;
        I.status = reinterpret_cast<uint32_t *>(ws + st_off) + k;
        I.n = ns[k];
        I.link = linkages[k];
        I.exchange = 0;
        I.flags = c->opt_profile ? hac::kFlagProfile : 0;
    }
    std::vector<int32_t> ord(count);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return ns[a] > ns[b]; });
    std::memcpy(hord, ord.data(), (size_t)count * 4);
    HIP_TRY(c, hipMemcpyAsync(ws + in_off, c->pinned, in_bytes + or_bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipStreamSynchronize(s));

    HIP_TRY(c, hipEventRecord(c->ev[0], s));
    HIP_TRY(c, hac::launch_zero(ws, (st_off + st_bytes) / 4, s));
    HIP_TRY(c, hipEventRecord(c->ev[1], s));
    int per_cu = std::max(1, hac::engine_occupancy(lds, 0));
    int grid = std::min(count, per_cu * c->cus);
    hipError_t e = hac::launch_batch(reinterpret_cast<hac::Instance *>(ws + in_off),
                                     reinterpret_cast<int32_t *>(ws + or_off), count, grid, lds,
                                     reinterpret_cast<hac::Control *>(ws), timeout_ticks(c), s);
    if (e != hipSuccess) return hip_fail(c, e, "batch kernel launch");
    HIP_TRY(c, hipEventRecord(c->ev[2], s));
    c->pending_wgs = grid;
    return finish(c, s, count, out, (flags & HAC_OUT_DEVICE) ? 0 : (size_t)rec_extent, flags);
}

}  // extern "C"
