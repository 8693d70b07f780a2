// Serving layer of the clustering library (declared in include/hac.h):
// an HBM arena with a first-fit allocator, in-order admission under the
// arena budget, publication of jobs to the persistent serving kernel through
// a ring in fine-grained host memory, and completion, all driven by one host
// thread per server.  While the kernel runs the host enqueues nothing on the
// device: the kernel reads each job's matrix from page-locked host memory
// itself and writes its merge records into page-locked host memory, so no
// copy waits behind the persistent kernel in a shared hardware queue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "hac.h"
#include "hac_arena.h"
#include "hac_ctx_info.h"
#include "hac_engine.h"
#include "hac_validate.h"

namespace {

constexpr size_t kAlign = 256;
constexpr uint32_t kRingCap = 16384;       // entries; >= max_jobs * largest group
constexpr int kMaxJobs = 4096;
constexpr int kMaxGroup = 64;
constexpr int kGroupN = 2048;              // jobs above this size run on a group
constexpr int kPolicyMaxGroup = 16;        // largest group chosen for latency alone
constexpr int kLargeN = 32768;             // above this, a job gets kMaxGroup workgroups (as hac_run)
constexpr int kIdleStopMs = 20;            // stop the kernel after this long with nothing to do
constexpr int kXcds = 8;                   // accelerator complex dies of an MI355X
constexpr int64_t kServeTimeoutMs = 120000;  // watchdog of waits inside the kernel
constexpr int64_t kSelfStopMs = 60000;     // kernel idle this long stops without the host

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

enum class JobState { kFree, kWaiting, kRunning, kDone };

// Bytes of one job: device matrix; page-locked records; staging copy of a
// pageable input.
struct JobLayout {
    size_t bytes, rec_bytes, stage_bytes;
};

JobLayout job_layout(int n) {
    JobLayout L;
    L.bytes = align_up((size_t)n * n * 4, kAlign);
    L.rec_bytes = align_up((size_t)std::max(n - 1, 1) * sizeof(hac_merge), kAlign);
    L.stage_bytes = L.bytes;
    return L;
}

struct Job {
    JobState state = JobState::kFree;
    uint32_t seq = 0;  // changes every time the slot is reused; never 0 once used
    const float *host = nullptr;
    const float *src_dev = nullptr;  // device address of page-locked input, or null (staged)
    int64_t ld = 0;
    int32_t n = 0, link = 0, g = 1;
    bool lazy = false;               // kFlagLazy: the step table fits the server's LDS
    size_t off = 0;                  // arena: matrix
    size_t rec_off = 0;              // records area
    size_t stage_off = 0;            // staging area (pageable input only)
    bool staged = false;
    JobLayout lay{};
    int rc = HAC_OK;
    std::vector<hac_merge> result;
};

}  // namespace

struct hac_server {
    hac::CtxInfo info{};
    size_t budget = 0;
    int max_n = 0, block = 1024, grid = 0;
    size_t lds = 0;
    uint64_t timeout = 0, idle_ticks = 0;

    char *arena = nullptr;
    hac::Arena alloc;
    size_t in_use = 0, peak = 0;
    char *recs = nullptr;      // page-locked: merge records of admitted jobs
    size_t recs_bytes = 0;
    hac::Arena recs_alloc;
    char *stage = nullptr;     // page-locked: copies of pageable inputs
    size_t stage_bytes = 0;
    hac::Arena stage_alloc;
    void *recs_dev = nullptr, *stage_dev = nullptr;  // device addresses of recs, stage
    hipStream_t kern = nullptr;
    hipEvent_t kern_done = nullptr;
    bool kern_running = false;
    int64_t launches = 0;
    uint64_t stopped_at = 0;  // entries consumed when the kernel last stopped

    char *hostmem = nullptr;  // fine-grained host memory: ServeHost | ring | done[]
    hac::ServeHost *host = nullptr;
    hac::ServeEntry *ring = nullptr;
    unsigned long long *done = nullptr;
    hac::ServeHost *host_dev = nullptr;  // the same memory as the device addresses it
    hac::ServeEntry *ring_dev = nullptr;
    unsigned long long *done_dev = nullptr;
    char *jobwords = nullptr;  // device: per job slot, status | members done | exchange slots
    size_t jobwords_stride = 0;
    int max_group = 1;
    uint64_t published = 0;
    std::vector<uint64_t> ring_owner;  // (id << 32 | seq) of each ring slot's job, 0 = none
    char *dev = nullptr;               // device: ServeDev | Control
    size_t dev_bytes = 0;
    char *pinned = nullptr;            // page-locked: launch image of dev

    std::vector<Job> jobs;
    std::vector<uint32_t> free_ids;
    std::deque<uint32_t> waiting;
    std::vector<uint32_t> running;
    int64_t submitted = 0, completed = 0;

    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool quit = false;
    int failed = HAC_OK;
    std::string err;
    std::chrono::steady_clock::time_point idle_since{}, launched_at{};
};

namespace {

int sfail(hac_server *s, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    s->err = buf;
    return code;
}

// A HIP failure inside the server: every later call reports it.
int sdevice(hac_server *s, hipError_t e, const char *what) {
    s->failed = e == hipErrorOutOfMemory ? HAC_ENOMEM : HAC_EDEVICE;
    return sfail(s, s->failed, "%s: %s", what, hipGetErrorString(e));
}

int pow2_ceil(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Workgroups for a job of n items: a group above kGroupN items for latency
// (kMaxGroup above kLargeN: the n = 65536 job took 0.94 s on the 32 its LDS
// needs, 0.77 s on 64, with the request mix's throughput unchanged), at least
// what the per-workgroup LDS requires.
int group_for(int n, size_t lds_cap) {
    int g = 1;
    if (n > kGroupN) g = n > kLargeN ? kMaxGroup : std::min(kPolicyMaxGroup, pow2_ceil(n / kGroupN));
    while (g < kMaxGroup && hac::lds_bytes(n, hac::own_rows(n, g), true) > lds_cap) g <<= 1;
    return g;
}

size_t page_bytes(const hac_server *s) {
    return align_up(sizeof(hac::ServeDev), kAlign) + align_up(sizeof(hac::Control), kAlign);
}

// Copy the launch image of the device words (head = tail = entries already
// consumed, no token, no stop, zeroed counters) and launch the kernel.
int launch_kernel(hac_server *s) {
    char *img = s->pinned;
    std::memset(img, 0, page_bytes(s));
    hac::ServeDev *d = reinterpret_cast<hac::ServeDev *>(img);
    d->head = s->stopped_at;
    d->tail = s->stopped_at;
    hipError_t e = hipMemcpyAsync(s->dev, img, page_bytes(s), hipMemcpyHostToDevice, s->kern);
    if (e != hipSuccess) return sdevice(s, e, "serving kernel set-up copy");
    hac::ServeLaunch L;
    L.host = s->host_dev;
    L.ring = s->ring_dev;
    L.cap = kRingCap;
    L.done = s->done_dev;
    L.idle_ticks = s->idle_ticks;
    L.dev = reinterpret_cast<hac::ServeDev *>(s->dev);
    L.block = s->block;
    L.grid = s->grid;
    L.lds = s->lds;
    hac::Control *ctl = reinterpret_cast<hac::Control *>(s->dev + align_up(sizeof(hac::ServeDev), kAlign));
    e = hac::launch_serve(L, ctl, s->timeout, s->kern);
    if (e != hipSuccess) return sdevice(s, e, "serving kernel launch");
    e = hipEventRecord(s->kern_done, s->kern);
    if (e != hipSuccess) return sdevice(s, e, "serving kernel event");
    s->kern_running = true;
    s->launches++;
    s->launched_at = std::chrono::steady_clock::now();
    return HAC_OK;
}

// Ask the kernel to stop (only with nothing outstanding) and wait for it.
int stop_kernel(hac_server *s) {
    if (!s->kern_running) return HAC_OK;
    __atomic_store_n(&s->host->stop, 1u, __ATOMIC_RELEASE);
    hipError_t e = hipEventSynchronize(s->kern_done);
    __atomic_store_n(&s->host->stop, 0u, __ATOMIC_RELEASE);
    s->kern_running = false;
    s->stopped_at = s->published;
    if (e != hipSuccess) return sdevice(s, e, "serving kernel");
    return HAC_OK;
}

bool ring_slot_free(const hac_server *s, uint64_t pos) {
    const uint64_t o = s->ring_owner[pos % kRingCap];
    if (o == 0) return true;
    const Job &J = s->jobs[o >> 32];
    return J.seq != (uint32_t)o || J.state == JobState::kDone || J.state == JobState::kFree;
}

// Device address of page-locked host memory (the same address: page-locked
// allocations are mapped into the device's address space at their host
// address), or null for pageable memory.
const float *device_address(const float *p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (a.type != hipMemoryTypeHost || !a.devicePointer) return nullptr;
    return p;
}

// Admit waiting jobs in arrival order while the arena (and the records and
// staging areas) have room, and publish each to the kernel.
bool admit(hac_server *s) {
    bool any = false;
    while (!s->waiting.empty() && s->failed == HAC_OK) {
        const uint32_t id = s->waiting.front();
        Job &J = s->jobs[id];
        bool room = true;
        for (int r = 0; r < J.g && room; ++r) room = ring_slot_free(s, s->published + r);
        if (!room) break;
        size_t off = 0, roff = 0, soff = 0;
        if (!s->alloc.alloc(J.lay.bytes, &off)) break;
        if (!s->recs_alloc.alloc(J.lay.rec_bytes, &roff)) {
            s->alloc.release(off, J.lay.bytes);
            break;
        }
        if (J.staged && !s->stage_alloc.alloc(J.lay.stage_bytes, &soff)) {
            s->alloc.release(off, J.lay.bytes);
            s->recs_alloc.release(roff, J.lay.rec_bytes);
            break;
        }
        J.off = off;
        J.rec_off = roff;
        J.stage_off = soff;
        const float *src = J.src_dev;
        int64_t ld = J.ld;
        if (J.staged) {
            // Pageable input: copy the n x n block into page-locked staging.
            float *dst = reinterpret_cast<float *>(s->stage + soff);
            for (int r = 0; r < J.n; ++r)
                std::memcpy(dst + (size_t)r * J.n, J.host + (size_t)r * J.ld, (size_t)J.n * 4);
            src = static_cast<const float *>(s->stage_dev) + soff / 4;
            ld = J.n;
        }
        s->in_use += J.lay.bytes;
        s->peak = std::max(s->peak, s->in_use);
        char *base = s->arena + J.off;
        char *words = s->jobwords + (size_t)id * s->jobwords_stride;
        for (int r = 0; r < J.g; ++r) {
            const uint64_t pos = s->published + r;
            hac::ServeEntry &E = s->ring[pos % kRingCap];
            E.inst.D = reinterpret_cast<float *>(base);
            E.inst.out = reinterpret_cast<hac_merge *>(static_cast<char *>(s->recs_dev) + roff);
            E.inst.rowkey = nullptr;
            E.inst.slots = J.g > 1 ? reinterpret_cast<uint64_t *>(words + kAlign) : nullptr;
            E.inst.status = reinterpret_cast<uint32_t *>(words);
            E.inst.n = J.n;
            E.inst.link = J.link;
            E.inst.exchange = 0;
            E.inst.flags = J.lazy ? hac::kFlagLazy : 0;
            E.src = src;
            E.ld = ld;
            E.g = J.g;
            E.rank = r;
            E.job = id;
            E.seq = J.seq;
            s->ring_owner[pos % kRingCap] = ((uint64_t)id << 32) | J.seq;
        }
        s->published += (uint64_t)J.g;
        __atomic_store_n(&s->host->tail, (unsigned long long)s->published, __ATOMIC_RELEASE);
        J.state = JobState::kRunning;
        s->running.push_back(id);
        s->waiting.pop_front();
        any = true;
        if (!s->kern_running && launch_kernel(s) != HAC_OK) break;
    }
    return any;
}

// Collect finished jobs: read back records and status, free the region.
bool collect(hac_server *s) {
    bool any = false;
    for (size_t q = 0; q < s->running.size() && s->failed == HAC_OK;) {
        const uint32_t id = s->running[q];
        Job &J = s->jobs[id];
        const unsigned long long word = __atomic_load_n(&s->done[id], __ATOMIC_ACQUIRE);
        if ((uint32_t)(word >> 32) != J.seq) {
            ++q;
            continue;
        }
        const uint32_t status = (uint32_t)word;
        const hac_merge *rec = reinterpret_cast<const hac_merge *>(s->recs + J.rec_off);
        if (status & hac::kErrInput) {
            J.rc = HAC_EINPUT;
        } else if (status & hac::kErrTimeout) {
            J.rc = HAC_ETIMEDOUT;
            s->failed = HAC_ETIMEDOUT;
            sfail(s, HAC_ETIMEDOUT, "watchdog expired inside the serving kernel");
        } else if (status & hac::kErrInternal) {
            J.rc = HAC_EINTERNAL;
        } else {
            J.rc = HAC_OK;
            J.result.assign(rec, rec + (J.n - 1));
        }
        s->alloc.release(J.off, J.lay.bytes);
        s->recs_alloc.release(J.rec_off, J.lay.rec_bytes);
        if (J.staged) s->stage_alloc.release(J.stage_off, J.lay.stage_bytes);
        s->in_use -= J.lay.bytes;
        J.state = JobState::kDone;
        s->completed++;
        s->running[q] = s->running.back();
        s->running.pop_back();
        any = true;
    }
    return any;
}

void worker_loop(hac_server *s) {
    (void)hipSetDevice(s->info.device);
    std::unique_lock<std::mutex> lk(s->mu);
    s->idle_since = std::chrono::steady_clock::now();
    for (;;) {
        if (s->quit) s->waiting.clear();
        if (s->kern_running && s->failed == HAC_OK) {
            // The kernel stops by itself only after a long idle period.
            const hipError_t q = hipEventQuery(s->kern_done);
            if (q != hipErrorNotReady) {
                s->kern_running = false;
                s->stopped_at = s->published;
                if (q != hipSuccess) sdevice(s, q, "serving kernel");
                else if (!s->running.empty()) {
                    s->failed = HAC_EINTERNAL;
                    // Read the kernel's words back for the report.
                    hac::ServeDev d{};
                    hac::Control ctl{};
                    (void)hipMemcpy(&d, s->dev, sizeof d, hipMemcpyDeviceToHost);
                    (void)hipMemcpy(&ctl, s->dev + align_up(sizeof(hac::ServeDev), kAlign), sizeof ctl,
                                    hipMemcpyDeviceToHost);
                    const double ms = std::chrono::duration<double, std::milli>(
                                          std::chrono::steady_clock::now() - s->launched_at).count();
                    sfail(s, HAC_EINTERNAL,
                          "serving kernel ended with jobs outstanding: %.3f ms after launch %lld; device head %llu "
                          "tail %llu token %u stop %u exits %u self_stops %u claims %llu error %u abort %u; "
                          "host published %llu stopped_at %llu running %zu host stop %u grid %d",
                          ms, (long long)s->launches, d.head, d.tail, d.token, d.stop, d.exits, d.self_stops,
                          d.claims, ctl.error, ctl.abort, (unsigned long long)s->published,
                          (unsigned long long)s->stopped_at, s->running.size(), s->host->stop, s->grid);
                }
            }
        }
        bool progressed = false;
        if (s->failed == HAC_OK) {
            progressed |= collect(s);
            progressed |= admit(s);
        }
        const bool outstanding = !s->waiting.empty() || !s->running.empty();
        const auto now = std::chrono::steady_clock::now();
        if (outstanding) s->idle_since = now;
        if (s->failed != HAC_OK) {
            // A failed server completes nothing more.  The kernel still runs
            // every published entry to its end (waits abort or time out)
            // before it honours the stop.
            stop_kernel(s);
            if (s->quit) break;
        } else if (s->quit && !outstanding) {
            // On quit, what was admitted finishes first.
            stop_kernel(s);
            break;
        } else if (!outstanding && s->kern_running &&
                   now - s->idle_since > std::chrono::milliseconds(kIdleStopMs)) {
            stop_kernel(s);
        }
        if (!progressed) s->cv.wait_for(lk, std::chrono::microseconds(outstanding ? 20 : 2000));
    }
}

void free_server(hac_server *s) {
    (void)hipSetDevice(s->info.device);
    if (s->kern_done) (void)hipEventDestroy(s->kern_done);
    if (s->kern) (void)hipStreamDestroy(s->kern);
    if (s->recs) (void)hipHostFree(s->recs);
    if (s->stage) (void)hipHostFree(s->stage);
    if (s->arena) (void)hipFree(s->arena);
    if (s->dev) (void)hipFree(s->dev);
    if (s->jobwords) (void)hipFree(s->jobwords);
    if (s->hostmem) (void)hipHostFree(s->hostmem);
    if (s->pinned) (void)hipHostFree(s->pinned);
    delete s;
}

}  // namespace

extern "C" {

int hac_server_create(hac_ctx *ctx, size_t hbm_budget_bytes, int32_t max_jobs, int32_t max_n,
                      hac_server **out) {
    if (!ctx || !out) return HAC_EINVAL;
    *out = nullptr;
    if (max_jobs < 1 || max_jobs > kMaxJobs || max_n < 2 || max_n > HAC_MAX_N || hbm_budget_bytes == 0)
        return HAC_EINVAL;
    hac_server *s = new hac_server();
    hac::ctx_info(ctx, &s->info);
    s->budget = hbm_budget_bytes;
    s->max_n = max_n;
    if (hipSetDevice(s->info.device) != hipSuccess) {
        free_server(s);
        return HAC_EDEVICE;
    }
    // LDS per workgroup: enough for every job size up to max_n with its group,
    // with the lazy mirror's step table where that fits.
    size_t lds = 0;
    for (int n = 2; n <= max_n; ++n) {
        const int own = hac::own_rows(n, group_for(n, s->info.lds_max));
        const size_t with = hac::lds_bytes(n, own, true, true);
        lds = std::max(lds, s->info.lazy && with <= s->info.lds_max ? with : hac::lds_bytes(n, own, true));
    }
    if (lds > s->info.lds_max) {
        free_server(s);
        return HAC_EINVAL;
    }
    s->lds = lds;
    s->block = 1024;
    // One workgroup of 1024 threads fills a CU's registers.  Leave one CU
    // per XCD free so that copy kernels the runtime may use for host
    // transfers, and other work on the device, can run beside the kernel.
    const int reserve = std::max(kXcds, s->info.cus / 32);
    s->grid = std::max(1, hac::serve_occupancy(lds, s->block)) * std::max(1, s->info.cus - reserve);
    if (group_for(max_n, s->info.lds_max) > s->grid) {
        free_server(s);
        return HAC_EINVAL;
    }
    const int64_t tms = s->info.timeout_ms > 0 ? s->info.timeout_ms : kServeTimeoutMs;
    const uint64_t khz = (uint64_t)(s->info.wallclock_khz > 0 ? s->info.wallclock_khz : 100000);
    s->timeout = (uint64_t)tms * khz;
    s->idle_ticks = (uint64_t)(s->info.timeout_ms > 0 ? s->info.timeout_ms : kSelfStopMs) * khz;

    hipError_t e = hipMalloc(reinterpret_cast<void **>(&s->arena), hbm_budget_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        s->arena = nullptr;
        free_server(s);
        return HAC_ENOMEM;
    }
    s->alloc.reset(hbm_budget_bytes);
    s->dev_bytes = page_bytes(s);
    const size_t host_bytes = align_up(sizeof(hac::ServeHost), kAlign) +
                              align_up((size_t)kRingCap * sizeof(hac::ServeEntry), kAlign) +
                              align_up((size_t)max_jobs * 8, kAlign);
    const size_t pinned_bytes = page_bytes(s);
    // Records of admitted jobs: room for 4M records and at least four of the
    // largest jobs.  Staging for pageable inputs: up to 1 GiB (and at least
    // one largest job up to the budget).
    s->recs_bytes = std::max((size_t)64 << 20, (size_t)4 * max_n * sizeof(hac_merge));
    s->stage_bytes = std::min(hbm_budget_bytes, std::max((size_t)1 << 30, align_up((size_t)max_n * max_n * 4, kAlign)));
    // Per job slot: status, members done, and exchange slots for the largest
    // group any job can get; zero now, and left zero by every job.
    for (int n = 2; n <= max_n; ++n) s->max_group = std::max(s->max_group, group_for(n, s->info.lds_max));
    s->jobwords_stride =
        align_up(kAlign + (s->max_group > 1 ? (size_t)2 * (s->max_group + 1) * hac::kSlotStride * 8 : 0), 4096);
    bool ok = hipMalloc(reinterpret_cast<void **>(&s->dev), s->dev_bytes) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&s->jobwords), s->jobwords_stride * max_jobs) == hipSuccess &&
              hipMemset(s->jobwords, 0, s->jobwords_stride * max_jobs) == hipSuccess &&
              hipDeviceSynchronize() == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void **>(&s->hostmem), host_bytes,
                            hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void **>(&s->pinned), pinned_bytes, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void **>(&s->recs), s->recs_bytes,
                            hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void **>(&s->stage), s->stage_bytes,
                            hipHostMallocMapped) == hipSuccess &&
              hipStreamCreateWithFlags(&s->kern, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&s->kern_done, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_server(s);
        return HAC_EDEVICE;
    }
    std::memset(s->hostmem, 0, host_bytes);
    std::memset(s->pinned, 0, pinned_bytes);
    s->host = reinterpret_cast<hac::ServeHost *>(s->hostmem);
    s->ring = reinterpret_cast<hac::ServeEntry *>(s->hostmem + align_up(sizeof(hac::ServeHost), kAlign));
    s->done = reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(s->ring) +
                                                     align_up((size_t)kRingCap * sizeof(hac::ServeEntry), kAlign));
    void *hd = nullptr;
    if (hipHostGetDevicePointer(&hd, s->hostmem, 0) != hipSuccess || !hd) {
        (void)hipGetLastError();
        free_server(s);
        return HAC_EDEVICE;
    }
    const ptrdiff_t ring_at = reinterpret_cast<char *>(s->ring) - s->hostmem;
    const ptrdiff_t done_at = reinterpret_cast<char *>(s->done) - s->hostmem;
    s->host_dev = reinterpret_cast<hac::ServeHost *>(hd);
    s->ring_dev = reinterpret_cast<hac::ServeEntry *>(static_cast<char *>(hd) + ring_at);
    s->done_dev = reinterpret_cast<unsigned long long *>(static_cast<char *>(hd) + done_at);
    void *rd = nullptr, *sd = nullptr;
    if (hipHostGetDevicePointer(&rd, s->recs, 0) != hipSuccess || !rd ||
        hipHostGetDevicePointer(&sd, s->stage, 0) != hipSuccess || !sd) {
        (void)hipGetLastError();
        free_server(s);
        return HAC_EDEVICE;
    }
    s->recs_dev = rd;
    s->stage_dev = sd;
    s->recs_alloc.reset(s->recs_bytes);
    s->stage_alloc.reset(s->stage_bytes);
    s->ring_owner.assign(kRingCap, 0);
    s->jobs.resize(max_jobs);
    for (int k = max_jobs - 1; k >= 0; --k) s->free_ids.push_back((uint32_t)k);
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return HAC_OK;
}

int hac_submit(hac_server *s, const float *host_dist, int64_t ld, int32_t n, int32_t linkage, uint64_t *ticket) {
    if (!s) return HAC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    {
        char msg[192];
        if (hac::check_submit_args(host_dist, ld, n, linkage, ticket, s->max_n, msg, sizeof msg) != HAC_OK)
            return sfail(s, HAC_EINVAL, "%s", msg);
    }
    if (s->failed != HAC_OK) return s->failed;
    if (s->quit) return sfail(s, HAC_EINVAL, "server is shutting down");
    const int g = group_for(n, s->info.lds_max);
    if (hac::lds_bytes(n, hac::own_rows(n, g), true) > s->lds || g > s->grid)
        return sfail(s, HAC_EINVAL, "n=%d does not fit the server's workgroups", n);
    const JobLayout lay = job_layout(n);
    if (lay.bytes > s->budget)
        return sfail(s, HAC_ENOMEM, "job of n=%d needs %zu bytes, budget %zu", n, lay.bytes, s->budget);
    const float *src_dev = device_address(host_dist);
    if (!src_dev && lay.stage_bytes > s->stage_bytes)
        return sfail(s, HAC_ENOMEM, "pageable matrix of n=%d exceeds the %zu-byte staging area; pass page-locked memory",
                     n, s->stage_bytes);
    if (s->free_ids.empty()) return sfail(s, HAC_EBUSY, "%zu jobs held", s->jobs.size());
    const uint32_t id = s->free_ids.back();
    s->free_ids.pop_back();
    Job &J = s->jobs[id];
    J.seq = J.seq + 1 == 0 ? 1 : J.seq + 1;
    J.host = host_dist;
    J.src_dev = src_dev;
    J.staged = src_dev == nullptr;
    J.ld = ld;
    J.n = n;
    J.link = linkage;
    J.g = g;
    J.lazy = s->info.lazy && hac::lds_bytes(n, hac::own_rows(n, g), true, true) <= s->lds;
    J.lay = lay;
    J.rc = HAC_OK;
    J.result.clear();
    s->submitted++;
    *ticket = ((uint64_t)J.seq << 32) | id;
    if (n == 1) {
        J.state = JobState::kDone;
        s->completed++;
        return HAC_OK;
    }
    J.state = JobState::kWaiting;
    s->waiting.push_back(id);
    s->cv.notify_all();
    return HAC_OK;
}

int hac_poll(hac_server *s, uint64_t ticket, hac_merge *out, int32_t *done) {
    if (!s || !done) return HAC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *done = 0;
    const uint32_t id = (uint32_t)ticket, seq = (uint32_t)(ticket >> 32);
    if (id >= s->jobs.size() || s->jobs[id].seq != seq || s->jobs[id].state == JobState::kFree)
        return sfail(s, HAC_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Job &J = s->jobs[id];
    if (J.state != JobState::kDone) {
        if (s->failed != HAC_OK) return s->failed;
        return HAC_OK;
    }
    *done = 1;
    const int rc = J.rc;
    if (rc == HAC_OK && out && !J.result.empty())
        std::memcpy(out, J.result.data(), J.result.size() * sizeof(hac_merge));
    J.state = JobState::kFree;
    std::vector<hac_merge>().swap(J.result);
    J.host = nullptr;
    s->free_ids.push_back(id);
    return rc;
}

int hac_server_get_stats(hac_server *s, hac_server_stats *out) {
    if (!s || !out) return HAC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->waiting = (int64_t)s->waiting.size();
    out->running = (int64_t)s->running.size();
    out->bytes_in_use = (int64_t)s->in_use;
    out->peak_bytes = (int64_t)s->peak;
    out->kernel_launches = s->launches;
    out->workgroups = s->grid;
    out->block = s->block;
    return HAC_OK;
}

const char *hac_server_last_error(hac_server *s) {
    if (!s) return "no server";
    std::lock_guard<std::mutex> lk(s->mu);
    return s->err.c_str();
}

int hac_server_destroy(hac_server *s) {
    if (!s) return HAC_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->quit = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    free_server(s);
    return HAC_OK;
}

}  // extern "C"
