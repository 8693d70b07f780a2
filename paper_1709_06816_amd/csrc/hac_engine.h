// Internal interface between the C-ABI layer (hac_api.cpp) and the device
// engine (hac_engine.hip).  Not installed; the public interface is hac.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hac.h"

namespace hac {

constexpr int kRunBlock = 1024;      // default threads per workgroup of the single-instance kernel (256, 512 or 1024)
constexpr int kBatchBlock = 256;     // default threads per workgroup of the batch kernel (256 or 1024)
constexpr int kSetupBlock = 256;     // threads per workgroup of the set-up kernel
constexpr int kSetupStrip = 4;       // tiles per workgroup of the set-up kernel
constexpr int kChunk = 64;           // rows owned in chunks of 64 (one wave's lanes)
constexpr int kTile = 64;            // mirror tile edge
constexpr int kSlotStride = 512;     // u64 words between exchange slots (4 KiB)

// Device status words of one launch.
enum : uint32_t {
    kErrInput = 1u,     // non-finite or out-of-range input
    kErrTimeout = 2u,   // a wait exceeded the watchdog
    kErrInternal = 4u,  // no live pair found although >= 2 clusters remain
    kHandover = 8u,     // not an error: the round engine left the instance to the
                        // one-merge-per-step kernel queued behind it
};

// Phases timed by each workgroup (device wall clock).
enum : int { kPhSetup = 0, kPhWait = 1, kPhUpdate = 2, kPhRescan = 3, kPhCand = 4, kPhases = 5 };

// Exchange between the workgroups of a group (tuning only; results identical).
enum : int {
    kExchAllToAll = 0,  // every workgroup polls every slot
    kExchReducer = 1,   // workgroup 0 polls every slot and broadcasts the minimum
};

struct Control {
    uint32_t error;            // OR of kErr* over the launch
    uint32_t abort;            // set by a workgroup that gives up: every wait exits
    uint32_t next;             // batch work queue head
    uint32_t rounds;           // rounds of merges run by the round engine
    unsigned long long rescans;
    unsigned long long rescan_elems;
    unsigned long long update_elems;
    unsigned long long forced;        // extra argmin rounds forced by a row's lower bound (kFlagDefer)
    unsigned long long prof_sum[8];   // per phase, summed over workgroups (wall-clock ticks)
    unsigned long long prof_max[8];   // per phase, largest workgroup total
    // The round engine's own share of rescans / rescan_elems / update_elems
    // (a kernel that takes over from it adds to the fields above only).
    unsigned long long rounds_rescans;
    unsigned long long rounds_rescan_elems;
    unsigned long long rounds_update_elems;
};

// One clustering instance as the engine sees it.
struct Instance {
    float *D;            // working matrix, n x n, leading dimension n
    hac_merge *out;      // n-1 records (device)
    uint64_t *rowkey;    // n first row minima from the set-up kernel (single-instance path)
    uint64_t *slots;     // exchange slots: 2 * (g + 1) * kSlotStride words (g > 1)
    uint32_t *status;    // per-instance kErr* word
    int32_t n;
    int32_t link;
    int32_t exchange;    // kExch* (g > 1)
    int32_t flags;       // kFlag*
};

enum : int32_t {
    kFlagProfile = 1,  // time the phases of the merge loop (costs ~0.5 us per merge)
    kFlagScan = 2,     // no cached row minima: every merge rescans every live row (Section 5.3 step 1)
    kFlagDefer = 4,    // rows whose partner merged keep a lower bound and are rescanned while
                       // their workgroup waits in the next exchange (single instance, g > 1)
    kFlagAfterRounds = 8,  // k_run queued behind the round engine: runs only on kHandover
    kFlagNoHandover = 16,  // round engine: never hand over, rounds to the end (HAC_OPT_ROUNDS = 2)
    kFlagStall = 32,       // failure test: workgroup 0 never publishes, so the other
                           // workgroups' bounded waits expire (HAC_OPT_INJECT_STALL)
    kFlagLazy = 64,        // lazy mirror (batch and serving kernels): the update writes row i
                           // only, and a pair's current value is read from the one of its two
                           // rows written last (write steps in LDS); needs lds_bytes(.., true)
};

// State left by the round engine when it hands an instance over part-way
// (kHandover): the one-merge-per-step kernel queued behind it
// resumes from it and writes its records, with their sort keys, after the
// round engine's.  All pointers null: a run from the start.
struct Resume {
    const uint32_t *live;    // n-bit live mask
    const int32_t *size;     // cluster size of every live slot
    uint64_t *keys;          // sort key of every record: ord(h):32 | i:16 | round:16
    const uint32_t *state;   // [0] merges done, [1] rounds run
};

// Rows a workgroup owns when g workgroups share n items.
int own_rows(int n, int g);
// Bytes of dynamic LDS one workgroup needs to own `own` rows of an n-item
// instance; `in_kernel_setup` adds room for the mirror tile (batch kernel),
// `lazy` for the row write steps of kFlagLazy.
size_t lds_bytes(int n, int own, bool in_kernel_setup, bool lazy = false);

// Fill `words` u32 with zero on `stream` (a kernel, not a memset node).
hipError_t launch_zero(void *p, size_t words, hipStream_t stream);

// Set-up kernel alone (validation, -0, mirror, first upper row minima into
// inst.rowkey, which it fills beforehand); status bits go to inst.status.
hipError_t launch_setup(const Instance &inst, const float *src, hipStream_t stream);

// Single instance: set-up kernel over the whole device, then the merge kernel
// on g workgroups (g > 1 uses a cooperative launch so that all are
// co-resident).  The set-up reads the strict upper triangle from `src` and
// writes both triangles of inst.D (src == inst.D: in place).  `setup_done`
// is recorded on the stream between the two.
hipError_t launch_run(const Instance &inst, const float *src, int g, int block, Control *ctl,
                      uint64_t timeout_ticks, hipStream_t stream, hipEvent_t setup_done);
// The merge kernel alone, after launch_setup has run on inst (queued behind
// the round engine: kFlagAfterRounds in inst.flags, `rs` its hand-over
// state, inst.out its record array).
hipError_t launch_merge(const Instance &inst, int g, int block, Control *ctl, uint64_t timeout_ticks,
                        hipStream_t stream, const Resume &rs = Resume{});

// A batch launch: `count` instances in the order of `order` (device
// int32[count], largest first); the first `ngroups` of them run on fixed
// groups of workgroups (device int32 gbase/gsize[ngroups]), the rest one
// workgroup each from a queue.
struct BatchLaunch {
    const Instance *insts;
    const int32_t *order;
    int count;
    const int32_t *gbase;
    const int32_t *gsize;
    int ngroups;
    int block;   // 256 or 1024 threads per workgroup
    int upd;     // chunks per wave in each update batch: 8 at 256 threads, 2 or 4 at 1024
    int grid;    // workgroups (all co-resident)
    size_t lds;  // dynamic LDS per workgroup
};
hipError_t launch_batch(const BatchLaunch &b, Control *ctl, uint64_t timeout_ticks, hipStream_t stream);

// An executable graph of one batch call: copy `up_bytes` from pinned host
// memory `up_src` to `up_dst`, zero `z0_words` u32 at z0 and `z1_words` at z1
// with fill kernels (no memset nodes), then the batch kernel, marked
// cooperative when it has groups.  The graph reads the descriptors from
// `up_src` at every launch, so new descriptors of the same shape need no
// rebuild.
hipError_t build_batch_graph(const BatchLaunch &b, Control *ctl, uint64_t timeout_ticks, void *up_dst,
                             const void *up_src, size_t up_bytes, void *z0, size_t z0_words, void *z1,
                             size_t z1_words, hipGraphExec_t *exec);

// Serving: a persistent kernel runs jobs that the host publishes as entries
// of a ring in fine-grained host memory, one entry per workgroup of a job.
// Per job slot (index `job`), device memory holds the status word, the
// count of members done and the group's exchange slots; they are zero when
// a job starts and the last member to finish clears them again.
struct ServeEntry {
    Instance inst;        // inst.D: device matrix; inst.out: records (page-locked host memory);
                          // inst.status: the job slot's words; inst.slots: its exchange slots (g > 1)
    const float *src;     // the job's matrix in page-locked host memory (device address)
    int64_t ld;           // its leading dimension (elements)
    int32_t g;            // workgroups on the job
    int32_t rank;         // this entry's workgroup within the job
    uint32_t job;         // job slot: index of its completion word
    uint32_t seq;         // completion word once done: seq << 32 | status
};
static_assert(sizeof(ServeEntry) % 8 == 0, "entries are read as 64-bit words");

struct ServeHost {        // fine-grained (coherent) host memory
    unsigned long long tail;   // entries published (release store by the host)
    uint32_t stop;             // set by the host when nothing is outstanding
    uint32_t pad;
};

struct ServeDev {         // device memory, set by the host before each launch
    unsigned long long head;   // next entry to claim
    unsigned long long tail;   // device copy of ServeHost::tail
    uint32_t token;            // 1 while a workgroup polls host memory
    uint32_t stop;             // device copy of ServeHost::stop
    uint32_t exits;            // workgroups that have left the kernel
    uint32_t self_stops;       // idle stops raised by the kernel itself
    unsigned long long claims; // entries taken
};

struct ServeLaunch {
    ServeHost *host;
    const ServeEntry *ring;    // fine-grained host memory, `cap` entries
    uint32_t cap;
    unsigned long long *done;  // fine-grained host memory, one completion word per job slot
    ServeDev *dev;
    int block;                 // 256 or 1024
    int grid;                  // workgroups (all co-resident)
    size_t lds;
    uint64_t idle_ticks;       // a workgroup idle this long stops the kernel by itself
};
hipError_t launch_serve(const ServeLaunch &s, Control *ctl, uint64_t timeout_ticks, hipStream_t stream);
int serve_occupancy(size_t lds, int block);

// Scratch of the allocation-free entry point (hac_run_noalloc): a static
// device array holding the control block, the status word, the first row
// minima (n <= HAC_NOALLOC_MAX_N) and the exchange slots of up to
// HAC_NOALLOC_MAX_WORKGROUPS workgroups, laid out as hac_run lays out its
// workspace.
constexpr size_t kScratchCtlBytes = 256;      // Control, aligned
constexpr size_t kScratchStatusBytes = 256;   // one status word, aligned
constexpr size_t kNoAllocScratchBytes = kScratchCtlBytes + kScratchStatusBytes + (size_t)8 * HAC_NOALLOC_MAX_N +
                                        (size_t)2 * (HAC_NOALLOC_MAX_WORKGROUPS + 1) * kSlotStride * 8;
static_assert(kNoAllocScratchBytes == HAC_NOALLOC_SCRATCH_BYTES, "hac.h states the scratch size");
static_assert(sizeof(Control) <= kScratchCtlBytes, "control block fits its scratch slot");
// Device address of that array on the current device (hipGetSymbolAddress);
// each device holds its own copy at its own address.
hipError_t engine_scratch(void **ptr);

// Kernel attribute set-up (dynamic LDS limits); call once per device.
// `max_lds` is the device's LDS per workgroup; *usable receives the dynamic
// LDS a launch may request.
hipError_t engine_setup(size_t max_lds, size_t *usable);

// Workgroups of the run (batch = false; the variant `run_flags` (kFlag*)
// selects) or batch kernel with `block` threads that fit on one CU with `lds`
// bytes of dynamic LDS.
int engine_occupancy(size_t lds, int block, bool batch, int32_t run_flags = 0);

}  // namespace hac
