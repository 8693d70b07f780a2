/*
 * hac.h -- Lance-Williams agglomerative clustering on one MI355X (gfx950).
 *
 * The library runs the n-1 merge iterations of the Lance-Williams algorithm
 * (Section 4, steps 1-4) over an n x n fp32 distance matrix held in device
 * memory: each iteration takes the closest pair of live clusters and updates
 * the merged cluster's row and column with the Table 1 coefficients.  All
 * iterations of one instance run inside one persistent kernel launch.
 *
 * Conventions shared by every entry point
 *   - Every function returns a hac_status: HAC_OK (0) or a negative error.
 *     No exception, abort() or exit() crosses this interface; the text of
 *     the last error of a context is available from hac_last_error().
 *   - Distance matrices are fp32, row-major, leading dimension n.  Only the
 *     strict upper triangle (a < b) is read as input (Section 5.2: a distance
 *     matrix needs only its upper half); diagonal and lower triangle are
 *     ignored on input and overwritten.  Values must be finite with
 *     |x| <= 2^100; -0 is treated as +0.  Otherwise HAC_EINPUT.
 *   - A merge record is (i, j, height, size): slots 0 <= i < j < n; the
 *     merged cluster keeps slot i and slot j is retired (Section 5.3, step 6),
 *     so slot i is always the smallest original member of its cluster.
 *     height is the distance of the pair at the merge, size the member count
 *     of the merged cluster.  Ties between equal distances go to the
 *     lexicographically smallest (i, j).
 *   - Arithmetic: fp32 storage; single/complete are min/max (exact);
 *     average, weighted average, centroid and Ward evaluate the Table 1
 *     formula in fp32 with coefficients computed as fp64 quotients rounded
 *     once to fp32 (1/2 for weighted average) and the fixed order
 *     ((a_i*D_ki) + (a_j*D_kj)) [+ (beta*D_ij)], no fused multiply-add; a
 *     zero result is stored as +0.
 *   - Centroid heights need not increase with the merge index, and are
 *     negative where the input is not a matrix of squared Euclidean
 *     distances.  They stay finite: the merged pair holds the minimum, so a
 *     negative minimum never grows in magnitude and one merge adds at most
 *     |D_ij|/4 to an entry, which bounds |D| by 2^100 * (1 + (n-1)/4).
 *   - n is limited to 1 <= n <= HAC_MAX_N.
 *   - Thread safety: one context per host thread.  Calls on one context are
 *     serialised by the caller.
 */
#ifndef HAC_H
#define HAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HAC_MAX_N 65536

typedef struct hac_ctx hac_ctx;

typedef enum {
    HAC_SINGLE = 0,   /* Table 1 row "Single Linkage":   min(D_ki, D_kj) */
    HAC_COMPLETE = 1, /* Table 1 row "Complete Linkage": max(D_ki, D_kj) */
    HAC_AVERAGE = 2,  /* Table 1 row "Group Average" */
    HAC_WARD = 3,     /* Table 1 row "Ward" */
    HAC_WEIGHTED = 4, /* Table 1 row "Weighted Average": (D_ki + D_kj) / 2 */
    HAC_CENTROID = 5  /* Table 1 row "Centroid" */
} hac_linkage;

typedef struct {
    int32_t i;      /* surviving slot */
    int32_t j;      /* retired slot, i < j */
    float height;   /* D_ij when merged */
    int32_t size;   /* members of the merged cluster */
} hac_merge;        /* 16 bytes */

typedef enum {
    HAC_OK = 0,
    HAC_EINVAL = -1,    /* bad argument: n out of range, NULL pointer, bad linkage or flag */
    HAC_EINPUT = -2,    /* non-finite or |x| > 2^100 value in a strict upper triangle */
    HAC_ENOMEM = -3,    /* device memory for the workspace could not be allocated */
    HAC_EDEVICE = -4,   /* a HIP call failed; see hac_last_error() */
    HAC_ENODEV = -5,    /* no usable gfx950 device */
    HAC_EBUSY = -6,     /* hac_submit: the server already holds max_jobs jobs */
    HAC_ETIMEDOUT = -7, /* the persistent kernel's watchdog fired */
    HAC_EINTERNAL = -8  /* an invariant of the algorithm was broken on the device */
} hac_status;

/* Flags for hac_run / hac_batch. */
#define HAC_PRESERVE_INPUT (1u << 0) /* work on a library-owned copy; dist is left unchanged */
#define HAC_OUT_DEVICE     (1u << 1) /* out is device memory; the call returns once the work is
                                        enqueued on the stream, and hac_sync() reports its status */
#define HAC_MODE_SCAN      (1u << 2) /* hac_run only: no cached row minima; before every merge each
                                        workgroup scans the live upper part of all its rows, the
                                        paper's own step (Section 5.3 step 1).  Same merge list,
                                        O(n^3) bytes instead of O(n^2): a reference for the
                                        memory-bound design the cache replaces */

/*
 * hac_create -- open a context on HIP device `device` (ordinal).
 *   out: receives the context (owned by the caller, released by hac_destroy).
 *   Errors: HAC_EINVAL (out NULL), HAC_ENODEV (no such device, or not
 *   gfx950), HAC_EDEVICE.
 */
int hac_create(int device, hac_ctx **out);

/* hac_destroy -- release the context and its device workspace.  NULL is a no-op. */
int hac_destroy(hac_ctx *ctx);

/*
 * hac_run -- cluster one instance (Section 4, steps 1-4, iterated n-1 times).
 *   dist:    device pointer, n*n fp32, row-major (caller-owned).  Used as the
 *            working matrix and overwritten unless HAC_PRESERVE_INPUT.
 *   n:       number of items, 1..HAC_MAX_N.  n == 1 yields no merges.
 *   linkage: a hac_linkage value.
 *   out:     n-1 records in merge order; host memory, or device memory with
 *            HAC_OUT_DEVICE (caller-owned either way).
 *   flags:   HAC_PRESERVE_INPUT | HAC_OUT_DEVICE | HAC_MODE_SCAN.
 *   stream:  hipStream_t to enqueue on; NULL = HIP's default (null) stream.
 *   Without HAC_OUT_DEVICE the call blocks until out is filled and returns
 *   the run's status; on HAC_EINPUT out is left untouched.
 */
int hac_run(hac_ctx *ctx, float *dist, int32_t n, int32_t linkage,
            hac_merge *out, uint32_t flags, void *stream);

/*
 * hac_run_noalloc -- hac_run for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same computation and the same merge list as hac_run on the
 * same input and options (it runs hac_run's kernels), but the call itself
 * allocates nothing: a run's device scratch (control block, status word,
 * first row minima, exchange slots; HAC_NOALLOC_SCRATCH_BYTES bytes) is a
 * static array of the library, one per device, whose address hac_create
 * looks up once; the page-locked host word it reads the status back through
 * is allocated by hac_create too.
 *   dist:    device pointer, n*n fp32, row-major (caller-owned); used as the
 *            working matrix and overwritten.  HAC_PRESERVE_INPUT is rejected
 *            (HAC_EINVAL): a copy would need n*n*4 bytes of workspace.
 *   n:       1..HAC_NOALLOC_MAX_N; a larger n returns HAC_EINVAL.
 *   linkage: a hac_linkage value.
 *   out:     device memory for n-1 records (caller-owned).
 *   flags:   0 or HAC_MODE_SCAN, optionally with HAC_OUT_DEVICE: then the
 *            call returns once the work is enqueued and hac_sync() reports the
 *            status; without it the call waits and returns the run's status.
 *   stream:  hipStream_t to enqueue on; NULL = HIP's default stream.
 *   The merge kernel runs on at most HAC_NOALLOC_MAX_WORKGROUPS workgroups
 *   (HAC_OPT_WORKGROUPS above that is clamped).  hac_get_stats reports the
 *   run like hac_run's.
 *   The scratch array is shared by every call on a device and keeps the
 *   last call's contents (each call clears what must start at zero), so
 *   calls that overlap on one GPU -- from two contexts, two host threads or
 *   two streams -- race: the caller serialises them.
 */
#define HAC_NOALLOC_MAX_N 65536
#define HAC_NOALLOC_MAX_WORKGROUPS 64
#define HAC_NOALLOC_SCRATCH_BYTES 1057280 /* 256 + 256 + 8 * 65536 + 2 * 65 * 4096 */
int hac_run_noalloc(hac_ctx *ctx, float *dist, int32_t n, int32_t linkage,
                    hac_merge *out, uint32_t flags, void *stream);

/*
 * hac_batch -- cluster `count` independent instances in one persistent launch.
 *   packed:      device pointer; instance k's n_k x n_k matrix starts at
 *                element offsets[k] (instances must not overlap).
 *   offsets:     host int64[count], element offsets into packed.
 *   ns:          host int32[count], sizes (each 1..HAC_MAX_BATCH_N).
 *   linkages:    host int32[count].
 *   out:         merge records; instance k's n_k-1 records start at record
 *                out_offsets[k] (host int64[count]).  Host memory, or device
 *                memory with HAC_OUT_DEVICE.
 *   Each instance's records are byte-identical to hac_run on that instance.
 */
#define HAC_MAX_BATCH_N 8192
int hac_batch(hac_ctx *ctx, float *packed, const int64_t *offsets, const int32_t *ns,
              const int32_t *linkages, int32_t count, hac_merge *out,
              const int64_t *out_offsets, uint32_t flags, void *stream);

/*
 * hac_rmsd -- the input producer: the matrix of RMSDs between n conformations
 * of one chain (the paper clusters protein conformations by such a matrix,
 * computed by a parallel RMSD step: Section 2.1's protein example, Section
 * 5.1).  RMSD(A, B) is the root mean square deviation of corresponding atoms
 * after the best superposition of A onto B by a proper rotation and a
 * translation.
 *   coords: device pointer, n x atoms x 3 fp32 (conformation-major, then
 *           atom, then x, y, z), caller-owned, read only.  Every coordinate
 *           must be finite with |x| <= 2^40, otherwise HAC_EINPUT and dist
 *           is not written.
 *   n:      conformations, 1..HAC_MAX_N.  atoms: 1..2^20.
 *   dist:   device pointer, n x n fp32, row-major, leading dimension n,
 *           caller-owned.  The strict upper triangle receives RMSD(a, b)
 *           for a < b and the diagonal 0; the lower triangle is not written
 *           (hac_run reads only the strict upper triangle, so dist can be
 *           passed to it directly).
 *   flags:  0.
 *   stream: hipStream_t to enqueue on; NULL = HIP's default stream.  The
 *           call returns when the matrix is complete.
 *   Arithmetic: centroids and squared norms in fp64; centred coordinates
 *   rounded to fp32; the nine cross-covariance sums in fp32 on the matrix
 *   cores; the largest eigenvalue of the 4 x 4 quaternion key matrix and the
 *   RMSD in fp64, rounded once to fp32.  The device workspace (12 bytes per
 *   atom and conformation) is kept by the context and grown on demand.
 *   Errors: HAC_EINVAL (NULL pointer, n or atoms out of range, flags != 0),
 *   HAC_EINPUT (a coordinate rejected; dist untouched), HAC_ENOMEM (the
 *   workspace could not be allocated), HAC_EDEVICE (a HIP call failed).
 */
int hac_rmsd(hac_ctx *ctx, const float *coords, int32_t n, int32_t atoms, float *dist, uint32_t flags,
             void *stream);

/* hac_sync -- wait for the context's last HAC_OUT_DEVICE call and return its status. */
int hac_sync(hac_ctx *ctx);

/* hac_last_error -- text of the context's last error ("" if none).  Valid until the next call. */
const char *hac_last_error(const hac_ctx *ctx);

/*
 * Tuning options (hac_set_option).  Results never depend on them; they only
 * change how work is spread over the GPU.
 *   HAC_OPT_WORKGROUPS   workgroups cooperating on one hac_run instance
 *                        (0 = automatic; clamped to what can be co-resident)
 *   HAC_OPT_SINGLE_WG_N  hac_run uses one workgroup when n <= this (0 = automatic)
 *   HAC_OPT_TIMEOUT_MS   watchdog for one wait inside the persistent kernel
 *                        (0 = default 10000 ms); expiry returns HAC_ETIMEDOUT
 *   HAC_OPT_EXCHANGE     how the workgroups of one instance agree on each merge:
 *                        0 = every workgroup reads every partial result,
 *                        1 = workgroup 0 reads them and broadcasts the minimum
 *   HAC_OPT_PROFILE      1 = time the phases of the merge loop on the device
 *                        (reported in hac_stats.phase_*; adds ~0.5 us per merge)
 *   HAC_OPT_BLOCK        threads per workgroup of hac_run: 256, 512 or 1024
 *                        (0 = automatic)
 *   HAC_OPT_AUTOTUNE     hac_batch picks its launch plan by timing candidates on
 *                        a scratch copy of the first batch of each size mix, and
 *                        caches the choice in the context (1 = on, the default;
 *                        0 = off): threads per workgroup (256 or 1024, each with
 *                        its own rescan tile size), then workgroups per large
 *                        instance (1, 2, 4, 8) and the share of the co-resident
 *                        workgroups the groups may take (a quarter, half, three
 *                        quarters: how many of the largest instances get a
 *                        group), then at 1024 threads the update tile (2 or 4
 *                        column chunks per wave loaded at once).  A candidate
 *                        whose run reports an error is never chosen.  Costs
 *                        twelve extra runs of that first batch; see
 *                        hac_stats.plan_source.
 *   HAC_OPT_BATCH_BLOCK  force hac_batch's threads per workgroup: 256 or 1024
 *   HAC_OPT_BATCH_GROUP  force hac_batch's workgroups per large instance (1..64)
 *   HAC_OPT_BATCH_UPDATE force hac_batch's update tile at 1024 threads: 2 or 4
 *                        column chunks per wave (0 = 4 when not tuned; 256
 *                        threads always use 8)
 *   HAC_OPT_GRAPH        hac_batch enqueues its descriptor upload, fills and
 *                        kernel as one HIP graph, instantiated once per layout
 *                        (instance count, plan, workspace) and relaunched with
 *                        the new descriptors (1 = on, the default; 0 = plain
 *                        stream launches).  Results are identical either way.
 *   HAC_OPT_DEFER        hac_run: a row whose cached partner merged keeps its
 *                        old minimum as a lower bound instead of being
 *                        rescanned at once; only when such a bound wins an
 *                        argmin do the workgroups rescan all their stale rows
 *                        and repeat that argmin, so the merge list is the same
 *                        either way (Section 4 step 1).  0 = never, 1 = on
 *                        groups of two or more workgroups (the default; a
 *                        workgroup alone does better rescanning at once),
 *                        2 = also on one workgroup.
 *   HAC_OPT_ROUNDS       hac_run, single and complete linkage: merge in rounds
 *                        instead of one pair per step.  Each round merges every
 *                        pair of clusters that are each other's nearest
 *                        neighbour under the key order (D, i, j) (single
 *                        linkage: the globally closest pair, plus those whose
 *                        distance is the only minimum of both rows), applies
 *                        all their updates at once and rescans the rows that
 *                        need it; the records come out in the order of Section
 *                        4's loop, byte-identical to it.  0 = never, 1 = for
 *                        n >= 1024 (the default; the remaining merges go to the
 *                        one-merge-per-step kernel once rounds merge few pairs
 *                        each: near the end of a run, and early for single
 *                        linkage on input with many equal values), 2 = always,
 *                        rounds to the end.  Not
 *                        used by hac_run_noalloc, HAC_MODE_SCAN or other
 *                        linkages.
 *   HAC_OPT_INJECT_STALL failure test: 1 = in every following hac_run that runs
 *                        on several workgroups, workgroup 0 never publishes its
 *                        first exchange, so the other workgroups' bounded waits
 *                        expire after HAC_OPT_TIMEOUT_MS, every workgroup leaves
 *                        the kernel and the call returns HAC_ETIMEDOUT (out
 *                        unspecified).  0 (the default) = off.
 *   HAC_OPT_LAZY_MIRROR  hac_batch, and servers created afterwards: 1 (the
 *                        default) = the Lance-Williams update writes only the
 *                        survivor's row, not the mirrored column, and each
 *                        workgroup remembers the merge step that last wrote
 *                        every row, so that a pair's current distance is read
 *                        from whichever of its two rows was written later
 *                        (instances whose step table does not fit the LDS
 *                        write both halves); 0 = always write both halves.
 *                        Results are identical either way; the working
 *                        matrix's contents afterwards are unspecified.
 */
typedef enum {
    HAC_OPT_WORKGROUPS = 1,
    HAC_OPT_SINGLE_WG_N = 2,
    HAC_OPT_TIMEOUT_MS = 3,
    HAC_OPT_EXCHANGE = 4,
    HAC_OPT_PROFILE = 5,
    HAC_OPT_BLOCK = 6,
    HAC_OPT_AUTOTUNE = 7,
    HAC_OPT_BATCH_BLOCK = 8,
    HAC_OPT_BATCH_GROUP = 9,
    HAC_OPT_GRAPH = 10,
    HAC_OPT_DEFER = 11,
    HAC_OPT_ROUNDS = 12,
    HAC_OPT_INJECT_STALL = 13,
    HAC_OPT_LAZY_MIRROR = 14,
    HAC_OPT_BATCH_UPDATE = 15
} hac_option;
int hac_set_option(hac_ctx *ctx, int32_t option, int64_t value);

/*
 * hac_stats -- figures of the context's last completed hac_run / hac_batch.
 *   kernel_ms:         device time of the merge kernel (HIP events on the run's stream)
 *   init_ms:           device time of the set-up kernels before it
 *   rescans:           rows whose cached minimum was recomputed
 *   rescan_elems:      matrix entries read by those recomputations
 *   update_elems:      (k) entries updated by the Lance-Williams step, summed over merges
 *   workgroups:        workgroups the merge kernel ran with
 *   block:             threads per workgroup
 *   phase_avg_ms[5]:   time per workgroup (device wall clock), averaged over the
 *                      workgroups, spent in: [0] set-up (mirror, checks, first
 *                      row minima), [1] waiting for / combining the group's
 *                      partial minima, [2] the Lance-Williams update, [3] row
 *                      rescans, [4] local candidate reduction
 *   phase_max_ms[5]:   the same, largest workgroup
 *   group:             hac_run: workgroups on the instance (= workgroups);
 *                      hac_batch: workgroups per large instance in the plan used
 *   graph:             hac_batch: 0 = stream launches, 1 = an existing graph was
 *                      relaunched, 2 = a graph was built for this call; with a
 *                      graph kernel_ms covers upload, fills and kernel
 *   forced_rounds:     with deferred rescans: extra argmin rounds taken because
 *                      a row's lower bound won (see HAC_OPT_DEFER); hac_batch:
 *                      summed over its instances
 *   deferred:          1 if the last call deferred its rescans (hac_batch
 *                      always does)
 *   rounds:            hac_run through rounds of merges (HAC_OPT_ROUNDS): rounds
 *                      run (0 otherwise)
 *   handed_over:       1 if those rounds stopped part-way (few merges per round:
 *                      the last ones of a run, or single linkage on input with
 *                      many equal values) and the one-merge-per-step kernel made
 *                      the remaining merges
 *   compactions:       HAC_MODE_SCAN: times the live rows and columns were
 *                      copied into a smaller matrix
 *   rounds_ms:         hac_run through rounds of merges: device time of the
 *                      round engine's kernel alone (kernel_ms also covers the
 *                      kernel that takes over from it and the record sort);
 *                      0 otherwise
 *   rounds_rescan_elems, rounds_update_elems: that kernel's share of
 *                      rescan_elems and update_elems
 *   plan_source:       hac_batch: 0 = default plan or one forced by
 *                      HAC_OPT_BATCH_BLOCK / HAC_OPT_BATCH_GROUP, 1 = tuned
 *                      during this call, 2 = the plan tuned earlier for the
 *                      same size mix (cached in the context)
 *   plan_share:        hac_batch with groups: quarters of the co-resident
 *                      workgroups the groups were allowed to take (0 otherwise)
 *   plan_update:       hac_batch: column chunks per wave in each update batch
 *                      (8 at 256 threads; 2 or 4 at 1024)
 */
typedef struct {
    double kernel_ms;
    double init_ms;
    int64_t rescans;
    int64_t rescan_elems;
    int64_t update_elems;
    int32_t workgroups;
    int32_t block;
    double phase_avg_ms[5];
    double phase_max_ms[5];
    int32_t group;
    int32_t graph;
    int64_t forced_rounds;
    int32_t deferred;
    int32_t rounds;
    int32_t handed_over;
    int32_t compactions;
    double rounds_ms;
    int64_t rounds_rescan_elems;
    int64_t rounds_update_elems;
    int32_t plan_source;
    int32_t plan_share;
    int32_t plan_update;
} hac_stats;
int hac_get_stats(const hac_ctx *ctx, hac_stats *out);

/*
 * Serving with continuous batching.  Not a paper algorithm: many independent
 * clustering jobs (each the computation described above) share one GPU.
 *
 * A server owns an HBM arena of hbm_budget_bytes and a persistent kernel on
 * its own stream.  Jobs are admitted in arrival order as soon as the arena
 * holds their matrix and workspace, and are then published to the running
 * kernel, whose workgroups take jobs as they free up, so jobs that arrive
 * while others run overlap with them on the device.  The kernel reads each
 * job's matrix straight from host memory over the bus: page-locked memory in
 * place, pageable memory from a page-locked staging copy that the server's
 * host thread makes at admission.  Merge records come back the same way, into
 * page-locked memory of the server.  Jobs with n above 2048 run on a group of
 * workgroups.  A job's merge list is byte-identical to hac_run on the same
 * matrix, whatever else runs beside it.  A host thread of the server drives
 * admission, publication and completion; the kernel stops after a short
 * idle period and is relaunched on demand.
 *
 * hac_server_create -- ctx: a context (its device and HAC_OPT_TIMEOUT_MS are
 *   read at creation; the server keeps no reference; the timeout bounds the
 *   kernel's waits, default 120 s, and how long the kernel waits idle for a
 *   stop from the host before it stops by itself, default 60 s);
 *   hbm_budget_bytes: arena size
 *   (allocated at once); max_jobs: jobs held at a time, 1..4096 (submitted
 *   and not yet returned by hac_poll); max_n: largest n a job may have
 *   (2..HAC_MAX_N), which fixes the kernel's LDS per workgroup.
 *   Errors: HAC_EINVAL, HAC_ENOMEM (arena), HAC_EDEVICE.
 * hac_submit -- queue one job.  host_dist: host fp32 matrix, row-major with
 *   leading dimension ld >= n (elements); the top-left n x n block is the
 *   job's matrix, read under the same conventions as hac_run.  The server
 *   reads host_dist until the job is complete: keep it valid and unchanged
 *   until hac_poll reports done (page-locked memory gives the full copy
 *   rate).  *ticket identifies the job.  Returns HAC_EBUSY if max_jobs jobs
 *   are held, HAC_ENOMEM if the job alone exceeds the budget, HAC_EINVAL for
 *   bad arguments, or the server's error if it has failed.
 * hac_poll -- *done = 1 and the job's n-1 records in out (host memory) once
 *   it is complete; the ticket is then released and its status returned
 *   (HAC_OK, HAC_EINPUT, HAC_ETIMEDOUT, ...).  *done = 0 while it runs.
 *   out may be NULL to discard the records.  Unknown ticket: HAC_EINVAL.
 * hac_server_destroy -- wait for admitted jobs to finish, stop the kernel,
 *   free everything.  Held tickets become invalid.
 * hac_server_get_stats -- counters of the server (see hac_server_stats).
 * hac_server_last_error -- text of the server's last error; valid until the
 *   next call on the server.
 * Calls on one server may come from any host threads.
 */
typedef struct hac_server hac_server;
typedef struct {
    int64_t submitted;
    int64_t completed;
    int64_t waiting;          /* queued, not yet admitted */
    int64_t running;          /* admitted (copying or on the device), not complete */
    int64_t bytes_in_use;     /* arena bytes held by admitted jobs */
    int64_t peak_bytes;       /* largest bytes_in_use so far */
    int64_t kernel_launches;  /* launches of the persistent kernel */
    int32_t workgroups;       /* workgroups of that kernel */
    int32_t block;            /* threads per workgroup */
} hac_server_stats;
int hac_server_create(hac_ctx *ctx, size_t hbm_budget_bytes, int32_t max_jobs, int32_t max_n, hac_server **out);
int hac_submit(hac_server *srv, const float *host_dist, int64_t ld, int32_t n, int32_t linkage, uint64_t *ticket);
int hac_poll(hac_server *srv, uint64_t ticket, hac_merge *out, int32_t *done);
int hac_server_get_stats(hac_server *srv, hac_server_stats *out);
const char *hac_server_last_error(hac_server *srv);
int hac_server_destroy(hac_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* HAC_H */
