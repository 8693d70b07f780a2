// Internal interface of the scan engine (hac_scan.hip): the paper's own
// closest-pair step, a scan of the whole live upper triangle before every
// merge (Section 5.3 step 1), over every CU.  Not installed; the public
// interface is hac.h (HAC_MODE_SCAN).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hac_engine.h"

namespace hac {

constexpr int kScanBlock = 1024;  // threads per workgroup

// Counters of one scan-engine launch (device memory, zeroed before it).
struct ScanCtl {
    uint32_t bar;      // grid barrier arrivals (monotonic)
    uint32_t abort;    // set by a workgroup that gives up
    uint32_t compactions;
    uint32_t pad;
};

// Device workspace of one run on n items with G workgroups (byte offsets).
struct ScanLayout {
    size_t ctl, cand, idx, bytes;
};
ScanLayout scan_layout(int n, int G);

// Floats the spare matrix needs: the working matrix is compacted into it
// with a leading dimension padded to a multiple of 4.
size_t scan_spare_floats(int n);

// Dynamic LDS of one workgroup, and how many workgroups fit on a CU.
size_t scan_lds_bytes(int n);
int scan_occupancy(int n);

// The merge kernel on G co-resident workgroups (cooperative launch).  D is
// the symmetric working matrix written by the set-up kernel (status read
// first: on kErrInput nothing runs); `spare` holds scan_spare_floats(n)
// floats; records go to `out` (device), statistics and errors to `ctl`
// (rescan_elems = live entries scanned, update_elems, rounds = compactions).
hipError_t launch_scan(float *D, float *spare, int n, int link, hac_merge *out, const uint32_t *status, Control *ctl,
                       void *ws, int G, uint64_t timeout_ticks, int flags, hipStream_t stream);

}  // namespace hac
