// hac_rmsd.h -- host side of the RMSD producer kernels (hac_rmsd.hip).
#ifndef HAC_RMSD_H
#define HAC_RMSD_H

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace hac {

// Largest accepted |coordinate|: keeps every product sum of the
// cross-covariances finite in fp32 for any atom count the API accepts, and
// every RMSD far below the clustering input limit 2^100.
constexpr double kRmsdMaxCoord = 1099511627776.0;  // 2^40
constexpr int kRmsdMaxAtoms = 1 << 20;

// Workspace of one call: centred coordinate planes, squared norms, status.
struct RmsdLayout {
    int npad = 0;            // conformations rounded up to a multiple of 64
    int quads = 0;           // groups of 4 atoms, a multiple of the chunk (padding atoms zero)
    size_t planes_bytes = 0;
    size_t sq_offset = 0;
    size_t status_offset = 0;
    size_t bytes = 0;        // whole workspace
    int64_t blocks = 0;      // workgroups: whole super-blocks on or above the diagonal
};

RmsdLayout rmsd_layout(int n, int atoms);

// Enqueue the producer on `stream`: xyz (device, n x atoms x 3 fp32, atom
// coordinates interleaved) -> out (device, n x n, leading dimension n; strict
// upper triangle and diagonal written).  The status word at
// ws + status_offset is nonzero when a coordinate was not finite or exceeded
// kRmsdMaxCoord, and then out is not written.
hipError_t launch_rmsd(const float *xyz, int n, int atoms, float *out, void *ws, hipStream_t stream);

}  // namespace hac

#endif  // HAC_RMSD_H
