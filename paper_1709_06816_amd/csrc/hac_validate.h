// Argument checks of the C-ABI entry points (include/hac.h), kept free of
// device code so that they can be built and exercised on the host alone
// (tests/native/validate_check.cpp runs them under ASan and UBSan).
// Each returns HAC_OK or HAC_EINVAL and, on error, writes a message to msg.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "hac.h"

namespace hac {

// hac_run / hac_run_noalloc: dist and out (out only for n > 1) non-null,
// 1 <= n <= max_n, linkage 0..HAC_CENTROID, no flag outside `allowed`.
int check_run_args(const void *dist, int32_t n, int32_t linkage, const void *out, uint32_t flags,
                   uint32_t allowed, int32_t max_n, char *msg, size_t len);

// hac_batch, count > 0: every pointer non-null, flags within
// HAC_PRESERVE_INPUT | HAC_OUT_DEVICE, every n_k in 1..HAC_MAX_BATCH_N,
// every linkage 0..HAC_CENTROID, offsets non-negative and small enough that
// offsets[k] + n_k^2 and out_offsets[k] + n_k - 1 do not overflow.  On
// success *extent = max_k offsets[k] + n_k^2 (elements) and *rec_extent =
// max_k out_offsets[k] + n_k - 1 (records).
int check_batch_args(const void *packed, const int64_t *offsets, const int32_t *ns, const int32_t *linkages,
                     int32_t count, const void *out, const int64_t *out_offsets, uint32_t flags, int64_t *extent,
                     int64_t *rec_extent, char *msg, size_t len);

// hac_submit: host_dist and ticket non-null, 1 <= n <= max_n, ld >= n,
// linkage 0..HAC_CENTROID.
int check_submit_args(const void *host_dist, int64_t ld, int32_t n, int32_t linkage, const void *ticket,
                      int32_t max_n, char *msg, size_t len);

// hac_rmsd: coords and dist non-null, 1 <= n <= HAC_MAX_N,
// 1 <= atoms <= max_atoms, flags == 0.
int check_rmsd_args(const void *coords, int32_t n, int32_t atoms, const void *dist, uint32_t flags,
                    int32_t max_atoms, char *msg, size_t len);

}  // namespace hac
