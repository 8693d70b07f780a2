// Argument checks of the C-ABI entry points (see hac_validate.h).
#include "hac_validate.h"

#include <stdarg.h>
#include <stdio.h>

namespace hac {
namespace {

int bad(char *msg, size_t len, const char *fmt, ...) {
    if (msg && len) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(msg, len, fmt, ap);
        va_end(ap);
    }
    return HAC_EINVAL;
}

bool linkage_ok(int32_t l) { return l >= HAC_SINGLE && l <= HAC_CENTROID; }

}  // namespace

int check_run_args(const void *dist, int32_t n, int32_t linkage, const void *out, uint32_t flags,
                   uint32_t allowed, int32_t max_n, char *msg, size_t len) {
    if (!dist) return bad(msg, len, "dist is NULL");
    if (n < 1 || n > max_n) return bad(msg, len, "n=%d outside 1..%d", n, max_n);
    if (!linkage_ok(linkage)) return bad(msg, len, "linkage %d is not 0..%d", linkage, (int)HAC_CENTROID);
    if (flags & ~allowed) return bad(msg, len, "unknown flags 0x%x", flags);
    if (n > 1 && !out) return bad(msg, len, "out is NULL");
    return HAC_OK;
}

int check_batch_args(const void *packed, const int64_t *offsets, const int32_t *ns, const int32_t *linkages,
                     int32_t count, const void *out, const int64_t *out_offsets, uint32_t flags, int64_t *extent,
                     int64_t *rec_extent, char *msg, size_t len) {
    if (count < 0) return bad(msg, len, "count=%d", count);
    if (!packed || !offsets || !ns || !linkages || !out || !out_offsets) return bad(msg, len, "NULL argument");
    if (flags & ~(HAC_PRESERVE_INPUT | HAC_OUT_DEVICE)) return bad(msg, len, "unknown flags 0x%x", flags);
    int64_t ext = 0, rext = 0;
    for (int32_t k = 0; k < count; ++k) {
        const int32_t n = ns[k];
        if (n < 1 || n > HAC_MAX_BATCH_N) return bad(msg, len, "instance %d: n=%d outside 1..%d", k, n, HAC_MAX_BATCH_N);
        if (!linkage_ok(linkages[k])) return bad(msg, len, "instance %d: linkage %d", k, linkages[k]);
        if (offsets[k] < 0 || out_offsets[k] < 0) return bad(msg, len, "instance %d: negative offset", k);
        const int64_t cells = (int64_t)n * n;
        if (offsets[k] > INT64_MAX - cells || out_offsets[k] > INT64_MAX - n)
            return bad(msg, len, "instance %d: offset too large", k);
        if (offsets[k] + cells > ext) ext = offsets[k] + cells;
        if (out_offsets[k] + n - 1 > rext) rext = out_offsets[k] + n - 1;
    }
    *extent = ext;
    *rec_extent = rext;
    return HAC_OK;
}

int check_submit_args(const void *host_dist, int64_t ld, int32_t n, int32_t linkage, const void *ticket,
                      int32_t max_n, char *msg, size_t len) {
    if (!host_dist || !ticket) return bad(msg, len, "NULL argument");
    if (n < 1 || n > max_n) return bad(msg, len, "n=%d outside 1..%d", n, max_n);
    if (ld < n) return bad(msg, len, "ld=%lld < n=%d", (long long)ld, n);
    if (!linkage_ok(linkage)) return bad(msg, len, "linkage %d", linkage);
    return HAC_OK;
}

int check_rmsd_args(const void *coords, int32_t n, int32_t atoms, const void *dist, uint32_t flags,
                    int32_t max_atoms, char *msg, size_t len) {
    if (!coords || !dist) return bad(msg, len, "coords or dist is NULL");
    if (n < 1 || n > HAC_MAX_N) return bad(msg, len, "n=%d outside 1..%d", n, HAC_MAX_N);
    if (atoms < 1 || atoms > max_atoms) return bad(msg, len, "atoms=%d outside 1..%d", atoms, max_atoms);
    if (flags != 0) return bad(msg, len, "unknown flags 0x%x", flags);
    return HAC_OK;
}

}  // namespace hac
