// Drives the C-ABI argument checks (paper_1709_06816_amd/csrc/hac_validate.cpp)
// through valid and invalid arguments, for building under AddressSanitizer
// and UndefinedBehaviorSanitizer on the host.  Prints "ok" and exits 0 when
// every check answered as documented in hac_validate.h.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "hac_validate.h"

#define CHECK(cond, what)                                  \
    do {                                                   \
        if (!(cond)) {                                     \
            fprintf(stderr, "failed: %s (line %d)\n", what, __LINE__); \
            return 1;                                      \
        }                                                  \
    } while (0)

int main() {
    using namespace hac;
    char msg[192];
    float x = 0;
    hac_merge rec[1];
    const uint32_t run_flags = HAC_PRESERVE_INPUT | HAC_OUT_DEVICE | HAC_MODE_SCAN;
    CHECK(check_run_args(&x, 4, HAC_COMPLETE, rec, 0, run_flags, HAC_MAX_N, msg, sizeof msg) == HAC_OK, "run ok");
    CHECK(check_run_args(&x, 1, HAC_WARD, nullptr, 0, run_flags, HAC_MAX_N, msg, sizeof msg) == HAC_OK, "n=1 no out");
    CHECK(check_run_args(nullptr, 4, 0, rec, 0, run_flags, HAC_MAX_N, msg, sizeof msg) == HAC_EINVAL, "null dist");
    CHECK(strstr(msg, "dist") != nullptr, "message names dist");
    CHECK(check_run_args(&x, 0, 0, rec, 0, run_flags, HAC_MAX_N, msg, sizeof msg) == HAC_EINVAL, "n=0");
    CHECK(check_run_args(&x, HAC_MAX_N + 1, 0, rec, 0, run_flags, HAC_MAX_N, msg, sizeof msg) == HAC_EINVAL, "n big");
    CHECK(check_run_args(&x, INT32_MIN, 0, rec, 0, run_flags, HAC_MAX_N, msg, sizeof msg) == HAC_EINVAL, "n min");
    CHECK(check_run_args(&x, 4, -1, rec, 0, run_flags, HAC_MAX_N, msg, sizeof msg) == HAC_EINVAL, "linkage -1");
    CHECK(check_run_args(&x, 4, 6, rec, 0, run_flags, HAC_MAX_N, msg, sizeof msg) == HAC_EINVAL, "linkage 6");
    CHECK(check_run_args(&x, 4, 0, rec, 8u, run_flags, HAC_MAX_N, msg, sizeof msg) == HAC_EINVAL, "flag 8");
    CHECK(check_run_args(&x, 4, 0, rec, HAC_PRESERVE_INPUT, HAC_OUT_DEVICE, HAC_MAX_N, msg, sizeof msg) == HAC_EINVAL,
          "flag not allowed");
    CHECK(check_run_args(&x, 4, 0, nullptr, 0, run_flags, HAC_MAX_N, msg, sizeof msg) == HAC_EINVAL, "null out");
    CHECK(check_run_args(&x, 4, 0, rec, 0, run_flags, 3, msg, 0) == HAC_EINVAL, "no message room");

    // Batches.
    std::vector<int64_t> off = {0, 64, 4160};
    std::vector<int32_t> ns = {8, 64, 1};
    std::vector<int32_t> lk = {0, 3, 5};
    std::vector<int64_t> oo = {0, 7, 70};
    int64_t ext = -1, rext = -1;
    CHECK(check_batch_args(&x, off.data(), ns.data(), lk.data(), 3, rec, oo.data(), 0, &ext, &rext, msg, sizeof msg) ==
              HAC_OK, "batch ok");
    CHECK(ext == 4161 && rext == 70, "batch extents");
    CHECK(check_batch_args(&x, off.data(), ns.data(), lk.data(), -1, rec, oo.data(), 0, &ext, &rext, msg,
                           sizeof msg) == HAC_EINVAL, "count -1");
    CHECK(check_batch_args(&x, nullptr, ns.data(), lk.data(), 3, rec, oo.data(), 0, &ext, &rext, msg, sizeof msg) ==
              HAC_EINVAL, "null offsets");
    CHECK(check_batch_args(&x, off.data(), ns.data(), lk.data(), 3, rec, oo.data(), HAC_MODE_SCAN, &ext, &rext, msg,
                           sizeof msg) == HAC_EINVAL, "scan flag");
    ns[1] = HAC_MAX_BATCH_N + 1;
    CHECK(check_batch_args(&x, off.data(), ns.data(), lk.data(), 3, rec, oo.data(), 0, &ext, &rext, msg, sizeof msg) ==
              HAC_EINVAL, "batch n big");
    ns[1] = 64;
    lk[2] = 7;
    CHECK(check_batch_args(&x, off.data(), ns.data(), lk.data(), 3, rec, oo.data(), 0, &ext, &rext, msg, sizeof msg) ==
              HAC_EINVAL, "batch linkage");
    lk[2] = 5;
    off[0] = -1;
    CHECK(check_batch_args(&x, off.data(), ns.data(), lk.data(), 3, rec, oo.data(), 0, &ext, &rext, msg, sizeof msg) ==
              HAC_EINVAL, "negative offset");
    off[0] = INT64_MAX - 10;  // offsets[k] + n^2 would overflow
    CHECK(check_batch_args(&x, off.data(), ns.data(), lk.data(), 3, rec, oo.data(), 0, &ext, &rext, msg, sizeof msg) ==
              HAC_EINVAL, "offset overflow");
    off[0] = 0;
    oo[2] = INT64_MAX;
    CHECK(check_batch_args(&x, off.data(), ns.data(), lk.data(), 3, rec, oo.data(), 0, &ext, &rext, msg, sizeof msg) ==
              HAC_EINVAL, "record offset overflow");
    oo[2] = 70;

    // Served jobs.
    uint64_t ticket = 0;
    CHECK(check_submit_args(&x, 10, 10, 2, &ticket, 16384, msg, sizeof msg) == HAC_OK, "submit ok");
    CHECK(check_submit_args(&x, 9, 10, 2, &ticket, 16384, msg, sizeof msg) == HAC_EINVAL, "ld < n");
    CHECK(check_submit_args(&x, 10, 10, 2, nullptr, 16384, msg, sizeof msg) == HAC_EINVAL, "null ticket");
    CHECK(check_submit_args(&x, 20000, 20000, 2, &ticket, 16384, msg, sizeof msg) == HAC_EINVAL, "n > max_n");
    CHECK(check_submit_args(&x, 10, 10, 9, &ticket, 16384, msg, sizeof msg) == HAC_EINVAL, "submit linkage");

    // RMSD producer.
    CHECK(check_rmsd_args(&x, 5, 3, &x, 0, 1 << 20, msg, sizeof msg) == HAC_OK, "rmsd ok");
    CHECK(check_rmsd_args(&x, 5, 0, &x, 0, 1 << 20, msg, sizeof msg) == HAC_EINVAL, "rmsd atoms");
    CHECK(check_rmsd_args(&x, HAC_MAX_N + 1, 3, &x, 0, 1 << 20, msg, sizeof msg) == HAC_EINVAL, "rmsd n");
    CHECK(check_rmsd_args(&x, 5, 3, nullptr, 0, 1 << 20, msg, sizeof msg) == HAC_EINVAL, "rmsd dist");
    CHECK(check_rmsd_args(&x, 5, 3, &x, 1, 1 << 20, msg, sizeof msg) == HAC_EINVAL, "rmsd flags");
    printf("ok\n");
    return 0;
}
