// What the serving layer needs to know about a context (internal).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "hac.h"

namespace hac {

struct CtxInfo {
    int device;
    int cus;
    int wallclock_khz;
    size_t lds_max;      // dynamic LDS a launch may request
    int64_t timeout_ms;  // 0 = default
    bool lazy;           // HAC_OPT_LAZY_MIRROR
};
void ctx_info(const hac_ctx *c, CtxInfo *out);

}  // namespace hac
