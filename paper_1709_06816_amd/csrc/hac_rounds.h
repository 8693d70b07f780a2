// Internal interface of the round engine (hac_rounds.hip): single and
// complete linkage by rounds of merges of reciprocal nearest neighbours.
// Not installed; the public interface is hac.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hac_engine.h"

namespace hac {

constexpr int kRoundsBlock = 1024;     // threads per workgroup of the round kernel
constexpr int kRoundsMaxPairs = 2048;  // pairs merged in one round at most

// Control block of a round-engine launch (device memory, zeroed before it).
struct RoundsCtl {
    uint32_t bar;             // grid barrier arrivals (monotonic)
    uint32_t abort;           // set by a workgroup that gives up
    uint32_t pairs;           // pairs claimed in the current round
    uint32_t resc;            // rows queued for a rescan in the current round
    uint32_t merges;          // at a hand-over: merges done (read as Resume::state[0])
    uint32_t round;           //   and rounds run (Resume::state[1])
    uint32_t pad[2];
};

// Device workspace of one round-engine run on an n-item instance with G
// workgroups; offsets in bytes from the workspace base (256-byte aligned).
struct RoundsLayout {
    size_t ctl, rk, cnt, size, role, resc, pairs, k1, rec, key, live, bytes;
};
RoundsLayout rounds_layout(int n, int G);

// Workgroups of the round kernel that fit on one CU.
int rounds_occupancy();

// Merge kernel of the round engine on G co-resident workgroups (cooperative
// launch).  Its records (claim order, with sort keys) stay in the workspace
// until launch_rank writes them in merge order to `out`.
// The matrix `D` must be the symmetric working matrix written by the set-up
// kernel (its status word `status` is read first: on kErrInput nothing runs).
// The round engine hands the rest of the merges over when rounds stop paying
// (kHandover in `status`, state in the workspace: rounds_resume) unless
// `flags` has kFlagNoHandover: a k_run launch with kFlagAfterRounds queued
// behind it then does them.
// `ws` is the workspace laid out by rounds_layout (its control block zeroed
// beforehand).  link is HAC_SINGLE or HAC_COMPLETE.
// Errors and statistics go to `ctl` (rescans, rescan_elems, update_elems,
// rounds; with kFlagProfile in `flags`, per-workgroup phase times: [0] first
// rescans, [1] grid barriers, [2] updates, [3] rescans, [4] pair detection).
hipError_t launch_rounds(float *D, int n, int link, uint32_t *status, Control *ctl, void *ws, int G,
                         uint64_t timeout_ticks, int flags, hipStream_t stream);

// Hand-over state inside a round-engine workspace (for launch_merge).
Resume rounds_resume(int n, int G, void *ws);

// Records of the workspace (round engine, then any kernel it handed over
// to) written to `out` in merge order.
// Nothing is written if the launch failed (status or ctl->error set).
hipError_t launch_rank(int n, hac_merge *out, const uint32_t *status, const Control *ctl, void *ws, int G,
                       hipStream_t stream);

// Record array of the workspace (the kernel queued behind the round engine
// writes its records there).
hac_merge *rounds_records(int n, int G, void *ws);

}  // namespace hac
