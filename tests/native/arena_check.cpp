// Randomised check of the serving arena's first-fit allocator against a
// byte-map model: no overlap, no block outside the range, every free byte in
// exactly one free block, neighbours always coalesced, first fit = the
// lowest-offset free block that is large enough.  Prints "ok" on success.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "hac_arena.h"

static int fail(const char *what, long a, long b) {
    std::printf("FAIL %s %ld %ld\n", what, a, b);
    return 1;
}

int main(int argc, char **argv) {
    const size_t size = 1 << 13;
    const int steps = argc > 1 ? std::atoi(argv[1]) : 200000;
    std::mt19937_64 rng(170906816);
    hac::Arena A;
    A.reset(size);
    std::vector<int> owner(size, -1);  // model: which live block holds each byte
    struct Blk { size_t off, bytes; };
    std::vector<Blk> live;
    for (int it = 0; it < steps; ++it) {
        if (live.empty() || rng() % 100 < 55) {
            const size_t want = 1 + rng() % (rng() % 8 == 0 ? 2048 : 96);
            // Model's first fit: lowest offset starting a free run >= want.
            long expect = -1;
            for (size_t p = 0, run = 0; p < size; ++p) {
                run = owner[p] < 0 ? run + 1 : 0;
                if (run == want) { expect = (long)(p + 1 - want); break; }
            }
            size_t off = 0;
            const bool ok = A.alloc(want, &off);
            if (ok != (expect >= 0)) return fail("alloc result", (long)ok, expect);
            if (!ok) continue;
            if ((long)off != expect) return fail("first fit", (long)off, expect);
            for (size_t p = off; p < off + want; ++p) {
                if (owner[p] >= 0) return fail("overlap", (long)p, owner[p]);
                owner[p] = (int)live.size();
            }
            live.push_back({off, want});
        } else {
            const size_t k = rng() % live.size();
            const Blk b = live[k];
            A.release(b.off, b.bytes);
            for (size_t p = b.off; p < b.off + b.bytes; ++p) owner[p] = -1;
            live[k] = live.back();
            live.pop_back();
            for (size_t q = 0; q < live.size(); ++q)
                for (size_t p = live[q].off; p < live[q].off + live[q].bytes; ++p) owner[p] = (int)q;
        }
        // Free blocks = maximal free runs of the model, exactly.
        size_t p = 0;
        auto it2 = A.free_blocks().begin();
        while (p < size) {
            if (owner[p] >= 0) { ++p; continue; }
            size_t q = p;
            while (q < size && owner[q] < 0) ++q;
            if (it2 == A.free_blocks().end()) return fail("missing free run", (long)p, (long)(q - p));
            if (it2->first != p || it2->second != q - p) return fail("free run", (long)it2->first, (long)p);
            ++it2;
            p = q;
        }
        if (it2 != A.free_blocks().end()) return fail("extra free block", (long)it2->first, (long)it2->second);
    }
    for (const Blk &b : live) A.release(b.off, b.bytes);
    if (A.free_blocks().size() != 1 || A.free_blocks().begin()->second != size)
        return fail("not whole after freeing all", (long)A.free_blocks().size(), 0);
    std::printf("ok\n");
    return 0;
}
