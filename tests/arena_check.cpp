// Randomised check of the host-side arena allocator against a byte map:
// blocks are aligned, never overlap, stay inside the range, and freeing
// everything coalesces back to one free block.  Exit status 0 on success.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "arena.hpp"

static int fail(const char *what, unsigned long long a, unsigned long long b)
{
    fprintf(stderr, "arena check failed: %s (%llu, %llu)\n", what, a, b);
    return 1;
}

int main()
{
    const size_t size = 1 << 20, align = 256;
    pyro::Arena ar(size, align);
    std::vector<int> owner(size, -1);  // byte -> block id
    struct Blk {
        size_t off, len;
    };
    std::vector<Blk> live;
    std::mt19937_64 rng(12345);
    int next = 0;
    for (int step = 0; step < 20000; ++step) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const size_t want = 1 + rng() % (size / 16);
            const size_t off = ar.alloc(want);
            if (off == pyro::Arena::kNone) {
                if (ar.largest_free() >= (want + align - 1) / align * align)
                    return fail("alloc refused although a block fits", want, ar.largest_free());
                continue;
            }
            const size_t len = (want + align - 1) / align * align;
            if (off % align) return fail("misaligned", off, align);
            if (off + len > size) return fail("out of range", off, len);
            for (size_t b = off; b < off + len; ++b)
                if (owner[b] != -1) return fail("overlap", off, b);
            for (size_t b = off; b < off + len; ++b) owner[b] = next;
            live.push_back({off, len});
            ++next;
        } else {
            const size_t k = rng() % live.size();
            const Blk blk = live[k];
            if (!ar.release(blk.off)) return fail("release of a live block refused", blk.off, blk.len);
            if (ar.release(blk.off)) return fail("double release accepted", blk.off, blk.len);
            for (size_t b = blk.off; b < blk.off + blk.len; ++b) owner[b] = -1;
            live[k] = live.back();
            live.pop_back();
        }
        size_t used = 0;
        for (auto &b : live) used += b.len;
        if (used != ar.used()) return fail("used bytes", used, ar.used());
    }
    for (auto &b : live)
        if (!ar.release(b.off)) return fail("final release", b.off, b.len);
    if (ar.used() != 0 || ar.free_blocks() != 1 || ar.largest_free() != size)
        return fail("not coalesced", ar.free_blocks(), ar.largest_free());
    printf("arena ok\n");
    return 0;
}
