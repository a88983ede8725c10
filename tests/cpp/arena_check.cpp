// Randomised check of the serving arena's allocator against a byte map:
// blocks never overlap, stay inside the arena, are 256-byte aligned, the used
// count matches, and releasing everything leaves one free range.
#include <cstdio>
#include <random>
#include <vector>

#include "arena.hpp"

int main() {
    const size_t cap = 1 << 20;
    gf2x::Arena A(cap);
    std::vector<unsigned char> owner(cap, 0);
    struct Blk { size_t off, bytes; };
    std::vector<Blk> live;
    std::mt19937_64 rng(12345);
    size_t used = 0;
    for (int it = 0; it < 200000; ++it) {
        bool do_alloc = live.empty() || rng() % 100 < 55;
        if (do_alloc) {
            size_t bytes = 1 + rng() % (rng() % 4 ? 4096 : 65536);
            size_t off = A.alloc(bytes);
            size_t len = gf2x::Arena::round(bytes);
            if (off == gf2x::Arena::npos) {
                if (A.largest_free() >= len) { std::printf("alloc failed with room\n"); return 1; }
                continue;
            }
            if (off % 256 || off + len > cap) { std::printf("bad block\n"); return 1; }
            for (size_t i = off; i < off + len; ++i) {
                if (owner[i]) { std::printf("overlap\n"); return 1; }
                owner[i] = 1;
            }
            live.push_back({off, bytes});
            used += len;
        } else {
            size_t k = rng() % live.size();
            Blk b = live[k];
            live[k] = live.back();
            live.pop_back();
            size_t len = gf2x::Arena::round(b.bytes);
            for (size_t i = b.off; i < b.off + len; ++i) owner[i] = 0;
            A.release(b.off, b.bytes);
            used -= len;
        }
        if (A.used() != used) { std::printf("used mismatch\n"); return 1; }
    }
    for (const Blk& b : live) A.release(b.off, b.bytes);
    if (A.used() != 0 || A.free_ranges() != 1 || A.largest_free() != cap) { std::printf("no coalesce\n"); return 1; }
    std::printf("arena ok\n");
    return 0;
}
