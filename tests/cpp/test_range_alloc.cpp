// Host-only test of the serving loop's range allocator (compiled with g++ by
// tests/test_host_logic.py).  Random alloc/release sequences are checked against a
// brute-force occupancy map.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "range_alloc.h"

static int fail(const char* what, long a, long b) {
    std::printf("FAIL %s %ld %ld\n", what, a, b);
    return 1;
}

int main() {
    const size_t cap = 1 << 20, align = 256;
    qc::RangeAllocator ra(cap, align);
    std::vector<char> used(cap / align, 0);
    struct Block { size_t off, bytes; };
    std::vector<Block> live;
    std::mt19937 rng(1707);
    for (int step = 0; step < 20000; ++step) {
        if (live.empty() || rng() % 3 != 0) {
            size_t bytes = 1 + rng() % 40000;
            size_t off = 0;
            const size_t need = (bytes + align - 1) / align;
            // does any run of `need` free units exist? (first fit must find the first one)
            long first = -1;
            for (size_t i = 0, run = 0; i < used.size(); ++i) {
                run = used[i] ? 0 : run + 1;
                if (run == need) { first = static_cast<long>(i + 1 - need); break; }
            }
            bool ok = ra.alloc(bytes, &off);
            if (ok != (first >= 0)) return fail("fit", ok, first);
            if (!ok) continue;
            if (static_cast<long>(off / align) != first) return fail("first-fit", off / align, first);
            for (size_t i = 0; i < need; ++i) {
                if (used[off / align + i]) return fail("overlap", off, i);
                used[off / align + i] = 1;
            }
            live.push_back({off, bytes});
        } else {
            size_t k = rng() % live.size();
            Block b = live[k];
            live.erase(live.begin() + static_cast<long>(k));
            ra.release(b.off, b.bytes);
            for (size_t i = 0; i < (b.bytes + align - 1) / align; ++i) used[b.off / align + i] = 0;
        }
        size_t in_use = 0;
        for (char c : used) in_use += c;
        if (ra.used() != in_use * align) return fail("used", ra.used(), in_use * align);
    }
    for (const Block& b : live) ra.release(b.off, b.bytes);
    if (ra.used() != 0 || ra.free_ranges() != 1 || ra.largest_free() != cap)
        return fail("coalesce", ra.free_ranges(), ra.largest_free());
    std::printf("OK\n");
    return 0;
}
