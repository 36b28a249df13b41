// Fuzz of the serving loop's ring allocator: allocations never overlap, stay in bounds, and an
// empty ring always accepts a request that fits the arena.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2603_17168_amd/csrc/cskv_ring.h"

int main() {
    std::mt19937_64 rng(7);
    long allocs = 0;
    for (int trial = 0; trial < 20000; ++trial) {
        cskv::Ring r;
        r.size = 1 + rng() % 256;
        std::deque<std::pair<size_t, size_t>> mine;
        for (int step = 0; step < 400; ++step) {
            if (!mine.empty() && rng() % 100 < 45) {
                r.free_front();
                mine.pop_front();
                continue;
            }
            const size_t b = (rng() % 5 == 0) ? 0 : rng() % (r.size + 1);
            size_t off = 0;
            const bool ok = r.alloc(b, &off);
            bool empty = true;
            for (auto& m : mine)
                if (m.second) empty = false;
            if (!ok) {
                if (empty) {
                    std::printf("FAIL: empty ring refused %zu of %zu\n", b, r.size);
                    return 1;
                }
                continue;
            }
            ++allocs;
            if (off + b > r.size) {
                std::printf("FAIL: out of bounds\n");
                return 1;
            }
            for (auto& m : mine) {
                if (b && m.second && !(off + b <= m.first || m.first + m.second <= off)) {
                    std::printf("FAIL: overlap [%zu,%zu) with [%zu,%zu)\n", off, off + b, m.first, m.first + m.second);
                    return 1;
                }
            }
            mine.push_back({off, b});
        }
    }
    std::printf("ok %ld allocations\n", allocs);
    return 0;
}
