// Host-logic test of the gap-free output fix-up (holes.h): simulates
// wavefronts that reserve output positions in blocks, emit uniquely numbered
// items, and leave holes; after applying the planned moves, [0, count) must
// hold every emitted item exactly once.
#include <cstdio>
#include <random>
#include <vector>

#include "holes.h"

int main() {
    std::mt19937_64 rng(12345);
    int failures = 0;
    for (int trial = 0; trial < 3000; trial++) {
        const uint64_t R = 1 + rng() % 64;
        const int waves = 1 + rng() % 40;
        struct W { uint64_t rb = 0, re = 0; };
        std::vector<W> w(waves);
        std::vector<int64_t> out(1 << 16, -1);
        uint64_t cursor = 0, count = 0;
        const int steps = rng() % 400;
        for (int st = 0; st < steps; st++) {
            W &x = w[rng() % waves];
            uint64_t k = rng() % (R + 1);
            for (uint64_t i = 0; i < k; i++) {
                if (x.re == x.rb) { x.rb = cursor; cursor += R; x.re = cursor; }
                out[x.rb++] = (int64_t)count++;
            }
        }
        std::vector<Hole> holes;
        for (auto &x : w) if (x.re > x.rb) holes.push_back(Hole{x.rb, x.re - x.rb});
        std::shuffle(holes.begin(), holes.end(), rng);
        auto mv = plan_hole_moves(holes, count, cursor);
        for (auto &m : mv) {
            for (uint64_t i = 0; i < m.len; i++) {
                if (m.dst + i >= count || m.src + i < count) { failures++; break; }
                out[m.dst + i] = out[m.src + i];
            }
        }
        std::vector<int> seen(count, 0);
        for (uint64_t i = 0; i < count; i++) {
            if (out[i] < 0 || (uint64_t)out[i] >= count || seen[out[i]]++) { failures++; break; }
        }
    }
    if (failures) { printf("FAIL %d\n", failures); return 1; }
    printf("ok\n");
    return 0;
}
