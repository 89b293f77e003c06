// Gap-free output after block-reserved emission (host logic, no HIP).
//
// Wavefronts reserve output positions in blocks; the unused tail of each
// wavefront's last block is a hole.  With `count` triangles written into
// [0, reserved) minus the holes, plan_hole_moves() returns copies that move
// the triangles found at or above `count` into the holes below `count`, so
// that [0, count) ends up fully populated.
#pragma once
#include <algorithm>
#include <cstdint>
#include <stdexcept>
#include <vector>

struct Hole {
    uint64_t start, len;
};

struct Move {
    uint64_t src, dst, len;  // in triangles
};

inline std::vector<Move> plan_hole_moves(std::vector<Hole> holes, uint64_t count, uint64_t reserved) {
    std::sort(holes.begin(), holes.end(), [](const Hole &x, const Hole &y) { return x.start < y.start; });
    std::vector<Hole> low, data;
    uint64_t at = count;  // walks [count, reserved), skipping holes
    for (const Hole &h : holes) {
        const uint64_t hs = h.start, he = h.start + h.len;
        if (hs < count) low.push_back(Hole{hs, (he < count ? he : count) - hs});
        if (he > count) {
            const uint64_t ds = hs > at ? hs : at;
            if (ds > at) data.push_back(Hole{at, ds - at});
            if (he > at) at = he;
        }
    }
    if (reserved > at) data.push_back(Hole{at, reserved - at});
    std::vector<Move> mv;
    size_t di = 0;
    uint64_t doff = 0;
    for (const Hole &h : low) {
        uint64_t filled = 0;
        while (filled < h.len) {
            if (di >= data.size()) throw std::runtime_error("hole fix-up: holes exceed displaced triangles");
            const uint64_t take = std::min(h.len - filled, data[di].len - doff);
            mv.push_back(Move{data[di].start + doff, h.start + filled, take});
            filled += take;
            doff += take;
            if (doff == data[di].len) {
                di++;
                doff = 0;
            }
        }
    }
    return mv;
}
