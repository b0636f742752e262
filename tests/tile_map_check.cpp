// Host check of the LDS tile map of the wave-per-line line pass
// (paper_2006_07583_amd/csrc/tile_map.h): the positions of a row form a
// permutation, slot() agrees with chunk(), and the 128-bit accesses the
// kernel makes are free of bank conflicts under both bank models (32 banks
// serving 8 lanes per cycle, 64 banks serving 16).  Exit status 0 = pass.
#define ADI_HD
#include "tile_map.h"

#include <cstdio>
#include <vector>

namespace {

constexpr int kR = 16, kLanes = 32;

// banks of the 16 bytes at element position pos
template <int ESZ>
void banks_of(int pos, int nbanks, std::vector<int>& out) {
    const int w0 = pos * ESZ / 4;
    for (int b = 0; b < 4; ++b) out.push_back((w0 + b) % nbanks);
}

template <int ESZ>
int check() {
    using M = adi::TileMap<kR, ESZ>;
    int fails = 0;
    // permutation of the row, and slot() consistent with chunk()
    std::vector<int> seen(kLanes * kR, 0);
    for (int i = 0; i < kLanes; ++i)
        for (int c = 0; c < M::NC; ++c)
            for (int e = 0; e < M::VEC; ++e) {
                const int p = M::chunk(i, c) + e;
                if (p < 0 || p >= kLanes * kR) { ++fails; continue; }
                ++seen[p];
                if (M::slot(i * kR + c * M::VEC + e) != p) ++fails;
            }
    for (int v : seen) fails += v != 1;
    // every chunk starts on a 16-byte boundary
    for (int i = 0; i < kLanes; ++i)
        for (int c = 0; c < M::NC; ++c) fails += (M::chunk(i, c) * ESZ) % 16 != 0;
    const int models[2][2] = {{32, 8}, {64, 16}};
    for (const auto& m : models) {
        const int nbanks = m[0], group = m[1];
        // each lane reading chunk c of its own segment
        for (int c = 0; c < M::NC; ++c)
            for (int g = 0; g < kLanes; g += group) {
                std::vector<int> used(nbanks, 0), b;
                for (int i = g; i < g + group; ++i) banks_of<ESZ>(M::chunk(i, c), nbanks, b);
                for (int x : b) fails += used[x]++ != 0;
            }
        // consecutive threads moving consecutive chunks of a row (staging)
        for (int g = 0; g < kLanes * M::NC; g += group) {
            std::vector<int> used(nbanks, 0), b;
            for (int q = g; q < g + group; ++q) banks_of<ESZ>(M::chunk(q / M::NC, q % M::NC), nbanks, b);
            for (int x : b) fails += used[x]++ != 0;
        }
    }
    return fails;
}

}  // namespace

int main() {
    const int f4 = check<4>(), f8 = check<8>();
    std::printf("tile map: FP32 %d failures, FP64 %d failures\n", f4, f8);
    return f4 + f8 == 0 ? 0 : 1;
}
