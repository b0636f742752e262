// Positions in the LDS tile row of the wave-per-line line pass
// (line_pass3.hip), kept in a header of their own so that host code can
// check them (tests/tile_map_check.cpp).
//
// A tile row holds one line's window of 32 R slots; lane i of the line owns
// slots i R .. i R + R - 1 and keeps them in its own segment of the row, but
// the segment's 16-byte chunks are rotated by a lane-dependent amount.
// Unrotated, the 128-bit accesses of consecutive lanes to their own segments
// (64 bytes in FP32, 128 in FP64) would meet in the same LDS banks every
// second (every) lane; rotated, the lanes of any group of 8 (32 banks) or 16
// (64 banks) consecutive lanes touch distinct banks, both for their own
// segments and for consecutive chunks of a row.
#pragma once

#ifndef ADI_HD
#define ADI_HD __host__ __device__
#endif

namespace adi {

// R slots per lane, ESZ bytes per element
template <int R, int ESZ> struct TileMap {
    static constexpr int VEC = 16 / ESZ, NC = R / VEC;
    static constexpr int S = NC == 4 ? 1 : 0, LNC = NC == 4 ? 2 : 3;
    static_assert(NC == 4 || NC == 8, "segments of 64 or 128 bytes");
    // chunk c of lane i's segment
    ADI_HD static inline int chunk(int i, int c) {
        const int rot = ((i >> S) + (i >> (S + LNC))) & (NC - 1);
        return i * R + ((c + rot) & (NC - 1)) * VEC;
    }
    // window slot sl
    ADI_HD static inline int slot(int sl) {
        const int o = sl % R;
        return chunk(sl / R, o / VEC) + o % VEC;
    }
};

}  // namespace adi
