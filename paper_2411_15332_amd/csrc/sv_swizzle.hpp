// LDS slot swizzle shared by the planner (lane choice) and the pass kernel.
//
// An exchange writes the tile to LDS in one layout and reads it back in
// another. Slot(l) = l ^ S(l), where S is linear over GF(2): it XORs into the
// low m slot bits a fixed nonzero m-bit vector for every tile-local bit b >= m
// that is set. S(l) only reads bits >= m and only writes bits < m, so the map
// is an involution (a bijection). A group of 2^m consecutive lanes then hits
// 2^m distinct bank groups whenever the images of the local bits assigned to
// lane bits 0..m-1 are linearly independent; the planner picks lanes so.
//   complex128 (16-byte slots): m = 3 (8 lanes x 16 B = one 128-byte LDS row)
//   complex64  (8-byte slots):  m = 4 (16 lanes x 8 B)
#pragma once

#include <cstdint>

#if defined(__HIP__)
#define SV_HD __host__ __device__
#else
#define SV_HD
#endif

namespace sv {

// Images for local bits b = m, m+1, ...: cycle through all nonzero vectors so
// that no 2-dimensional subspace (for m = 3) holds many of them. Packed as
// 4-bit nibbles, entry i at bits [4i, 4i+4):
//   m = 3: 1, 2, 4, 3, 6, 7, 5
//   m = 4: 1, 2, 4, 8, 3, 6, 12, 11, 5, 10, 7, 14, 15, 13, 9
static constexpr uint64_t kSwz3Packed = 0x5763421ull;
static constexpr uint64_t kSwz4Packed = 0x9DFE7A5BC638421ull;

// Image of tile-local bit b in the low m bits of the slot index.
SV_HD inline uint32_t swz_image(int b, int m) {
    if (b < m) return 1u << b;
    if (m == 3) return (uint32_t)((kSwz3Packed >> (4 * ((b - 3) % 7))) & 0xF);
    return (uint32_t)((kSwz4Packed >> (4 * ((b - 4) % 15))) & 0xF);
}

// S(l) restricted to the bits >= m of l.
SV_HD inline uint32_t swz_fold(uint32_t l, int m) {
    uint32_t s = 0;
    for (int b = m; b < 32; ++b)
        if ((l >> b) & 1u) s ^= swz_image(b, m);
    return s;
}

}  // namespace sv
