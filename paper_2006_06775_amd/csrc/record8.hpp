// record8.hpp -- the mechanics pre-test on the grid build's 8-byte records (internal).
//
// Per axis a record holds the box index mod 4 above the offset within the box in units of
// b / 2^14 (16 bits), and the radius in the same units rounded up plus one unit.  For two agents
// whose boxes are within one of each other along every axis, the fields' differences modulo
// 2^16, read as signed, are the offsets in units; the test below passes every pair whose
// centres are closer than the sum of the radii.
#pragma once

#include "common.hpp"

namespace bdm {

// The own pre-test record arranged for touch8i: the x|y word as stored, and the z field negated
// modulo 2^16 beside the own radius, so that one packed 16-bit add gives (z_j - z_i, R_i + R_j).
struct Own8 {
    uint32_t xy, zr;
};
__device__ __forceinline__ Own8 own8(uint2 a) {
    return Own8{a.x, ((0x10000u - (a.y & 0xFFFFu)) & 0xFFFFu) | (a.y & 0xFFFF0000u)};
}

// Conservative contact pre-test on the 8-byte records (units of b / 2^14; pre8_axis in k_grid.hip), in
// exact integer arithmetic.  Per axis the 16-bit fields
// differ, modulo 2^16 and read as signed, by the offset in units (boxes within one of each other;
// see pre8_axis), which is below 2^15 in magnitude; so the packed 16-bit differences, a signed
// dot product of the (x, y) pair (below 2^31) and the z square (the sum below 3 * 2^30, exact as
// an unsigned word) give the squared decoded distance exactly.  A pair the exact law counts as a
// contact has a decoded distance below r_i + r_j + 1.76 units and each stored radius is at least
// one unit above the true one, so the decoded distance is below R_i + R_j: no contact fails.
typedef short bdm_s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short bdm_u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ bool touch8i(const Own8 &a, uint2 c) {
    const bdm_s16x2 d = __builtin_bit_cast(bdm_s16x2, c.x) - __builtin_bit_cast(bdm_s16x2, a.xy);
    const int dxy = __builtin_amdgcn_sdot2(d, d, 0, false);
    const uint32_t zr = __builtin_bit_cast(uint32_t, __builtin_bit_cast(bdm_u16x2, c.y) + __builtin_bit_cast(bdm_u16x2, a.zr));
    const int dz = int(int16_t(uint16_t(zr)));
    const uint32_t d2 = uint32_t(dxy) + uint32_t(dz * dz);
    const uint32_t R = zr >> 16;
    return d2 < R * R;
}

}  // namespace bdm
