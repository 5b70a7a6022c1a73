// Reading one sample of the received grid, given as complex64 (RXF = 0) or in block floating
// point form (RXF = 1, ranphy_bfp_compress: blocks of B = 16 antennas, or all NR when NR is
// below 16, each one exponent word e then the 9-bit two's complement mantissas m of the
// block's I, Q values as a little-endian bit stream, value m 2^e).  Antenna i of a block has
// its two fields in bits 18 i .. 18 i + 17, inside the block's last word, so the second word
// is read only when the fields reach it.  The values equal bfp_decompress_kernel's bit for bit.
#pragma once

#include "geom.h"

namespace ranphy {

template <int RXF>
__device__ __forceinline__ float2 rx_at(const float2* __restrict__ rx, int64_t re, int NR,
                                        int r) {
  if constexpr (RXF == 0) {
    return rx[re * NR + r];
  } else {
    const bool wide = NR >= 16;
    const int B = wide ? 16 : NR;
    const int W = 1 + (18 * B + 31) / 32;
    const int i = wide ? (r & 15) : r;
    const unsigned* b = reinterpret_cast<const unsigned*>(rx) +
                        (re * (wide ? (NR >> 4) : 1) + (wide ? (r >> 4) : 0)) * W;
    const int bit = 18 * i, word = 1 + (bit >> 5), sh = bit & 31;
    const unsigned long long f =
        (((unsigned long long)b[word + (sh > 14 ? 1 : 0)] << 32) | b[word]) >> sh;
    const int e = (int)b[0];
    return make_float2(ldexpf((float)((int)((unsigned)f << 23) >> 23), e),
                       ldexpf((float)((int)((unsigned)(f >> 9) << 23) >> 23), e));
  }
}

}  // namespace ranphy
