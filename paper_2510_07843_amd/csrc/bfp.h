// Block floating point compression of the received grid (bfp.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ranphy {

// Antennas per block for Nr antennas (16, or Nr below 16); 0 when unsupported.
int bfp_block(int n_rx);
// 32-bit words per block of b antennas: the exponent and the packed 9-bit mantissas.
int64_t bfp_words_per_block(int b);
hipError_t launch_bfp_compress(int b, int64_t n_blocks, const float* rx, unsigned* out,
                               hipStream_t s);
hipError_t launch_bfp_decompress(int b, int64_t n_blocks, const unsigned* in, float* rx,
                                 hipStream_t s);

}  // namespace ranphy
