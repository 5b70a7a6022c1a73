// Block floating point (BFP) compression of the received grid: the fronthaul compression the
// paper proposes for distributed MIMO (Sec. VI-A), which fixes no format.  Format (a reading):
// blocks of B consecutive antennas of one resource element (B = 16 for a multiple of 16
// antennas, else B = Nr < 16); the block's 2B real values (I and Q interleaved, antenna order)
// share the exponent e, the smallest integer with max |v| <= 255 * 2^e (0 for zeros), and
// each is stored as the 9-bit two's complement mantissa m = round-half-even(v / 2^e), so that
// the value is m * 2^e.  A block is one 32-bit word holding e followed by ceil(18 B / 32)
// words of mantissas, a little-endian bit stream with m_i in bits 9 i .. 9 i + 8.  All
// scalings are by powers of two, so the arithmetic is exact in FP32.  Compression takes one
// thread per block, decompression one thread per complex sample.
#include "bfp.h"

namespace ranphy {
namespace {

constexpr int kMaxMant = 255;

__host__ __device__ constexpr int bfp_words(int b) { return 1 + (18 * b + 31) / 32; }

// Smallest e with a <= 255 * 2^e, compared as a * 2^-e <= 255 (exact for every finite a).
// With k = ilogb(a), 2^k <= a < 2^(k+1) puts e at k - 7 or k - 6, so each loop takes at most
// one step; a non-finite a (not a valid sample) gets e = 121 and saturated mantissas.
__device__ __forceinline__ int bfp_exponent(float a) {
  if (a == 0.f) return 0;
  if (!(a <= __FLT_MAX__)) return 121;
  int e = ilogbf(a) - 7;
  for (int it = 0; it < 3 && ldexpf(a, -e) > (float)kMaxMant; ++it) ++e;
  for (int it = 0; it < 3 && ldexpf(a, 1 - e) <= (float)kMaxMant; ++it) --e;
  return e;
}

template <int B>
__global__ void __launch_bounds__(256) bfp_compress_kernel(const float* __restrict__ rx,
                                                           unsigned* __restrict__ out,
                                                           int64_t n_blocks) {
  constexpr int W = bfp_words(B);
  const int64_t blk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (blk >= n_blocks) return;
  float v[2 * B];
  const float* src = rx + blk * 2 * B;
#pragma unroll
  for (int i = 0; i < 2 * B; ++i) v[i] = src[i];
  float a = 0.f;
#pragma unroll
  for (int i = 0; i < 2 * B; ++i) a = fmaxf(a, fabsf(v[i]));
  const int e = bfp_exponent(a);
  unsigned w[W - 1];
#pragma unroll
  for (int j = 0; j < W - 1; ++j) w[j] = 0u;
#pragma unroll
  for (int i = 0; i < 2 * B; ++i) {
    const float q = fminf(fmaxf(rintf(ldexpf(v[i], -e)), -256.f), (float)kMaxMant);
    const unsigned m = (unsigned)(int)q & 0x1FFu;
    const int bit = 9 * i, word = bit >> 5, sh = bit & 31;
    w[word] |= m << sh;
    if (sh > 23) w[word + 1] |= m >> (32 - sh);
  }
  unsigned* dst = out + blk * W;
  dst[0] = (unsigned)e;
#pragma unroll
  for (int j = 0; j < W - 1; ++j) dst[1 + j] = w[j];
}

// One thread per complex sample (antenna i of a block): the block's exponent word and the one
// or two words holding its 18 bits, then one coalesced float2 store.  A sample's fields end at
// bit 18 i + 17 <= 18 B - 1, inside the block's last mantissa word, so the second word is read
// only when the fields reach it and never past the block.
template <int B>
__global__ void __launch_bounds__(256) bfp_decompress_kernel(const unsigned* __restrict__ in,
                                                             float2* __restrict__ rx,
                                                             int64_t n_samples) {
  constexpr int W = bfp_words(B);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_samples) return;
  const int64_t blk = t / B;
  const int i = (int)(t - blk * B);
  const unsigned* src = in + blk * W;
  const int e = (int)src[0];
  const int bit = 18 * i, word = bit >> 5, sh = bit & 31;
  const unsigned lo = src[1 + word];
  const unsigned hi = sh > 14 ? src[2 + word] : 0u;
  const uint64_t f = (((uint64_t)hi << 32) | lo) >> sh;
  const int m0 = (int)((unsigned)f << 23) >> 23;  // sign-extend each 9-bit field
  const int m1 = (int)((unsigned)(f >> 9) << 23) >> 23;
  rx[t] = make_float2(ldexpf((float)m0, e), ldexpf((float)m1, e));
}

}  // namespace

int bfp_block(int n_rx) { return n_rx % 16 == 0 ? 16 : (n_rx < 16 ? n_rx : 0); }
int64_t bfp_words_per_block(int b) { return bfp_words(b); }

// One kernel instance per block width (1..16 antennas): the block's values stay in registers.
#define RANPHY_BFP_SWITCH(KERNEL, ...)                                                     \
  switch (b) {                                                                             \
    case 1: hipLaunchKernelGGL((KERNEL<1>), grid, dim3(256), 0, s, __VA_ARGS__); break;    \
    case 2: hipLaunchKernelGGL((KERNEL<2>), grid, dim3(256), 0, s, __VA_ARGS__); break;    \
    case 3: hipLaunchKernelGGL((KERNEL<3>), grid, dim3(256), 0, s, __VA_ARGS__); break;    \
    case 4: hipLaunchKernelGGL((KERNEL<4>), grid, dim3(256), 0, s, __VA_ARGS__); break;    \
    case 5: hipLaunchKernelGGL((KERNEL<5>), grid, dim3(256), 0, s, __VA_ARGS__); break;    \
    case 6: hipLaunchKernelGGL((KERNEL<6>), grid, dim3(256), 0, s, __VA_ARGS__); break;    \
    case 7: hipLaunchKernelGGL((KERNEL<7>), grid, dim3(256), 0, s, __VA_ARGS__); break;    \
    case 8: hipLaunchKernelGGL((KERNEL<8>), grid, dim3(256), 0, s, __VA_ARGS__); break;    \
    case 9: hipLaunchKernelGGL((KERNEL<9>), grid, dim3(256), 0, s, __VA_ARGS__); break;    \
    case 10: hipLaunchKernelGGL((KERNEL<10>), grid, dim3(256), 0, s, __VA_ARGS__); break;  \
    case 11: hipLaunchKernelGGL((KERNEL<11>), grid, dim3(256), 0, s, __VA_ARGS__); break;  \
    case 12: hipLaunchKernelGGL((KERNEL<12>), grid, dim3(256), 0, s, __VA_ARGS__); break;  \
    case 13: hipLaunchKernelGGL((KERNEL<13>), grid, dim3(256), 0, s, __VA_ARGS__); break;  \
    case 14: hipLaunchKernelGGL((KERNEL<14>), grid, dim3(256), 0, s, __VA_ARGS__); break;  \
    case 15: hipLaunchKernelGGL((KERNEL<15>), grid, dim3(256), 0, s, __VA_ARGS__); break;  \
    case 16: hipLaunchKernelGGL((KERNEL<16>), grid, dim3(256), 0, s, __VA_ARGS__); break;  \
    default: return hipErrorInvalidValue;                                                  \
  }

// Launches cover at most kChunk blocks each (a grid's threads stay well inside 32 bits).
constexpr int64_t kChunk = int64_t(1) << 26;

hipError_t launch_bfp_compress(int b, int64_t n_blocks, const float* rx, unsigned* out,
                               hipStream_t s) {
  for (int64_t b0 = 0; b0 < n_blocks; b0 += kChunk) {
    const int64_t n = n_blocks - b0 < kChunk ? n_blocks - b0 : kChunk;
    const dim3 grid((unsigned)((n + 255) / 256));
    const float* src = rx + b0 * 2 * b;
    unsigned* dst = out + b0 * bfp_words(b);
    RANPHY_BFP_SWITCH(bfp_compress_kernel, src, dst, n)
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_bfp_decompress(int b, int64_t n_blocks, const unsigned* in, float* rx,
                                 hipStream_t s) {
  for (int64_t b0 = 0; b0 < n_blocks; b0 += kChunk) {
    const int64_t n = n_blocks - b0 < kChunk ? n_blocks - b0 : kChunk;
    const dim3 grid((unsigned)((n * b + 255) / 256));
    const unsigned* src = in + b0 * bfp_words(b);
    float2* dst = reinterpret_cast<float2*>(rx) + b0 * b;
    RANPHY_BFP_SWITCH(bfp_decompress_kernel, src, dst, n * b)
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
#undef RANPHY_BFP_SWITCH

}  // namespace ranphy
