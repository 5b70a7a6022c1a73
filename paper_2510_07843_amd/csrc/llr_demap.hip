// Max-log LLR soft demapping of Gray square QAM, one thread per (resource element, layer);
// the per-axis arithmetic is in llr_math.h.
#include "geom.h"
#include "llr_math.h"

namespace ranphy {
namespace {

// One (RE, layer) element per thread.
template <int QM>
__global__ void __launch_bounds__(256) llr_kernel(int64_t n, const float2* __restrict__ x,
                                                  const float* __restrict__ nv,
                                                  float* __restrict__ llr) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float out[QM];
  llr_one<QM>(x[e], nv[e], out);
  float2* __restrict__ dst = reinterpret_cast<float2*>(llr + e * QM);
#pragma unroll
  for (int b = 0; b < QM / 2; ++b) dst[b] = make_float2(out[2 * b], out[2 * b + 1]);
}

// One element per thread, outputs staged in LDS so that the block's contiguous output
// (256 QM floats) leaves as 16-byte stores with consecutive threads on consecutive pieces
// (llr 16-byte aligned).
template <int QM>
__global__ void __launch_bounds__(256) llr_kernel_lds(int64_t n, const float2* __restrict__ x,
                                                      const float* __restrict__ nv,
                                                      float* __restrict__ llr) {
  __shared__ __attribute__((aligned(16))) float stage[256 * QM];
  const int64_t e0 = (int64_t)blockIdx.x * 256;
  const int cnt = (int)min<int64_t>(256, n - e0);
  const int t = threadIdx.x;
  if (t < cnt) {
    float out[QM];
    llr_one<QM>(x[e0 + t], nv[e0 + t], out);
#pragma unroll
    for (int b = 0; b < QM; ++b) stage[t * QM + b] = out[b];
  }
  __syncthreads();
  const int nf = cnt * QM;
  float4* __restrict__ dst = reinterpret_cast<float4*>(llr + e0 * QM);
  const float4* __restrict__ src = reinterpret_cast<const float4*>(stage);
  for (int f = t; f < nf / 4; f += 256) dst[f] = src[f];
  for (int f = (nf / 4) * 4 + t; f < nf; f += 256) llr[e0 * QM + f] = stage[f];
}

}  // namespace

hipError_t launch_llr_demap(const Geom& g, const float2* x, const float* nv, float* llr,
                            hipStream_t s) {
  const int64_t n = (int64_t)g.n_slots * g.n_dsym * g.n_sc * g.n_layers;
  if (n == 0) return hipSuccess;
  const dim3 block(256);
  const dim3 grid((unsigned)((n + 255) / 256));
  if (((uintptr_t)llr & 15u) == 0) {
    switch (g.qm) {
      case 2: hipLaunchKernelGGL(llr_kernel_lds<2>, grid, block, 0, s, n, x, nv, llr); break;
      case 4: hipLaunchKernelGGL(llr_kernel_lds<4>, grid, block, 0, s, n, x, nv, llr); break;
      case 6: hipLaunchKernelGGL(llr_kernel_lds<6>, grid, block, 0, s, n, x, nv, llr); break;
      case 8: hipLaunchKernelGGL(llr_kernel_lds<8>, grid, block, 0, s, n, x, nv, llr); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (g.qm) {
    case 2: hipLaunchKernelGGL(llr_kernel<2>, grid, block, 0, s, n, x, nv, llr); break;
    case 4: hipLaunchKernelGGL(llr_kernel<4>, grid, block, 0, s, n, x, nv, llr); break;
    case 6: hipLaunchKernelGGL(llr_kernel<6>, grid, block, 0, s, n, x, nv, llr); break;
    case 8: hipLaunchKernelGGL(llr_kernel<8>, grid, block, 0, s, n, x, nv, llr); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ranphy
