// Exact max-log LLR of Gray square QAM per axis, shared by the demapper kernel and the
// detector's fused demapping epilogue.
//
// The 2-D minimum over the constellation splits per axis for square Gray QAM, and on one
// axis the exact max-log value needs only the nearest PAM level and the distance to the
// nearest decision boundary of each bit, so the cost is O(Qm) instead of O(2^Qm):
//   u   = axis value in unnormalised units (levels +-1, +-3, .., +-(2^m - 1)), m = Qm/2;
//   a*  = nearest level, e = u - a*;
//   t_0 = u,  t_i = 2^(m-i) - |t_{i-1}|   (bit i is 0 where t_i > 0, its boundaries are the
//         zeros of t_i and |t_i| is the distance to the nearest one);
//   the nearest level with bit i flipped lies just across that boundary, at distance
//   |t_i| + 1, so  llr_i = sign(t_i) ((|t_i| + 1)^2 - e^2) / (scale^2 nv).
// Bits b0, b2, .. come from the in-phase axis and b1, b3, .. from the quadrature axis.
#pragma once

#include <hip/hip_runtime.h>

namespace ranphy {

// The sign of each LLR is the sign of t_i.  Where t_i is zero (u on that bit's boundary) the
// numerator is zero too, so the sign of zero never matters.
template <int M>
__device__ __forceinline__ void axis_llr(float u, float inv, float* out /* stride 2 */) {
  constexpr float lim = (float)((1 << M) - 1);
  float a = 2.f * floorf(0.5f * u) + 1.f;
  a = fminf(fmaxf(a, -lim), lim);
  const float e = u - a;
  const float e2 = e * e;
  float t = u;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    if (i > 0) t = (float)(1 << (M - i)) - fabsf(t);
    const float dd = fabsf(t) + 1.f;
    out[2 * i] = copysignf(fmaf(dd, dd, -e2) * inv, t);
  }
}

// 1 / (scale^2 nv) by the hardware reciprocal (1 ulp): the LLRs carry the relative error of
// the variance estimate, orders of magnitude above it.  nv = 0 gives infinite LLRs and an
// infinite nv zero ones, as exact division would.
template <int QM>
__device__ __forceinline__ void llr_one(float2 v, float nvv, float* out) {
  constexpr int M = QM / 2;
  constexpr float sc2 = 2.f * (float)((1 << QM) - 1) / 3.f;  // scale^2
  const float scale = __builtin_sqrtf(sc2);
  const float inv = __builtin_amdgcn_rcpf(sc2 * nvv);
  axis_llr<M>(v.x * scale, inv, out);
  axis_llr<M>(v.y * scale, inv, out + 1);
}

}  // namespace ranphy
