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

template <int M>
__device__ __forceinline__ void axis_llr(float u, float* out /* stride 2 */) {
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
    const float num = dd * dd - e2;
    out[2 * i] = (t >= 0.f) ? num : -num;
  }
}

template <int QM>
__device__ __forceinline__ void llr_one(float2 v, float nvv, float* out) {
  constexpr int M = QM / 2;
  constexpr float sc2 = 2.f * (float)((1 << QM) - 1) / 3.f;  // scale^2
  const float scale = sqrtf(sc2);
  const float inv = 1.f / (sc2 * nvv);
  axis_llr<M>(v.x * scale, out);
  axis_llr<M>(v.y * scale, out + 1);
#pragma unroll
  for (int b = 0; b < QM; ++b) out[b] *= inv;
}

}  // namespace ranphy
