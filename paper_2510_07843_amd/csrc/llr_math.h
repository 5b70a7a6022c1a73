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
//
// axis_llr takes uh = u / 2 (the axis value times scale / 2, which is exactly half of the
// value times scale): floor(u / 2) needs no extra multiply, and every use of u is formed
// from uh with an exact doubling inside a fused multiply-add, so each rounded result is the
// one the same expression in u would give.
template <int M>
__device__ __forceinline__ void axis_llr(float uh, float inv, float* out /* stride 2 */) {
  constexpr float lim = (float)((1 << M) - 1);
  float a = fmaf(floorf(uh), 2.f, 1.f);
  a = fminf(fmaxf(a, -lim), lim);
  const float e = fmaf(uh, 2.f, -a);  // u - a
  const float e2 = e * e;
  float t = uh;                       // t_0 = u: only its sign and |u| + 1 are used
#pragma unroll
  for (int i = 0; i < M; ++i) {
    float dd;
    if (i == 0) {
      dd = fmaf(fabsf(uh), 2.f, 1.f);  // |u| + 1
    } else if (i == 1) {
      t = fmaf(-fabsf(uh), 2.f, (float)(1 << (M - 1)));  // 2^(m-1) - |u|
      dd = fabsf(t) + 1.f;
    } else {
      t = (float)(1 << (M - i)) - fabsf(t);
      dd = fabsf(t) + 1.f;
    }
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
  const float half_scale = 0.5f * __builtin_sqrtf(sc2);          // exact halving
  const float inv = __builtin_amdgcn_rcpf(sc2 * nvv);
  axis_llr<M>(v.x * half_scale, inv, out);
  axis_llr<M>(v.y * half_scale, inv, out + 1);
}

}  // namespace ranphy
