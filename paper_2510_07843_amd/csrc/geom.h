// Slot geometry shared by the host layer and the kernels of libranphy.
//
// The host validates a ranphy_slot_desc once and derives everything a kernel needs:
// subcarrier and pilot counts, the list of data symbols and, per data symbol, the two
// DMRS occasions and the weight of the linear time interpolation.  The struct is passed
// to every kernel by value (it lives in the kernel-argument segment, read through the
// scalar cache).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ranphy {

constexpr int kMaxSymb = 14;
constexpr int kMaxRx = 64;
constexpr int kMaxLayers = 16;

struct Geom {
  int n_slots;
  int n_symb;
  int n_sc;
  int n_rx;
  int n_layers;
  int qm;
  int comb;     // C
  int comb_log2;
  int td;       // T
  int n_occ;
  int n_pilot;  // ceil(n_sc / C)
  int n_dsym;
  int sym0[4];
  int dsym[16];     // data symbol indices, ascending
  int t_o0[16];     // per data symbol: occasion before ...
  int t_o1[16];     // ... and after it
  float t_w[16];    // weight of t_o1: H = H_o0 + t_w (H_o1 - H_o0)
};

// Frequency interpolation rule for layer (port) p at subcarrier k: the two pilot indices
// of that port and the weight a of the second one.  Linear between the port's consecutive
// pilots at k = c + C j (c = p mod C), nearest pilot held outside the first and last one.
__device__ __forceinline__ void freq_rule(const Geom& g, int p, int k, int& j0, int& j1,
                                          float& a) {
  const int C = g.comb, L = g.comb_log2;  // C is a power of two
  const int c = p & (C - 1);
  const int jp = (g.n_sc - c + C - 1) >> L;
  const int last = c + C * (jp - 1);
  if (k <= c) {
    j0 = j1 = 0;
    a = 0.f;
  } else if (k >= last) {
    j0 = j1 = jp - 1;
    a = 0.f;
  } else {
    j0 = (k - c) >> L;
    j1 = j0 + 1;
    a = ldexpf((float)(k - c - C * j0), -L);  // exact: / C with C = 2^L
  }
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// LS estimate at one pilot from its T received samples y[t] and pilot values q[t]:
// (1/T) sum_t y_t conj(q_t), every rounding step written out (fused multiply-adds in a fixed
// order, then the exact scaling by 1/T) so that every kernel forming it gets the same bits.
template <int T>
__device__ __forceinline__ float2 ls_pilot(const float2 (&q)[T], const float2 (&y)[T]) {
  float re = 0.f, im = 0.f;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    re = fmaf(q[t].x, y[t].x, fmaf(q[t].y, y[t].y, re));
    im = fmaf(q[t].x, y[t].y, fmaf(-q[t].y, y[t].x, im));
  }
  constexpr float inv = 1.f / (float)T;
  return make_float2(re * inv, im * inv);
}

// Kernel launchers (one translation unit each).  They return a hipError_t.
// rx: the complex64 grid, or with bfp its block floating point words (ranphy_bfp_compress).
hipError_t launch_chest_ls(const Geom& g, const float2* rx, bool bfp, const float2* pilots,
                           float2* h, int h_res, hipStream_t s);
hipError_t launch_mmse_re(const Geom& g, const float2* rx, const float2* h, int h_res,
                          const float* noise_var, float2* x, float* nv, hipStream_t s);
// One thread per subcarrier (one DMRS occasion, Nr in {1,2,4,8}, Nl <= 8, Nr Nl <= 64).
bool mmse_sc_eligible(const Geom& g);
hipError_t launch_mmse_sc(const Geom& g, const float2* rx, const float2* h, int h_res,
                          const float* nvar, float2* x, float* nv, hipStream_t s);
hipError_t launch_llr_demap(const Geom& g, const float2* x, const float* nv, float* llr,
                            hipStream_t s);

// The channel-estimate denoiser (cnn.hip).  Tensors [group][pixel][image][2] FP32.
int64_t cnn_param_count();
int64_t cnn_workspace_bytes(int rows, int cols, int nimg, int ngrp, bool train);
// With per-group noise variances nv (may be null: none) the network refines noise-normalised
// estimates, and groups with nv[g] < gate_min keep x.
hipError_t cnn_forward(int rows, int cols, int nimg, int ngrp, const float* params,
                       const float* x, float* out, void* ws, hipStream_t s,
                       const float* nv = nullptr, float gate_min = 0.f);
hipError_t cnn_grad(int rows, int cols, int nimg, int ngrp, const float* params, const float* x,
                    const float* target, const float* nv, float* grad, float* loss, void* ws,
                    hipStream_t s);
hipError_t cnn_adam(float* params, const float* grad, float* m, float* v, int step, float lr,
                    hipStream_t s);

}  // namespace ranphy
