// libranphy host layer: descriptor validation, geometry derivation, kernel dispatch.
//
// Everything here runs on the host before any launch, so every error path can be
// exercised without a GPU.  The library allocates nothing and keeps no state between
// calls.
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "batch.h"
#include "bfp.h"
#include "geom.h"
#include "ranphy.h"

namespace ranphy {

// rx: the complex64 grid, or with bfp its block floating point words (16-antenna blocks).
// pil: NULL to read h, or the pilots, the pilot-resolution estimate then being formed in the
// kernel (h unused, h_res pilot).
hipError_t launch_mmse_mfma(const Geom& g, const float2* rx, bool bfp, const float2* h,
                            const float2* pil, int h_res, const float* noise_var, float2* x,
                            float* nv, float* llr, int prec, hipStream_t s);
bool mmse_mfma_eligible(const Geom& g, const void* rx, const void* h, const void* x,
                        const void* nv, const void* llr);

namespace {

bool is_pow2_comb(int c) { return c == 2 || c == 4 || c == 8; }

// Validate `d` and fill `g`; returns a ranphy status.
int make_geom(const ranphy_slot_desc* d, Geom* g) {
  if (!d) return RANPHY_ERR_INVALID;
  if (d->n_slots < 0 || d->n_prb < 1 || d->n_prb > 275) return RANPHY_ERR_INVALID;
  if (d->n_symb < 1 || d->n_symb > kMaxSymb) return RANPHY_ERR_INVALID;
  if (d->n_rx < 1 || d->n_layers < 1) return RANPHY_ERR_INVALID;
  if (d->qm != 2 && d->qm != 4 && d->qm != 6 && d->qm != 8) return RANPHY_ERR_INVALID;
  if (!is_pow2_comb(d->dmrs_comb)) return RANPHY_ERR_INVALID;
  if (d->dmrs_td != 1 && d->dmrs_td != 2) return RANPHY_ERR_INVALID;
  if (d->n_occ < 1 || d->n_occ > 4) return RANPHY_ERR_INVALID;
  for (int o = 0; o < d->n_occ; ++o) {
    if (d->dmrs_sym0[o] < 0 || d->dmrs_sym0[o] + d->dmrs_td > d->n_symb) return RANPHY_ERR_INVALID;
    if (o > 0 && d->dmrs_sym0[o] < d->dmrs_sym0[o - 1] + d->dmrs_td) return RANPHY_ERR_INVALID;
  }
  if (d->n_rx > kMaxRx || d->n_layers > kMaxLayers) return RANPHY_ERR_UNSUPPORTED;
  if (d->n_layers > d->n_rx) return RANPHY_ERR_UNSUPPORTED;
  if (d->n_layers > d->dmrs_comb * d->dmrs_td) return RANPHY_ERR_UNSUPPORTED;

  Geom z = {};
  z.n_slots = d->n_slots;
  z.n_symb = d->n_symb;
  z.n_sc = 12 * d->n_prb;
  z.n_rx = d->n_rx;
  z.n_layers = d->n_layers;
  z.qm = d->qm;
  z.comb = d->dmrs_comb;
  z.comb_log2 = d->dmrs_comb == 2 ? 1 : (d->dmrs_comb == 4 ? 2 : 3);
  z.td = d->dmrs_td;
  z.n_occ = d->n_occ;
  z.n_pilot = (z.n_sc + z.comb - 1) / z.comb;
  double centre[4];
  for (int o = 0; o < z.n_occ; ++o) {
    z.sym0[o] = d->dmrs_sym0[o];
    centre[o] = d->dmrs_sym0[o] + 0.5 * (d->dmrs_td - 1);
  }
  z.n_dsym = 0;
  for (int s = 0; s < z.n_symb; ++s) {
    bool dmrs = false;
    for (int o = 0; o < z.n_occ; ++o) dmrs = dmrs || (s >= z.sym0[o] && s < z.sym0[o] + z.td);
    if (dmrs) continue;
    const int di = z.n_dsym++;
    z.dsym[di] = s;
    // Linear interpolation in time between occasion centres, held outside them.
    int o0 = 0, o1 = 0;
    double w = 0.0;
    if (z.n_occ > 1 && s > centre[0]) {
      if (s >= centre[z.n_occ - 1]) {
        o0 = o1 = z.n_occ - 1;
      } else {
        for (int o = 0; o + 1 < z.n_occ; ++o)
          if (s >= centre[o] && s < centre[o + 1]) {
            o0 = o;
            o1 = o + 1;
            w = (s - centre[o]) / (centre[o + 1] - centre[o]);
          }
      }
    }
    z.t_o0[di] = o0;
    z.t_o1[di] = o1;
    z.t_w[di] = (float)w;
  }
  if (z.n_dsym == 0) return RANPHY_ERR_INVALID;
  *g = z;
  return RANPHY_OK;
}

bool aligned8(const void* p) { return p != nullptr && ((uintptr_t)p & 7u) == 0; }

bool precision_valid(int p) {
  return p == RANPHY_PREC_FP32 || p == RANPHY_PREC_FP16 || p == RANPHY_PREC_BF16 ||
         p == RANPHY_PREC_FP16_REFINED || p == RANPHY_PREC_BF16_REFINED;
}

int status_of(hipError_t e) { return e == hipSuccess ? RANPHY_OK : RANPHY_ERR_LAUNCH; }

}  // namespace
}  // namespace ranphy

using ranphy::Geom;

extern "C" {

int ranphy_abi_version(void) { return RANPHY_ABI_VERSION; }

const char* ranphy_status_str(int status) {
  switch (status) {
    case RANPHY_OK: return "ok";
    case RANPHY_ERR_INVALID: return "invalid argument (descriptor field, NULL or misaligned pointer)";
    case RANPHY_ERR_UNSUPPORTED: return "unsupported shape";
    case RANPHY_ERR_LAUNCH: return "HIP kernel launch failed";
    default: return "unknown status";
  }
}

int64_t ranphy_buffer_floats(const ranphy_slot_desc* d, int buf, int h_res) {
  Geom g;
  const int rc = ranphy::make_geom(d, &g);
  if (rc) return rc;
  const int64_t S = g.n_slots;
  switch (buf) {
    case RANPHY_BUF_RX: return 2 * S * g.n_symb * g.n_sc * g.n_rx;
    case RANPHY_BUF_PILOTS: return 2 * S * g.n_occ * g.td * g.n_pilot * g.n_layers;
    case RANPHY_BUF_H:
      if (h_res != RANPHY_H_PILOT && h_res != RANPHY_H_FULL) return RANPHY_ERR_INVALID;
      return 2 * S * g.n_occ * (h_res == RANPHY_H_PILOT ? g.n_pilot : g.n_sc) * g.n_rx * g.n_layers;
    case RANPHY_BUF_NOISE_VAR: return S;
    case RANPHY_BUF_X: return 2 * S * g.n_dsym * g.n_sc * g.n_layers;
    case RANPHY_BUF_NV: return S * g.n_dsym * g.n_sc * g.n_layers;
    case RANPHY_BUF_LLR: return S * g.n_dsym * g.n_sc * g.n_layers * g.qm;
    default: return RANPHY_ERR_INVALID;
  }
}

int ranphy_chest_ls(const ranphy_slot_desc* d, const float* rx, const float* pilots, float* h,
                    int h_res, void* stream) {
  Geom g;
  const int rc = ranphy::make_geom(d, &g);
  if (rc) return rc;
  if (h_res != RANPHY_H_PILOT && h_res != RANPHY_H_FULL) return RANPHY_ERR_INVALID;
  if (g.n_slots == 0) return RANPHY_OK;
  if (!ranphy::aligned8(rx) || !ranphy::aligned8(pilots) || !ranphy::aligned8(h))
    return RANPHY_ERR_INVALID;
  return ranphy::status_of(ranphy::launch_chest_ls(
      g, reinterpret_cast<const float2*>(rx), false, reinterpret_cast<const float2*>(pilots),
      reinterpret_cast<float2*>(h), h_res, static_cast<hipStream_t>(stream)));
}

int ranphy_chest_ls_bfp(const ranphy_slot_desc* d, const uint32_t* packed, const float* pilots,
                        float* h, int h_res, void* stream) {
  Geom g;
  const int rc = ranphy::make_geom(d, &g);
  if (rc) return rc;
  if (h_res != RANPHY_H_PILOT && h_res != RANPHY_H_FULL) return RANPHY_ERR_INVALID;
  if (ranphy::bfp_block(g.n_rx) == 0) return RANPHY_ERR_UNSUPPORTED;
  if (g.n_slots == 0) return RANPHY_OK;
  if (packed == nullptr || ((uintptr_t)packed & 3u) || !ranphy::aligned8(pilots) ||
      !ranphy::aligned8(h))
    return RANPHY_ERR_INVALID;
  return ranphy::status_of(ranphy::launch_chest_ls(
      g, reinterpret_cast<const float2*>(packed), true, reinterpret_cast<const float2*>(pilots),
      reinterpret_cast<float2*>(h), h_res, static_cast<hipStream_t>(stream)));
}

int ranphy_mmse_detect_prec(const ranphy_slot_desc* d, const float* rx, const float* h,
                            int h_res, const float* noise_var, float* x, float* nv,
                            int precision, void* stream) {
  Geom g;
  const int rc = ranphy::make_geom(d, &g);
  if (rc) return rc;
  if (h_res != RANPHY_H_PILOT && h_res != RANPHY_H_FULL) return RANPHY_ERR_INVALID;
  if (!ranphy::precision_valid(precision)) return RANPHY_ERR_INVALID;
  if (g.n_slots == 0) return RANPHY_OK;
  if (!ranphy::aligned8(rx) || !ranphy::aligned8(h) || !ranphy::aligned8(x) ||
      !ranphy::aligned8(nv) || noise_var == nullptr || ((uintptr_t)noise_var & 3u))
    return RANPHY_ERR_INVALID;
  const float2* rx2 = reinterpret_cast<const float2*>(rx);
  const float2* h2 = reinterpret_cast<const float2*>(h);
  float2* x2 = reinterpret_cast<float2*>(x);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool mfma = ranphy::mmse_mfma_eligible(g, rx, h, x, nv, nullptr);
  if (precision != RANPHY_PREC_FP32 && !mfma) return RANPHY_ERR_UNSUPPORTED;
  if (mfma)
    return ranphy::status_of(
        ranphy::launch_mmse_mfma(g, rx2, false, h2, nullptr, h_res, noise_var, x2, nv, nullptr,
                                 precision, s));
  // Small arrays with one DMRS occasion: one thread per subcarrier shares the Gram and its
  // factorisation over the data symbols, once the batch has a subcarrier for every lane of
  // the chip (256 CUs x 4 SIMDs x 64 lanes); smaller batches (a single slot) finish sooner
  // with one thread per resource element.
  constexpr int64_t kScMinThreads = 256 * 4 * 64;
  if (ranphy::mmse_sc_eligible(g) && (int64_t)g.n_slots * g.n_sc >= kScMinThreads)
    return ranphy::status_of(ranphy::launch_mmse_sc(g, rx2, h2, h_res, noise_var, x2, nv, s));
  return ranphy::status_of(ranphy::launch_mmse_re(g, rx2, h2, h_res, noise_var, x2, nv, s));
}

int ranphy_mmse_detect(const ranphy_slot_desc* d, const float* rx, const float* h, int h_res,
                       const float* noise_var, float* x, float* nv, void* stream) {
  return ranphy_mmse_detect_prec(d, rx, h, h_res, noise_var, x, nv, RANPHY_PREC_FP32, stream);
}

int ranphy_mmse_llr(const ranphy_slot_desc* d, const float* rx, const float* h, int h_res,
                    const float* noise_var, float* x, float* nv, float* llr, int precision,
                    void* stream) {
  Geom g;
  const int rc = ranphy::make_geom(d, &g);
  if (rc) return rc;
  if (h_res != RANPHY_H_PILOT && h_res != RANPHY_H_FULL) return RANPHY_ERR_INVALID;
  if (!ranphy::precision_valid(precision)) return RANPHY_ERR_INVALID;
  if (g.n_slots == 0) return RANPHY_OK;
  if ((x == nullptr) != (nv == nullptr)) return RANPHY_ERR_INVALID;
  if (!ranphy::aligned8(rx) || !ranphy::aligned8(h) || !ranphy::aligned8(llr) ||
      (x != nullptr && (!ranphy::aligned8(x) || !ranphy::aligned8(nv))) ||
      noise_var == nullptr || ((uintptr_t)noise_var & 3u))
    return RANPHY_ERR_INVALID;
  if (!ranphy::mmse_mfma_eligible(g, rx, h, x, nv, llr)) return RANPHY_ERR_UNSUPPORTED;
  return ranphy::status_of(ranphy::launch_mmse_mfma(
      g, reinterpret_cast<const float2*>(rx), false, reinterpret_cast<const float2*>(h), nullptr,
      h_res, noise_var, reinterpret_cast<float2*>(x), nv, llr, precision,
      static_cast<hipStream_t>(stream)));
}

int ranphy_mmse_llr_bfp(const ranphy_slot_desc* d, const uint32_t* packed, const float* h,
                        int h_res, const float* noise_var, float* x, float* nv, float* llr,
                        int precision, void* stream) {
  Geom g;
  const int rc = ranphy::make_geom(d, &g);
  if (rc) return rc;
  if (h_res != RANPHY_H_PILOT && h_res != RANPHY_H_FULL) return RANPHY_ERR_INVALID;
  if (!ranphy::precision_valid(precision)) return RANPHY_ERR_INVALID;
  if (g.n_slots == 0) return RANPHY_OK;
  if ((x == nullptr) != (nv == nullptr)) return RANPHY_ERR_INVALID;
  if (!ranphy::aligned8(packed) || !ranphy::aligned8(h) || !ranphy::aligned8(llr) ||
      (x != nullptr && (!ranphy::aligned8(x) || !ranphy::aligned8(nv))) ||
      noise_var == nullptr || ((uintptr_t)noise_var & 3u))
    return RANPHY_ERR_INVALID;
  // the matrix-core shapes (n_rx a multiple of 16: 16-antenna blocks); the words need only
  // 8-byte alignment
  if (!ranphy::mmse_mfma_eligible(g, nullptr, h, x, nv, llr)) return RANPHY_ERR_UNSUPPORTED;
  return ranphy::status_of(ranphy::launch_mmse_mfma(
      g, reinterpret_cast<const float2*>(packed), true, reinterpret_cast<const float2*>(h),
      nullptr, h_res, noise_var, reinterpret_cast<float2*>(x), nv, llr, precision,
      static_cast<hipStream_t>(stream)));
}

int ranphy_llr_demap(const ranphy_slot_desc* d, const float* x, const float* nv, float* llr,
                     void* stream) {
  Geom g;
  const int rc = ranphy::make_geom(d, &g);
  if (rc) return rc;
  if (g.n_slots == 0) return RANPHY_OK;
  if (!ranphy::aligned8(x) || !ranphy::aligned8(nv) || !ranphy::aligned8(llr))
    return RANPHY_ERR_INVALID;
  return ranphy::status_of(ranphy::launch_llr_demap(g, reinterpret_cast<const float2*>(x), nv,
                                                    llr, static_cast<hipStream_t>(stream)));
}

int64_t ranphy_cnn_param_count(void) { return ranphy::cnn_param_count(); }

int64_t ranphy_cnn_workspace_bytes(int rows, int cols, int n_img, int n_groups, int train) {
  if (rows < 1 || cols < 1 || n_img < 1 || n_groups < 0) return RANPHY_ERR_INVALID;
  return ranphy::cnn_workspace_bytes(rows, cols, n_img, n_groups, train != 0);
}

static int cnn_check(int rows, int cols, int n_img, int n_groups, const void* ws,
                     int64_t ws_bytes, int train) {
  if (rows < 1 || cols < 1 || n_img < 1 || n_groups < 0) return RANPHY_ERR_INVALID;
  if ((int64_t)rows * cols > (1 << 20) || n_img > (1 << 20) ||
      (int64_t)rows * cols * n_img > (1 << 30))
    return RANPHY_ERR_UNSUPPORTED;
  if (ws == nullptr || ((uintptr_t)ws & 255u) ||
      ws_bytes < ranphy::cnn_workspace_bytes(rows, cols, n_img, n_groups, train != 0))
    return RANPHY_ERR_INVALID;
  return RANPHY_OK;
}

static bool aligned4(const void* p) { return p != nullptr && ((uintptr_t)p & 3u) == 0; }

int ranphy_cnn_forward(const float* params, const float* x, const float* noise_var,
                       float min_noise_var, float* out, int rows, int cols, int n_img,
                       int n_groups, void* workspace, int64_t workspace_bytes, void* stream) {
  const int rc = cnn_check(rows, cols, n_img, n_groups, workspace, workspace_bytes, 0);
  if (rc) return rc;
  if (n_groups == 0) return RANPHY_OK;
  if (!aligned4(params) || !ranphy::aligned8(x) || !ranphy::aligned8(out) ||
      (noise_var != nullptr && !aligned4(noise_var)) || !(min_noise_var >= 0.f))
    return RANPHY_ERR_INVALID;
  return ranphy::status_of(ranphy::cnn_forward(rows, cols, n_img, n_groups, params, x, out,
                                               workspace, static_cast<hipStream_t>(stream),
                                               noise_var, min_noise_var));
}

int ranphy_cnn_grad(const float* params, const float* x, const float* target,
                    const float* noise_var, float* grad, float* loss, int rows, int cols,
                    int n_img, int n_groups, void* workspace, int64_t workspace_bytes,
                    void* stream) {
  const int rc = cnn_check(rows, cols, n_img, n_groups, workspace, workspace_bytes, 1);
  if (rc) return rc;
  if (n_groups < 1) return RANPHY_ERR_INVALID;
  if (!aligned4(params) || !ranphy::aligned8(x) || !ranphy::aligned8(target) ||
      !aligned4(grad) || !aligned4(loss) || (noise_var != nullptr && !aligned4(noise_var)))
    return RANPHY_ERR_INVALID;
  return ranphy::status_of(ranphy::cnn_grad(rows, cols, n_img, n_groups, params, x, target,
                                            noise_var, grad, loss, workspace,
                                            static_cast<hipStream_t>(stream)));
}

int ranphy_cnn_adam(float* params, const float* grad, float* m, float* v, int step, float lr,
                    void* stream) {
  if (!aligned4(params) || !aligned4(grad) || !aligned4(m) || !aligned4(v) || step < 1 ||
      !(lr > 0.f))
    return RANPHY_ERR_INVALID;
  return ranphy::status_of(
      ranphy::cnn_adam(params, grad, m, v, step, lr, static_cast<hipStream_t>(stream)));
}

}  // extern "C"

// The refinement of a pilot-resolution estimate over a caller's or the library's workspace:
// as many slots per pass as `workspace_bytes` holds (one slot at least, else
// RANPHY_ERR_UNSUPPORTED).  Arguments are validated by the callers.
static int denoise_passes(const Geom& g, const float* params, const float* noise_var,
                          float min_noise_var, const float* h_in, float* h_out, void* workspace,
                          int64_t workspace_bytes, hipStream_t s) {
  const int rows = g.n_occ, cols = g.n_pilot, nimg = g.n_rx * g.n_layers;
  int chunk = 0;
  for (int c = g.n_slots; c >= 1; c = c / 2) {
    if (ranphy::cnn_workspace_bytes(rows, cols, nimg, c, false) <= workspace_bytes) {
      chunk = c;
      break;
    }
  }
  if (chunk == 0) return RANPHY_ERR_UNSUPPORTED;
  const int64_t per_slot = (int64_t)rows * cols * nimg * 2;  // floats
  for (int s0 = 0; s0 < g.n_slots; s0 += chunk) {
    const int n = g.n_slots - s0 < chunk ? g.n_slots - s0 : chunk;
    const hipError_t e = ranphy::cnn_forward(
        rows, cols, nimg, n, params, h_in + s0 * per_slot, h_out + s0 * per_slot, workspace, s,
        noise_var != nullptr ? noise_var + s0 : nullptr, min_noise_var);
    if (e != hipSuccess) return RANPHY_ERR_LAUNCH;
  }
  return RANPHY_OK;
}

static int denoise_check(const Geom& g, const float* params, const float* noise_var,
                         float min_noise_var, const float* h_in, const float* h_out) {
  if (!aligned4(params) || !ranphy::aligned8(h_in) || !ranphy::aligned8(h_out) ||
      (noise_var != nullptr && !aligned4(noise_var)) || !(min_noise_var >= 0.f))
    return RANPHY_ERR_INVALID;
  return RANPHY_OK;
}

// ---- the library's own workspace for ranphy_cnn_denoise_noalloc --------------------------
// One array per GPU, in device memory for the life of the process.  Host code never uses the
// array's name as an address (on the host it names a stand-in): the device address comes
// from hipGetSymbolAddress, looked up once per device with that device current.
static __device__ __align__(256) unsigned char scratch[RANPHY_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_dev[kMaxDevices];  // device address of `scratch` per device, once looked up

// Device address of `scratch` on the device of stream s (the current device for the null
// stream).  0 on success, else a RANPHY error.
int scratch_for(hipStream_t s, void** out) {
  int cur = -1, dev = -1;
  if (hipGetDevice(&cur) != hipSuccess) return RANPHY_ERR_LAUNCH;
  dev = cur;
  if (s != nullptr && hipStreamGetDevice(s, &dev) != hipSuccess) return RANPHY_ERR_INVALID;
  if (dev < 0 || dev >= kMaxDevices) return RANPHY_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_dev[dev] == nullptr) {
    if (dev != cur && hipSetDevice(dev) != hipSuccess) return RANPHY_ERR_LAUNCH;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (dev != cur) (void)hipSetDevice(cur);
    if (e != hipSuccess || p == nullptr) return RANPHY_ERR_LAUNCH;
    scratch_dev[dev] = p;
  }
  *out = scratch_dev[dev];
  return RANPHY_OK;
}
}  // namespace

extern "C" {

int ranphy_cnn_denoise(const ranphy_slot_desc* d, const float* params, const float* noise_var,
                       float min_noise_var, const float* h_in, float* h_out, void* workspace,
                       int64_t workspace_bytes, void* stream) {
  Geom g;
  const int rc = ranphy::make_geom(d, &g);
  if (rc) return rc;
  if (g.n_slots == 0) return RANPHY_OK;
  if (workspace == nullptr || ((uintptr_t)workspace & 255u)) return RANPHY_ERR_INVALID;
  const int rc2 = denoise_check(g, params, noise_var, min_noise_var, h_in, h_out);
  if (rc2) return rc2;
  const int rc3 = denoise_passes(g, params, noise_var, min_noise_var, h_in, h_out, workspace,
                                 workspace_bytes, static_cast<hipStream_t>(stream));
  // a workspace too small for one slot is the caller's argument error here
  return rc3 == RANPHY_ERR_UNSUPPORTED ? RANPHY_ERR_INVALID : rc3;
}

int ranphy_cnn_denoise_noalloc(const ranphy_slot_desc* d, const float* params,
                               const float* noise_var, float min_noise_var, const float* h_in,
                               float* h_out, void* stream) {
  Geom g;
  const int rc = ranphy::make_geom(d, &g);
  if (rc) return rc;
  if (g.n_slots == 0) return RANPHY_OK;
  const int rc2 = denoise_check(g, params, noise_var, min_noise_var, h_in, h_out);
  if (rc2) return rc2;
  // one slot must fit the array; checked before anything touches the GPU
  if (ranphy::cnn_workspace_bytes(g.n_occ, g.n_pilot, g.n_rx * g.n_layers, 1, false) >
      RANPHY_NOALLOC_SCRATCH_BYTES)
    return RANPHY_ERR_UNSUPPORTED;
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* ws = nullptr;
  const int rc3 = scratch_for(s, &ws);
  if (rc3) return rc3;
  return denoise_passes(g, params, noise_var, min_noise_var, h_in, h_out, ws,
                        RANPHY_NOALLOC_SCRATCH_BYTES, s);
}

// ---- the whole chain in one launch (up to 8 layers) ----------------------------------------

// More than 8 layers: the matrix-core detector, estimating its pilot rows itself.
static int receive_mfma(const Geom& g, const void* rx, bool bfp, const float* pilots,
                        const float* noise_var, float* llr, void* stream) {
  if (!ranphy::mmse_mfma_eligible(g, bfp ? nullptr : rx, nullptr, nullptr, nullptr, llr))
    return RANPHY_ERR_UNSUPPORTED;
  return ranphy::status_of(ranphy::launch_mmse_mfma(
      g, reinterpret_cast<const float2*>(rx), bfp, nullptr,
      reinterpret_cast<const float2*>(pilots), RANPHY_H_PILOT, noise_var, nullptr, nullptr, llr,
      RANPHY_PREC_FP32, static_cast<hipStream_t>(stream)));
}

int ranphy_receive(const ranphy_slot_desc* d, const float* rx, const float* pilots,
                   const float* noise_var, float* llr, void* stream) {
  Geom g;
  const int rc = ranphy::make_geom(d, &g);
  if (rc) return rc;
  if (g.n_slots == 0) return RANPHY_OK;
  if (!ranphy::aligned8(rx) || !ranphy::aligned8(pilots) || !ranphy::aligned8(llr) ||
      noise_var == nullptr || ((uintptr_t)noise_var & 3u))
    return RANPHY_ERR_INVALID;
  if (g.n_layers > ranphy::kBatchMaxLayers)
    return receive_mfma(g, rx, false, pilots, noise_var, llr, stream);
  const int nk = ranphy::receive_tile(g, 256);
  if (nk < 1) return RANPHY_ERR_UNSUPPORTED;
  return ranphy::status_of(ranphy::launch_receive(
      g, reinterpret_cast<const float2*>(rx), false, reinterpret_cast<const float2*>(pilots),
      noise_var, llr, nk, static_cast<hipStream_t>(stream)));
}

int ranphy_receive_bfp(const ranphy_slot_desc* d, const uint32_t* packed, const float* pilots,
                       const float* noise_var, float* llr, void* stream) {
  Geom g;
  const int rc = ranphy::make_geom(d, &g);
  if (rc) return rc;
  if (ranphy::bfp_block(g.n_rx) == 0) return RANPHY_ERR_UNSUPPORTED;
  if (g.n_slots == 0) return RANPHY_OK;
  if (packed == nullptr || ((uintptr_t)packed & 3u) || !ranphy::aligned8(pilots) ||
      !ranphy::aligned8(llr) || noise_var == nullptr || ((uintptr_t)noise_var & 3u))
    return RANPHY_ERR_INVALID;
  if (g.n_layers > ranphy::kBatchMaxLayers) {  // the detector's words are read 8 bytes at a time
    if ((uintptr_t)packed & 7u) return RANPHY_ERR_INVALID;
    return receive_mfma(g, packed, true, pilots, noise_var, llr, stream);
  }
  const int nk = ranphy::receive_tile(g, 256);
  if (nk < 1) return RANPHY_ERR_UNSUPPORTED;
  return ranphy::status_of(ranphy::launch_receive(
      g, reinterpret_cast<const float2*>(packed), true, reinterpret_cast<const float2*>(pilots),
      noise_var, llr, nk, static_cast<hipStream_t>(stream)));
}

// ---- block floating point compression of the received grid --------------------------------

namespace {
// Blocks of the received grid of `g` (one per resource element and antenna group), or a
// negative status when the antenna count has no block width.
int64_t bfp_blocks(const Geom& g, int* b) {
  *b = ranphy::bfp_block(g.n_rx);
  if (*b == 0) return RANPHY_ERR_UNSUPPORTED;
  return (int64_t)g.n_slots * g.n_symb * g.n_sc * (g.n_rx / *b);
}
}  // namespace

int64_t ranphy_bfp_words(const ranphy_slot_desc* d) {
  Geom g;
  const int rc = ranphy::make_geom(d, &g);
  if (rc) return rc;
  int b;
  const int64_t n = bfp_blocks(g, &b);
  return n < 0 ? n : n * ranphy::bfp_words_per_block(b);
}

int ranphy_bfp_compress(const ranphy_slot_desc* d, const float* rx, uint32_t* packed,
                        void* stream) {
  Geom g;
  const int rc = ranphy::make_geom(d, &g);
  if (rc) return rc;
  int b;
  const int64_t n = bfp_blocks(g, &b);
  if (n < 0) return (int)n;
  if (n == 0) return RANPHY_OK;
  if (!ranphy::aligned8(rx) || packed == nullptr || ((uintptr_t)packed & 3u))
    return RANPHY_ERR_INVALID;
  return ranphy::status_of(
      ranphy::launch_bfp_compress(b, n, rx, packed, static_cast<hipStream_t>(stream)));
}

int ranphy_bfp_decompress(const ranphy_slot_desc* d, const uint32_t* packed, float* rx,
                          void* stream) {
  Geom g;
  const int rc = ranphy::make_geom(d, &g);
  if (rc) return rc;
  int b;
  const int64_t n = bfp_blocks(g, &b);
  if (n < 0) return (int)n;
  if (n == 0) return RANPHY_OK;
  if (!ranphy::aligned8(rx) || packed == nullptr || ((uintptr_t)packed & 3u))
    return RANPHY_ERR_INVALID;
  return ranphy::status_of(
      ranphy::launch_bfp_decompress(b, n, packed, rx, static_cast<hipStream_t>(stream)));
}

// ---- many UEs in one persistent launch ----------------------------------------------------

static int batch_build(const ranphy_ue* ues, int n_ue, int tile_re, std::vector<char>* out) {
  if (ues == nullptr || n_ue < 1 || tile_re < 1) return RANPHY_ERR_INVALID;
  std::vector<ranphy::BatchUe> recs(n_ue);
  std::vector<ranphy::BatchItem> items;
  for (int u = 0; u < n_ue; ++u) {
    const ranphy_ue& e = ues[u];
    if (e.desc.n_slots != 1) return RANPHY_ERR_INVALID;
    Geom g;
    const int rc = ranphy::make_geom(&e.desc, &g);
    if (rc) return rc;
    if (g.n_layers > ranphy::kBatchMaxLayers) return RANPHY_ERR_UNSUPPORTED;
    if (!ranphy::aligned8(e.rx) || !ranphy::aligned8(e.pilots) || !ranphy::aligned8(e.llr) ||
        e.noise_var == nullptr || ((uintptr_t)e.noise_var & 3u))
      return RANPHY_ERR_INVALID;
    recs[u].g = g;
    recs[u].rx = reinterpret_cast<const float2*>(e.rx);
    recs[u].pil = reinterpret_cast<const float2*>(e.pilots);
    recs[u].nv = e.noise_var;
    recs[u].llr = e.llr;
    // tiles of about tile_re resource elements whose pilot estimates fit the block's LDS
    const int per = ranphy::batch_row_stride(g.n_rx, g.n_layers);
    int want = std::max(1, tile_re / g.n_dsym);
    if (g.n_occ == 1) want = std::min(want, ranphy::kBatchFactSc);
    for (int k0 = 0; k0 < g.n_sc;) {
      // the widest tile up to want whose staged data fit, by the shape's path (pair,
      // filter, or pilot rows only); decided per shape, so the arithmetic of a resource
      // element does not depend on tile_re
      using Cap = ranphy::TileCap<8, 3>;
      const bool pair = g.n_occ == 2 && ranphy::batch_pair_path(g, Cap::rows, Cap::fac);
      const bool wpath = g.n_occ == 1 && ranphy::batch_w_path(g, Cap::rows);
      int nk = std::min(want, g.n_sc - k0);
      for (; nk >= 1; --nk) {
        const int rows = ranphy::batch_tile_rows(g, k0, nk);
        if (pair ? ranphy::batch_pair_fits(g, rows, nk, Cap::rows, Cap::fac)
                 : (wpath ? ranphy::batch_w_fits(g, rows, nk, Cap::rows) : rows * per <= Cap::rows))
          break;
      }
      if (nk < 1) return RANPHY_ERR_UNSUPPORTED;
      // class: layers, modulation, antennas
      items.push_back({u, k0, nk, (g.n_layers * 16 + g.qm) * 128 + g.n_rx});
      k0 += nk;
    }
  }
  // heaviest classes first (Gram work per RE ~ Nr Nl (Nl + 1) / 2), one class's items adjacent
  auto cost = [&](const ranphy::BatchItem& it) {
    const Geom& g = recs[it.ue].g;
    return (int64_t)g.n_rx * g.n_layers * (g.n_layers + 1) / 2;
  };
  std::stable_sort(items.begin(), items.end(), [&](const ranphy::BatchItem& a,
                                                   const ranphy::BatchItem& b) {
    const int64_t ca = cost(a), cb = cost(b);
    if (ca != cb) return ca > cb;
    return a.cls < b.cls;
  });
  ranphy::BatchHdr hdr{};
  hdr.head = 0;
  hdr.n_items = (int)items.size();
  hdr.n_ue = n_ue;
  const int64_t ue_bytes = (int64_t)sizeof(ranphy::BatchUe) * n_ue;
  hdr.items_off = (int)((ranphy::kBatchUeOff + ue_bytes + 255) & ~int64_t(255));
  out->assign((size_t)hdr.items_off + sizeof(ranphy::BatchItem) * items.size(), 0);
  std::memcpy(out->data(), &hdr, sizeof(hdr));
  std::memcpy(out->data() + ranphy::kBatchUeOff, recs.data(), (size_t)ue_bytes);
  std::memcpy(out->data() + hdr.items_off, items.data(), sizeof(ranphy::BatchItem) * items.size());
  return RANPHY_OK;
}

int64_t ranphy_batch_plan_bytes(const ranphy_ue* ues, int n_ue, int tile_re) {
  std::vector<char> buf;
  const int rc = batch_build(ues, n_ue, tile_re, &buf);
  return rc ? rc : (int64_t)buf.size();
}

int ranphy_batch_plan(const ranphy_ue* ues, int n_ue, int tile_re, void* plan,
                      int64_t plan_bytes) {
  std::vector<char> buf;
  const int rc = batch_build(ues, n_ue, tile_re, &buf);
  if (rc) return rc;
  if (plan == nullptr || ((uintptr_t)plan & 255u) || plan_bytes < (int64_t)buf.size())
    return RANPHY_ERR_INVALID;
  return ranphy::status_of(hipMemcpy(plan, buf.data(), buf.size(), hipMemcpyHostToDevice));
}

int ranphy_batch_run(void* plan, int n_blocks, void* stream) {
  if (plan == nullptr || ((uintptr_t)plan & 255u) || n_blocks < 1) return RANPHY_ERR_INVALID;
  return ranphy::status_of(ranphy::launch_batch(plan, n_blocks, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
