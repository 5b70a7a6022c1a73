// Plan of the multi-UE persistent launch (batch.hip), shared by the host layer that builds it
// and the kernel that reads it.  Layout in device memory: BatchHdr at byte 0, the UE records
// from byte kBatchUeOff, the work items from byte hdr.items_off.
#pragma once

#include "geom.h"

namespace ranphy {

struct BatchUe {
  Geom g;  // one slot of this UE's allocation
  const float2* rx;
  const float2* pil;
  const float* nv;
  float* llr;
};

struct BatchItem {
  int ue, k0, nk, cls;  // subcarriers k0 .. k0 + nk - 1 of UE ue, all data symbols
};

struct BatchHdr {
  unsigned head;  // next item to take; cleared before every run
  int n_items;
  int n_ue;
  int items_off;
};

constexpr int kBatchLds = 4096;  // complex values of staged pilot estimates per block (32 KB)
// One DMRS occasion: the channel is held over the slot, so each subcarrier's Gram factor is
// formed once per tile and staged in LDS for the tile's resource elements.
constexpr int kBatchFactSc = 56;  // subcarriers per tile of a one-occasion UE
constexpr int kBatchFactNP = 36;  // lower-triangle entries of an 8 x 8 factor
constexpr int kBatchUeOff = 256;
constexpr int kBatchMaxLayers = 8;

// Complex values per staged pilot row (one pilot index of one occasion: Nr x Nl estimates),
// made odd so that rows of neighbouring pilots start in different LDS banks.
__host__ __device__ inline int batch_row_stride(int nr, int nl) { return (nr * nl) | 1; }
// Two DMRS occasions and at most 4 layers: per subcarrier the tile stages the channel pair
// (H0, H1 - H0) as float4 per antenna and layer after the pilot rows (from an even complex
// offset, so 16-byte aligned), padded by one float4 per subcarrier, and the three Gram pieces
// in the factor area (an odd count of complex values per subcarrier).
__host__ __device__ inline int batch_pair_stride(int nr, int nl) { return nr * nl + 1; }
__host__ __device__ inline int batch_gram_stride(int nl) { return (3 * nl * (nl + 1) / 2) | 1; }
__host__ __device__ inline int batch_pair_base(int rows, int rs) { return (rows * rs + 1) & ~1; }
// LDS capacities of a block serving up to MAXNL layers with BLOCKS blocks per CU: complex
// values of pilot rows and channel pairs (rows), complex values of factors or Gram pieces
// (fac), the factor and aux strides per subcarrier, and the subcarriers of a one-occasion
// tile (fsc).  A CU has 160 KB of LDS.
template <int MAXNL, int BLOCKS>
struct TileCap;
template <>
struct TileCap<8, 3> {
  static constexpr int rows = kBatchLds, fac = kBatchFactSc * kBatchFactNP, fnp = kBatchFactNP,
                       aux = 2 * 8 + 1, fsc = kBatchFactSc;
  static constexpr bool one_occ = false;
  // pilot estimates per thread whose loads are in flight together
  static constexpr int stage_batch = 4;
  // LLRs per element written as one record by lane groups (0: lane by lane).  The
  // multi-UE form keeps lane-by-lane stores: the record exchange's registers cost it more
  // (spills) than the scattered stores do (measured).
  static constexpr int store_floats = 0;
  static constexpr bool multi_occ = false;
  // received samples read by lane groups in whole 16-antenna lines (for_rx): the multi-UE
  // launch 0.65 -> 0.59 ms (its 64-antenna UEs read 4 lines per element)
  static constexpr bool line_loads = true;
};
template <>
struct TileCap<4, 4> {  // two-occasion tiles of 16 x 4 fit 21 subcarriers
  static constexpr int rows = 3776, fac = 1024, fnp = 10, aux = 2 * 4 + 1, fsc = kBatchFactSc;
  static constexpr bool one_occ = false;
  static constexpr int stage_batch = 4;
  static constexpr int store_floats = 32;  // whole 128-byte records of 4 layers x 256QAM
  static constexpr bool multi_occ = true;  // launched for two or more occasions only
  static constexpr bool line_loads = true;
};
template <>
struct TileCap<4, 5> {  // one-occasion tiles only
  static constexpr int rows = 2944, fac = 640, fnp = 10, aux = 2 * 4 + 1, fsc = kBatchFactSc;
  static constexpr bool one_occ = true;
  static constexpr int stage_batch = 1;  // within the 5-block register budget
  static constexpr int store_floats = 0;   // likewise (measured on the paper's 2x2 and 4x4)
  static constexpr bool multi_occ = false;
  static constexpr bool line_loads = false;  // its 96 registers: the group loads spill here
};

__host__ __device__ inline bool batch_pair_fits(const Geom& g, int rows, int nk, int cap_rows,
                                                int cap_fac) {
  if (g.n_occ != 2 || g.n_layers > 4) return false;
  const int base = batch_pair_base(rows, batch_row_stride(g.n_rx, g.n_layers));
  return base + 2 * nk * batch_pair_stride(g.n_rx, g.n_layers) <= cap_rows &&
         nk * batch_gram_stride(g.n_layers) <= cap_fac;
}
// One DMRS occasion: per subcarrier the tile may stage the unbiased filter W = diag(1/mu)
// G^-1 H^H (Nl x Nr complex, odd stride) after the pilot rows, so that a resource element
// needs only x = W y.  It fits when the rows and nk filters fit the rows area.
__host__ __device__ inline int batch_w_stride(int nr, int nl) { return (nr * nl) | 1; }
__host__ __device__ inline bool batch_w_fits(const Geom& g, int rows, int nk, int cap_rows) {
  if (g.n_occ != 1) return false;
  const int base = batch_pair_base(rows, batch_row_stride(g.n_rx, g.n_layers));
  return base + nk * batch_w_stride(g.n_rx, g.n_layers) <= cap_rows;
}
// Pilot rows any tile of nk consecutive subcarriers can span (every occasion, every port).
__host__ __device__ inline int batch_rows_bound(const Geom& g, int nk) {
  return g.n_occ * ((nk - 1) / g.comb + 4);
}
// Whether a shape takes the pair (two occasions) or the filter (one occasion) path: decided by
// the shape alone, so that the arithmetic of a resource element does not depend on the tile
// width; a shape qualifies when any tile of 8 subcarriers fits, and the host then picks tile
// widths that fit.
__host__ __device__ inline bool batch_pair_path(const Geom& g, int cap_rows, int cap_fac) {
  return batch_pair_fits(g, batch_rows_bound(g, 8), 8, cap_rows, cap_fac);
}
// The filter form pays where the per-element substitutions it removes are a large share of
// the work and its filters leave the tiles wide: 3..8 layers, at most 64 antenna-layer pairs
// (measured on the paper's square shapes and the multi-UE mix).
__host__ __device__ inline bool batch_w_path(const Geom& g, int cap_rows) {
  return g.n_layers >= 3 && g.n_rx * g.n_layers <= 64 &&
         batch_w_fits(g, batch_rows_bound(g, 8), 8, cap_rows);
}
// Pilot rows (occasions x pilot indices) a tile of nk subcarriers starting at k0 reads.
int batch_tile_rows(const Geom& g, int k0, int nk);
hipError_t launch_batch(void* plan, int blocks, hipStream_t s);
// The one-launch chain for slots of one shape (ranphy_receive): tile width (0 if none fits).
int receive_tile(const Geom& g, int tile_re);
// rx: the complex64 grid, or with bfp its block floating point words (ranphy_bfp_compress).
hipError_t launch_receive(const Geom& g, const float2* rx, bool bfp, const float2* pil,
                          const float* nvar, float* llr, int nk, hipStream_t s);

}  // namespace ranphy
