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

// Pilot rows (occasions x pilot indices) a tile of nk subcarriers starting at k0 reads.
int batch_tile_rows(const Geom& g, int k0, int nk);
hipError_t launch_batch(void* plan, int blocks, hipStream_t s);
// The one-launch chain for slots of one shape (ranphy_receive): tile width (0 if none fits).
int receive_tile(const Geom& g, int tile_re);
hipError_t launch_receive(const Geom& g, const float2* rx, const float2* pil, const float* nvar,
                          float* llr, int nk, hipStream_t s);

}  // namespace ranphy
