// Host-side table packing (see pack.cpp).
#pragma once

#include <cstdint>
#include <vector>

#include "fk_internal.h"

namespace fk {

// One row group of a table: row flavour ``a`` (-1 for DIS) and the
// contraction index as segments of source rows (PDF row = flavour*nx + x).
struct GroupPlan {
  int a = -1;
  int K = 0, KE = 0;
  std::vector<int> seg_row, seg_len;
  size_t base = 0;  // unit offset of the group's packed FK in the table
};

// One datapoint chunk of the transposed DIS table.
struct TChunk {
  int i0 = 0, n = 0, KE = 0;
  size_t base = 0;  // unit offset in the transposed table
};

struct PackedTable {
  std::vector<GroupPlan> groups;   // forward row groups
  std::vector<GroupPlan> agroups;  // hadronic only: adjoint row groups (into fkT)
  std::vector<float> scale;   // s_i, powers of two
  std::vector<uint8_t> fk;    // packed forward units (16 bytes each)
  std::vector<uint8_t> fkT;   // DIS: transposed units; hadronic: full symmetric part
  std::vector<TChunk> tchunks;
  std::vector<int> active;    // DIS: active flavours
  int nact = 0, npairs = 0;
};

uint16_t round_bf16(double x);
uint8_t round_e4m3(double x);
double datapoint_scale(double absmax, double qmax);

void pack_dis(const double *fk, const uint8_t *mask, int N, int F, int X, int dtype, PackedTable &pt);
void pack_had(const double *fk, const uint8_t *mask, int N, int F, int X, int dtype, PackedTable &pt);

}  // namespace fk
