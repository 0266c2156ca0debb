// Plan: the resolved model description, shared by host code and kernels.
#pragma once

#include <stdint.h>

#include "ngvol.h"

namespace ngvol {

struct LevelDesc {
  int32_t N;        // vertices per axis
  uint32_t dense;   // 1 if N^3 <= T (row-major slots), else hashed
  uint32_t offset;  // first entry of this level in the concatenated tables
  uint32_t mask;    // T - 1 for hashed levels
};

// Passed to kernels by value (lives in the kernel-argument segment, read
// through the scalar cache).
struct ModelDesc {
  int32_t L, F, n_in, width, n_hidden, n_layers;
  int32_t out_relu;  // 1: ReLU on the output neuron
  int64_t n_table;  // table floats
  int64_t n_params;
  int32_t w_off[NGVOL_MAX_LAYERS];  // matrix offsets relative to the MLP block
  int32_t n_mlp;
  LevelDesc lv[NGVOL_MAX_LEVELS];
};

}  // namespace ngvol

struct ngvol_plan {
  ngvol_layout layout;
  ngvol::ModelDesc md;
  int kin;    // input width padded to a multiple of 32 (MFMA K blocks)
  int loss;   // NGVOL_LOSS_L2 | NGVOL_LOSS_L1 (training steps)
  int cus;    // compute units of the device the plan was created on
  int device;
};
