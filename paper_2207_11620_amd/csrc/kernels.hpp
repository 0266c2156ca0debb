// Internal interface between the C-ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "plan.hpp"

namespace ngvol {

// Table storage read by the encoding: FP16 copy if present, else FP32 master.
struct TablePtrs {
  const float* f32;
  const __half* f16;
};

template <typename TT>
__device__ __forceinline__ const TT* table_ptr(const TablePtrs& t);
template <>
__device__ __forceinline__ const float* table_ptr<float>(const TablePtrs& t) { return t.f32; }
template <>
__device__ __forceinline__ const __half* table_ptr<__half>(const TablePtrs& t) { return t.f16; }

// A training batch, resolved for the kernels.
// Macro-cell grid on the device: cells per axis, voxel dims, cell size.
struct McGeom {
  int32_t dims[3], m[3], cell;
  uint32_t* range;  // [cells][2] order-preserving keys (min, max), or NULL
  const float* mu;  // [cells], or NULL
};

// Order-preserving key of a binary32 value (unsigned compare = float compare).
__host__ __device__ inline uint32_t order_key(uint32_t bits) {
  return (bits & 0x80000000u) ? ~bits : (bits | 0x80000000u);
}

// Macro-cell of a point already clamped to [0,1]: floor(p * D) in binary32,
// divided by the cell size, capped at the last cell.
__device__ __forceinline__ uint32_t mc_index(const McGeom& g, float x, float y, float z) {
  const float p[3] = {x, y, z};
  uint32_t c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int v = (int)floorf(__fmul_rn(p[a], (float)g.dims[a]));
    const int ci = v / g.cell;
    c[a] = (uint32_t)(ci < g.m[a] - 1 ? ci : g.m[a] - 1);
  }
  return (c[2] * (uint32_t)g.m[1] + c[1]) * (uint32_t)g.m[0] + c[0];
}

// Extend cell c's range by value v (NaN ignored).  A plain read first skips
// the atomics whenever the range already covers v (ranges only widen, so a
// stale read can only cause an unneeded atomic).
__device__ __forceinline__ void mc_extend(uint32_t* range, uint32_t c, float v) {
  if (v != v) return;
  const uint32_t key = order_key(__float_as_uint(v));
  uint32_t* r = range + 2 * (size_t)c;
  if (key < __hip_atomic_load(r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(r, key);
  if (key > __hip_atomic_load(r + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(r + 1, key);
}

struct BatchArgs {
  int64_t B;
  const float* xyz;     // explicit coordinates, or NULL to generate
  const float* target;  // explicit targets
  const void* volume;   // ground truth for generated batches
  int32_t dims[3];
  int32_t vdtype;
  uint64_t seed;
  int64_t step;
  const int64_t* step_ptr;  // if set, the batch index is read from here (the state's draw or step counter)
  McGeom mc;                // mc.range set: the samples extend the macro-cell ranges
  __device__ __forceinline__ int64_t step_index() const { return step_ptr ? *step_ptr : step; }
};

// Spatial binning of n samples (k = 0: not binned).  Workspace byte offsets
// of the sorted coordinates, the per-sample auxiliary array (query
// permutation or training targets) and the histogram buffers.
struct BinPlan {
  int k, sb, n_bins, blocks;
  int64_t chunk;
  size_t rec_off, counts_off, totals_off, offsets_off, bytes;
  // level-split query (large query sets): feature planes and query slots
  bool split;
  size_t planes_off, idx_off;
};
BinPlan bin_plan(const ngvol_plan* plan, int64_t n);
// Sorts `xyz` (queries; aux = original index) or the batch `ba` (training;
// aux = target) into float4 records (x, y, z, aux) in the workspace.
hipError_t launch_bin(const ngvol_plan* plan, const BinPlan& bp, const float* xyz, const struct BatchArgs* ba,
                      int64_t n, void* ws, hipStream_t st);

// counts[blocks][nb] (per-block bucket counts) -> exclusive prefix over
// blocks in place; totals[nb] = bucket sizes; offsets[nb] = bucket starts.
hipError_t launch_count_offsets(uint32_t* counts, int blocks, int nb, uint32_t* totals, uint32_t* offsets,
                                hipStream_t st);

// Bucketed scatter of dL/dfeature into the table gradient (no global
// atomics except where one bucket is split over several workgroups).
struct ScatterPlan {
  int bshift, n_buckets, blocks, rec_words, max_items;
  int64_t chunk, n_records, chunk_records;
  size_t rec_off, counts_off, totals_off, offsets_off, items_off, bytes;
};
ScatterPlan scatter_plan(const ngvol_plan* plan, int64_t B);
// A non-finite gradient sum sets *nonfinite (the step is then skipped).
hipError_t launch_scatter(const ngvol_plan* plan, const ScatterPlan& sp, const struct BatchArgs& ba,
                          const float* dfeat, float* grad, void* ws, int32_t* nonfinite, hipStream_t st);

// Workspace carve-up of a training step (byte offsets).
struct TrainWorkspace {
  size_t e_off, g_off, de_off, partial_off, misc_off, scatter_off, total;
  int bwd_grid;
  ScatterPlan sc;
};

// Persistent tile schedule: waves of workgroups with the same id mod 8 (the
// XCD a workgroup is dispatched to) walk one contiguous eighth of the tiles,
// so that spatially sorted samples keep each XCD's L2 working set compact.
// Every tile is visited exactly once whatever the grid size.
struct TileIter {
  int64_t next, step, end;
  __device__ explicit TileIter(int64_t n_tiles) {
    const int wpb = blockDim.x >> 6, wave = threadIdx.x >> 6;
    const int G = gridDim.x;
    if (G >= 8) {
      const int x = blockIdx.x & 7, r = blockIdx.x >> 3;
      const int nbx = (G - x + 7) >> 3;
      const int64_t per = (n_tiles + 7) >> 3;
      const int64_t lo = (int64_t)x * per;
      end = lo + per < n_tiles ? lo + per : n_tiles;
      next = lo + (int64_t)r * wpb + wave;
      step = (int64_t)nbx * wpb;
    } else {
      next = (int64_t)blockIdx.x * wpb + wave;
      step = (int64_t)G * wpb;
      end = n_tiles;
    }
  }
};

// Level groups per XCD (level-split query): XCD x evaluates count[x] levels
// first[x], first[x]+8, ... for its part of the queries; width = levels of
// plane storage per group.
struct SplitArgs {
  int first[8], count[8];
  int part[8], parts[8];
  int width;
};
// Brick-staged level groups (2 levels of plane storage per query): the
// grouping's bins (Morton order, 2^k per axis) give each brick's records;
// pair p holds levels lev[p][0..1] (-1: none), lds_off[p][i] is the byte
// offset of level i's vertex box in LDS (-1: gathered from the table), and
// XCD x works on the (pair, brick) items [item_lo[x], item_lo[x+1]) of the
// pair-major list (item = pair * n_bins + brick).
struct BrickArgs {
  const uint32_t* bin_off;
  const uint32_t* bin_cnt;
  int k, n_bins;
  int lev[8][2];      // levels of list pair i (-1: none)
  int lds_off[8][2];  // LDS byte offsets of their staged boxes (-1: gathered)
  int n_shared;       // list pairs 0 .. n_shared-1: their bricks are shared by all XCDs
  int item_lo[9];     // XCD x: list items [item_lo[x], item_lo[x+1]) of the other pairs
  int gw;
};
bool use_split(const ngvol_plan* plan, int64_t n);
int64_t split_slab(const ngvol_plan* plan, int64_t n);
size_t split_planes_bytes(const ngvol_plan* plan, int64_t n);
// rec: grouped records (x, y, z, original index); planes/idx: workspace of
// split_planes_bytes and split_slab * 4 bytes.
// bin_off/bin_cnt (nullable): the grouping's per-bin record ranges over 2^bin_k
// bins per axis, for the brick-staged level kernel.
struct BinRanges {
  const uint32_t* off;
  const uint32_t* cnt;
  int k;
};
hipError_t launch_infer_split(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const float4* rec, int64_t n,
                              float* out, void* planes, uint32_t* idx, BinRanges bins, hipStream_t st);
template <int P, int W>
hipError_t launch_infer_split_p(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const float4* rec, int64_t n,
                                float* out, void* planes, uint32_t* idx, BinRanges bins, hipStream_t st);

// LDS of the staged forward weights: the fragments of W_0..W_{h-1}
// (mlp_weight_bytes), then W_out and its output-layer fragments (wout_bytes).
size_t mlp_weight_bytes(const ngvol_plan* plan);
size_t wout_bytes(const ngvol_plan* plan);
size_t fwd_lds_bytes(const ngvol_plan* plan);
// Persistent grid: enough workgroups of waves_per_block waves for n_tiles
// wave work units, at most blocks_per_cu per compute unit.
inline int grid_for(const ngvol_plan* plan, int64_t n_tiles, int waves_per_block, int blocks_per_cu) {
  int64_t need = (n_tiles + waves_per_block - 1) / waves_per_block;
  const int64_t cap = (int64_t)plan->cus * blocks_per_cu;
  if (need > cap) need = cap;
  if (need < 1) need = 1;
  return (int)need;
}
// LDS of a workgroup (160 KB on gfx950)
constexpr size_t kLdsLimit = 160 * 1024;
// fwd_lds_bytes plus the per-wave encoding stages of the fused kernels, and
// the waves per workgroup those kernels use
size_t enc_lds_bytes(const ngvol_plan* plan, int waves);
int enc_waves(const ngvol_plan* plan);
// MLP backward launch shape: waves per workgroup and where dW accumulates
// (LDS, or gdw: the workgroup's row of the partial-sum buffer).
struct BwdConfig {
  int waves;
  bool gdw;
};
size_t bwd_lds_bytes(const ngvol_plan* plan, int waves, bool gdw);
BwdConfig bwd_config(const ngvol_plan* plan);
int bwd_waves(const ngvol_plan* plan);
int bwd_grid(const ngvol_plan* plan, int64_t n);
TrainWorkspace train_workspace(const ngvol_plan* plan, int64_t B);

hipError_t launch_encode(const ngvol_plan* plan, TablePtrs tp, const float* xyz, int64_t n, float* feat,
                         hipStream_t st);
hipError_t launch_encode_debug(const ngvol_plan* plan, const float* xyz, int64_t n, uint32_t* idx, float* w,
                               hipStream_t st);
// Either xyz[n][3] in output order, or rec[n] sorted records whose .w holds
// the output slot: out[slot] = Phi(rec.xyz).
hipError_t launch_infer(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const float* xyz, const float4* rec,
                        int64_t n, float* out, hipStream_t st);
hipError_t launch_sq_error_grid(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const void* vol, int dtype,
                                const int32_t dims[3], double* sq, hipStream_t st);
hipError_t launch_mlp_fwd(const ngvol_plan* plan, const float* mlp, const void* feat, int dtype, int64_t n,
                          float* out, hipStream_t st);
hipError_t launch_train_fwd(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const BatchArgs& ba, void* e_buf,
                            float* g_buf, double* loss_acc, float gscale, int loss, hipStream_t st);
hipError_t launch_sample_batch(const BatchArgs& ba, float* xyz, float* y, hipStream_t st);
// The same launchers for one MLP precision P and width W (each defined in
// the object built for that shape).
template <int P, int W>
hipError_t launch_infer_p(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const float* xyz, const float4* rec,
                          int64_t n, float* out, hipStream_t st);
template <int P, int W>
hipError_t launch_sq_error_grid_p(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const void* vol, int dtype,
                                  const int32_t dims[3], double* sq, hipStream_t st);
template <int P, int W>
hipError_t launch_mlp_fwd_p(const ngvol_plan* plan, const float* mlp, const void* feat, int dtype, int64_t n,
                            float* out, hipStream_t st);
template <int P, int W>
hipError_t launch_train_fwd_p(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const BatchArgs& ba,
                              void* e_buf, float* g_buf, double* loss_acc, float gscale, int loss, hipStream_t st);

// Backward.  MODE 0: training (e_buf holds the stored encoding in the
// plan's precision, de is scattered into the table gradient; coordinates
// from ba).  MODE 1: standalone MLP backward on FP32 features, writing
// dfeat (nullable).  dW partial sums per block go to `partial`
// ([grid][n_mlp]); launch_reduce_partials adds them into grad.
hipError_t launch_bwd(const ngvol_plan* plan, int mode, const float* mlp, const void* e_buf, const float* g_buf,
                      const BatchArgs& ba, float* grad, float* dfeat, float* partial, int grid, int32_t* nonfinite,
                      float bscale, hipStream_t st);
hipError_t launch_reduce_partials(const ngvol_plan* plan, const float* partial, int grid, float* grad,
                                  int32_t* nonfinite, hipStream_t st);
hipError_t launch_encode_bwd(const ngvol_plan* plan, const float* xyz, int64_t n, const float* dfeat, float* grad,
                             hipStream_t st);

// Adam with bias correction; step k (0-based applied steps) uses
// lr * decay_base^floor((k - decay_start) / decay_interval) once k >= decay_start
// (decay_interval > 0), and l2_reg * w is added to the MLP weights' gradient.
struct AdamArgs {
  double lr, b1, b2, eps;
  double l2_reg;
  int64_t decay_start, decay_interval;
  double decay_base;
  float inv_scale;
};
hipError_t launch_adam(const ngvol_plan* plan, float* params, __half* table_f16, float* grad, float* m, float* v,
                       int64_t* step, const int32_t* nonfinite, const AdamArgs& a, hipStream_t st);
hipError_t launch_step_begin(double* loss_acc, int32_t* nonfinite, hipStream_t st);
hipError_t launch_step_end(const double* loss_acc, int32_t* nonfinite, int64_t* step, int64_t* draws,
                           int32_t* skipped, double* loss_out, double inv_b, hipStream_t st);
// *p = 0 (a kernel, so that graph capture records no memset node)
hipError_t launch_zero_f64(double* p, hipStream_t st);
// *mse = *mse * inv_n; *psnr = -10 log10(*mse) if psnr != NULL
hipError_t launch_psnr_finish(double* mse, double inv_n, double* psnr, hipStream_t st);
hipError_t launch_make_f16(const float* params, __half* out, int64_t n, hipStream_t st);

// Per-call arguments of a batched multi-model query (kernel arguments).
constexpr int kMultiMax = NGVOL_MULTI_MAX;
struct MultiArgs {
  int k;
  int chunk_tiles;
  int64_t item_prefix[kMultiMax + 1];  // work items of models 0..m-1
  const float* params[kMultiMax];
  const __half* f16[kMultiMax];
  const float* xyz[kMultiMax];
  float* out[kMultiMax];
  int64_t n[kMultiMax];
};
// next_item: the group's device work counter (zeroed by the launch).
hipError_t launch_multi_infer(const ngvol_plan* plan0, const ModelDesc* table, const MultiArgs& a, bool f16,
                              int blocks_per_cu, uint32_t* next_item, hipStream_t st);

}  // namespace ngvol
