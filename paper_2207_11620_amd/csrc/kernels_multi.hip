// Batched queries of many independent neural volumes in one persistent
// launch.
//
// The models of a group share the MLP shape (precision, padded input width,
// width, depth) and the feature count, so one kernel instantiation serves
// them all; they differ in levels, resolutions and table sizes, which are
// read from a device table of model descriptors.  Work is cut into items of
// `chunk_tiles` 16-sample tiles of one model, ordered model by model; the
// workgroups take the next item from a device counter, so all of them work
// within one window of consecutive items and the GPU evaluates the models
// one after another (one model's tables in the caches at a time, no launch
// gaps between models; workgroups that took items grid-stride drifted apart
// by several models and shared the L2 among them), and each workgroup
// restages a model's MLP weights in LDS when it reaches that model's items.
#include <type_traits>

#include "kernels.hpp"
#include "mlp_tile.hpp"

namespace ngvol {

template <int P, int F, int KIN, int W, typename TT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P != 0 && KIN == 32 ? 4 : 1)))
k_multi_infer(const ModelDesc* __restrict__ table, MultiArgs a, uint32_t* __restrict__ next_item) {
  typedef typename Prec<P>::Frag Frag;
  typedef typename Prec<P>::T T;
  typedef WeightLayout<P, KIN, W> WL;
  extern __shared__ __align__(16) unsigned char smem[];
  Frag* lds_frag = reinterpret_cast<Frag*>(smem);
  const int nh = table[0].n_hidden;  // shared by the group
  const size_t wbytes = (size_t)WL::frags(nh, false) * 64 * sizeof(Frag);
  float* lds_wout = reinterpret_cast<float*>(smem + wbytes);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  T* stage = reinterpret_cast<T*>(smem + stage_offset<P, W>(wbytes) + wave * Stage<P, KIN>::wave_bytes);
  T* row = stage + lane * Stage<P, KIN>::pitch;

  // items are taken in order from the counter (zeroed before the launch);
  // a workgroup leaves at the first number past the last item, so every
  // workgroup ends.  The number is passed through LDS, alternating between
  // two slots: a slot is written again only after the next barrier, which
  // every wave reaches after reading it.
  __shared__ uint32_t taken[2];
  const int64_t total = a.item_prefix[a.k];
  int cur = -1;
  int m = 0;
  for (int it = 0;; ++it) {
    if (threadIdx.x == 0) taken[it & 1] = atomicAdd(next_item, 1u);
    __syncthreads();
    const int64_t item = (int64_t)taken[it & 1];
    if (item >= total) break;  // uniform over the workgroup
    while (item >= a.item_prefix[m + 1]) ++m;
    // the model index is uniform across the workgroup: say so, so that its
    // descriptor is read through the scalar cache
    m = __builtin_amdgcn_readfirstlane(m);
    if (m != cur) {
      __syncthreads();
      stage_weights<P, KIN, W>(table[m], a.params[m] + table[m].n_table, lds_frag, lds_wout, false);
      __syncthreads();
      cur = m;
    }
    const ModelDesc& md = table[m];
    const TT* tab;
    if constexpr (std::is_same<TT, __half>::value) tab = a.f16[m];
    else tab = a.params[m];
    const float* xyz = a.xyz[m];
    float* out = a.out[m];
    const int64_t n = a.n[m];
    const int64_t n_groups = (n + 63) >> 6;
    // an item is chunk_tiles 16-sample tiles, i.e. chunk_tiles / 4 wave groups
    const int64_t gpi = a.chunk_tiles >> 2;
    const int64_t first = (item - a.item_prefix[m]) * gpi;
    for (int j = wave; j < gpi; j += wpb) {
      const int64_t t = first + j;
      if (t >= n_groups) break;
      const int64_t s = t * 64 + lane;
      const bool valid = s < n;
      const int64_t sc = valid ? s : n - 1;
      const float x = clamp01(xyz[3 * sc]), y = clamp01(xyz[3 * sc + 1]), z = clamp01(xyz[3 * sc + 2]);
      encode_row<P, F, KIN>(md, tab, x, y, z, row, [](int, const Oct<P>&) {});
      wave_sync();
      const float yo = mlp_wave64<P, KIN, W>(nh, md.out_relu != 0, lds_frag, lds_wout, stage);
      wave_sync();
      if (valid) out[s] = yo;
    }
  }
}

__global__ void k_multi_reset(uint32_t* next_item) {
  if (threadIdx.x == 0) *next_item = 0u;
}

hipError_t launch_multi_infer(const ngvol_plan* plan0, const ModelDesc* table, const MultiArgs& a, bool f16,
                              int blocks_per_cu, uint32_t* next_item, hipStream_t st) {
  const ModelDesc& md = plan0->md;
  // a kernel, not a memset, so that the call can be captured in a graph
  hipLaunchKernelGGL(k_multi_reset, dim3(1), dim3(64), 0, st, next_item);
  const size_t lds = enc_lds_bytes(plan0, 4);
  int64_t grid = a.item_prefix[a.k];
  const int64_t cap = (int64_t)plan0->cus * blocks_per_cu;
  if (grid > cap) grid = cap;
  if (grid < 1) grid = 1;
#define NGV_MI(P, KIN, W)                                                                                      \
  do {                                                                                                         \
    if (f16)                                                                                                   \
      hipLaunchKernelGGL((k_multi_infer<P, 2, KIN, W, __half>), dim3((unsigned)grid), dim3(256), lds, st, table, a, \
                         next_item);                                                                           \
    else                                                                                                       \
      hipLaunchKernelGGL((k_multi_infer<P, 2, KIN, W, float>), dim3((unsigned)grid), dim3(256), lds, st, table, a,  \
                         next_item);                                                                           \
  } while (0)
#define NGV_MI_W(P, KIN)                                   \
  do {                                                     \
    if (md.width == 32) NGV_MI(P, KIN, 32);                \
    else if (md.width == 64) NGV_MI(P, KIN, 64);           \
    else return hipErrorInvalidValue;                      \
  } while (0)
#define NGV_MI_K(P)                                        \
  do {                                                     \
    if (plan0->kin == 32) NGV_MI_W(P, 32);                 \
    else if (plan0->kin == 64) NGV_MI_W(P, 64);            \
    else return hipErrorInvalidValue;                      \
  } while (0)
  if (md.F != 2) return hipErrorInvalidValue;
  switch (plan0->layout.precision) {
    case 0: NGV_MI_K(0); break;
    case 1: NGV_MI_K(1); break;
    case 2: NGV_MI_K(2); break;
    default: return hipErrorInvalidValue;
  }
#undef NGV_MI_K
#undef NGV_MI_W
#undef NGV_MI
  return hipGetLastError();
}

}  // namespace ngvol
