// Training forward (Section 4): sampling step or explicit batch, encoding
// (stored for the backward), MLP, loss and the output gradient.
// build: one object per MLP precision and width (NGV_PSEL, NGV_WSEL)
#include <type_traits>

#include "kernels.hpp"
#include "dispatch.hpp"
#include "mlp_tile.hpp"

namespace ngvol {

// ---------------------------------------------------------------------------
// Training forward: sampling step (or explicit batch), encoding (stored for
// the backward), MLP, loss, and g = S * dL/dy: gscale * (y_hat - y) for L2
// (gscale = 2S/B), gscale * sign(y_hat - y) for L1 (gscale = S/B).
// ---------------------------------------------------------------------------
template <int P, int F, int KIN, int W, typename TT, typename VT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P != 0 && KIN == 32 ? 4 : 1)))
k_train_fwd(ModelDesc md, TablePtrs tp, const float* __restrict__ mlp, BatchArgs ba, void* __restrict__ e_buf,
            float* __restrict__ g_buf, double* __restrict__ loss_acc, float gscale, int l1) {
  typedef typename Prec<P>::Frag Frag;
  typedef typename Prec<P>::T T;
  typedef WeightLayout<P, KIN, W> WL;
  extern __shared__ __align__(16) unsigned char smem[];
  Frag* lds_frag = reinterpret_cast<Frag*>(smem);
  const size_t wbytes = (size_t)WL::frags(md.n_hidden, false) * 64 * sizeof(Frag);
  float* lds_wout = reinterpret_cast<float*>(smem + wbytes);
  stage_weights<P, KIN, W>(md, mlp, lds_frag, lds_wout, false);
  __syncthreads();

  const TT* table = table_ptr<TT>(tp);
  const VT* vol = reinterpret_cast<const VT*>(ba.volume);
  T* e = reinterpret_cast<T*>(e_buf);  // stored encoding [B][KIN] in the operand type
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T* stage = reinterpret_cast<T*>(smem + stage_offset<P, W>(wbytes) + wave * Stage<P, KIN>::wave_bytes);
  T* row = stage + lane * Stage<P, KIN>::pitch;
  const int64_t B = ba.B;
  const int64_t bstep = ba.step_index();
  double lsum = 0.0;
  const int64_t n_groups = (B + 63) >> 6;
  TileIter it(n_groups);
  for (int64_t t = it.next; t < it.end; t += it.step) {
    const int64_t s = t * 64 + lane;
    const bool valid = s < B;
    const int64_t sc = valid ? s : B - 1;
    float x, y, z, target;
    if (ba.xyz) {
      x = clamp01(ba.xyz[3 * sc]);
      y = clamp01(ba.xyz[3 * sc + 1]);
      z = clamp01(ba.xyz[3 * sc + 2]);
      target = ba.target[sc];
    } else {
      x = batch_coord(ba.seed, bstep, B, sc, 0);
      y = batch_coord(ba.seed, bstep, B, sc, 1);
      z = batch_coord(ba.seed, bstep, B, sc, 2);
      target = volume_sample<VT>(vol, ba.dims[0], ba.dims[1], ba.dims[2], x, y, z);
    }
    encode_row<P, F, KIN>(md, table, x, y, z, row, [&](int sb, const Oct<P>& o) {
      if (valid) *reinterpret_cast<Oct<P>*>(e + s * KIN + 8 * sb) = o;
    });
    wave_sync();
    const float yv = mlp_wave64<P, KIN, W>(md.n_hidden, md.out_relu != 0, lds_frag, lds_wout, stage);
    wave_sync();
    if (valid && ba.mc.range) mc_extend(ba.mc.range, mc_index(ba.mc, x, y, z), target);
    if (valid) {
      const float r = yv - target;
      // with an output ReLU the gradient passes only where its input was
      // positive (ReLU'(0) = 0): there the output is positive too
      const bool pass = !md.out_relu || yv > 0.0f;
      if (l1) {
        g_buf[s] = pass ? (r > 0.0f ? gscale : (r < 0.0f ? -gscale : 0.0f)) : 0.0f;
        lsum += (double)fabsf(r);
      } else {
        g_buf[s] = pass ? gscale * r : 0.0f;
        lsum += (double)r * (double)r;
      }
    }
  }
  lsum = wave_sum(lsum);
  if (lane == 0 && lsum != 0.0) atomicAdd(loss_acc, lsum);
}

template <int P, int W>
hipError_t launch_train_fwd_p(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const BatchArgs& ba,
                              void* e_buf, float* g_buf, double* loss_acc, float gscale, int loss, hipStream_t st) {
  const ModelDesc& md = plan->md;
  const int l1 = loss == NGVOL_LOSS_L1;
  const int64_t n_groups = (ba.B + 63) / 64;  // 64 samples per wave
  const int waves = enc_waves(plan);
  const size_t lds = enc_lds_bytes(plan, waves);
  const int grid = grid_for(plan, n_groups, waves, 32 / waves);
  const bool vf16 = ba.xyz == nullptr && ba.vdtype == NGVOL_DT_F16;
  NGV_DISPATCH_F_KIN(md.F, plan->kin, {
    if (tp.f16) {
      if (vf16)
        hipLaunchKernelGGL((k_train_fwd<P, F, KIN, W, __half, __half>), dim3(grid), dim3(64 * waves), lds, st, md, tp, mlp, ba,
                           e_buf, g_buf, loss_acc, gscale, l1);
      else
        hipLaunchKernelGGL((k_train_fwd<P, F, KIN, W, __half, float>), dim3(grid), dim3(64 * waves), lds, st, md, tp, mlp, ba,
                           e_buf, g_buf, loss_acc, gscale, l1);
    } else {
      if (vf16)
        hipLaunchKernelGGL((k_train_fwd<P, F, KIN, W, float, __half>), dim3(grid), dim3(64 * waves), lds, st, md, tp, mlp, ba,
                           e_buf, g_buf, loss_acc, gscale, l1);
      else
        hipLaunchKernelGGL((k_train_fwd<P, F, KIN, W, float, float>), dim3(grid), dim3(64 * waves), lds, st, md, tp, mlp, ba,
                           e_buf, g_buf, loss_acc, gscale, l1);
    }
  });
  return hipGetLastError();
}

template hipError_t launch_train_fwd_p<NGV_PSEL, NGV_WSEL>(const ngvol_plan*, TablePtrs, const float*, const BatchArgs&, void*,
                                                 float*, double*, float, int, hipStream_t);

#if NGV_PRIMARY
hipError_t launch_train_fwd(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const BatchArgs& ba, void* e_buf,
                            float* g_buf, double* loss_acc, float gscale, int loss, hipStream_t st) {
  NGV_DISPATCH_P(plan->layout.precision,
                 NGV_DISPATCH_W(plan->md.width, return launch_train_fwd_p<P, W>(plan, tp, mlp, ba, e_buf, g_buf, loss_acc, gscale, loss, st)));
  return hipErrorInvalidValue;
}
#endif

}  // namespace ngvol
