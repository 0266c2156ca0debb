// Forward kernels: encoding, fused query, standalone MLP, grid squared
// error, sampling step.
// build: one object per MLP precision and width (NGV_PSEL, NGV_WSEL)
#include <type_traits>

#include "kernels.hpp"
#include "dispatch.hpp"
#include "mlp_tile.hpp"

namespace ngvol {

// ---------------------------------------------------------------------------
// Standalone encoding: feat[n][n_in] FP32.
// ---------------------------------------------------------------------------
template <int F, int KIN, typename TT>
__global__ void __launch_bounds__(256) k_encode(ModelDesc md, TablePtrs tp, const float* __restrict__ xyz, int64_t n,
                                                float* __restrict__ feat) {
  // one sample per lane; all lanes on the same level at a time
  const TT* table = table_ptr<TT>(tp);
  const int lane = threadIdx.x & 63;
  const int64_t n_groups = (n + 63) >> 6;
  TileIter it(n_groups);
  for (int64_t t = it.next; t < it.end; t += it.step) {
    const int64_t s = t * 64 + lane;
    const bool valid = s < n;
    const int64_t sc = valid ? s : n - 1;
    const float x = clamp01(xyz[3 * sc]), y = clamp01(xyz[3 * sc + 1]), z = clamp01(xyz[3 * sc + 2]);
    for (int l = 0; l < md.L; ++l) {
      Corners cr;
      level_corners(md.lv[l], x, y, z, cr);
      float acc[F];
      gather_level<F>(cr, table, (uint32_t)(md.n_table / F), acc);
      if (valid) {
#pragma unroll
        for (int f = 0; f < F; ++f) feat[s * md.n_in + l * F + f] = acc[f];
      }
    }
  }
}

#if NGV_PRIMARY
// Corner slots and weights: one thread per (sample, level).
__global__ void __launch_bounds__(256) k_encode_debug(ModelDesc md, const float* __restrict__ xyz, int64_t n,
                                                      uint32_t* __restrict__ idx, float* __restrict__ w) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * md.L) return;
  const int64_t s = t / md.L;
  const int l = (int)(t % md.L);
  Corners cr;
  level_corners(md.lv[l], clamp01(xyz[3 * s]), clamp01(xyz[3 * s + 1]), clamp01(xyz[3 * s + 2]), cr);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (idx) idx[t * 8 + k] = cr.slot[k] - md.lv[l].offset;
    if (w) w[t * 8 + k] = cr.w[k];
  }
}
#endif

// ---------------------------------------------------------------------------
// Fused query.  MODE 0: out[s] = Phi(xyz[s]).  MODE 1: grid voxel centres,
// accumulate (Phi - volume)^2 in FP64.
// ---------------------------------------------------------------------------
template <int P, int F, int KIN, int W, typename TT, int MODE, typename VT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P != 0 && KIN == 32 ? 4 : 1)))
k_infer(ModelDesc md, TablePtrs tp, const float* __restrict__ mlp, const float* __restrict__ xyz,
        const float4* __restrict__ rec, int64_t n, float* __restrict__ out, const VT* __restrict__ vol, int dx, int dy,
        int dz, double* __restrict__ sq_sum) {
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
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T* stage = reinterpret_cast<T*>(smem + stage_offset<P, W>(wbytes) + wave * Stage<P, KIN>::wave_bytes);
  T* row = stage + lane * Stage<P, KIN>::pitch;
  double err = 0.0;
  const int64_t n_groups = (n + 63) >> 6;
  TileIter it(n_groups);
  for (int64_t t = it.next; t < it.end; t += it.step) {
    const int64_t s = t * 64 + lane;
    const bool valid = s < n;
    const int64_t sc = valid ? s : n - 1;
    float x, y, z;
    int64_t slot = s;
    if constexpr (MODE == 0) {
      if (rec) {
        const float4 r = rec[sc];
        x = clamp01(r.x);
        y = clamp01(r.y);
        z = clamp01(r.z);
        slot = (int64_t)__float_as_uint(r.w);
      } else {
        x = clamp01(xyz[3 * sc]);
        y = clamp01(xyz[3 * sc + 1]);
        z = clamp01(xyz[3 * sc + 2]);
      }
    } else {
      const int64_t ix = sc % dx, iy = (sc / dx) % dy, iz = sc / ((int64_t)dx * dy);
      x = ((float)ix + 0.5f) / (float)dx;
      y = ((float)iy + 0.5f) / (float)dy;
      z = ((float)iz + 0.5f) / (float)dz;
    }
    encode_row<P, F, KIN>(md, table, x, y, z, row, [](int, const Oct<P>&) {});
    wave_sync();
    const float yv = mlp_wave64<P, KIN, W>(md.n_hidden, md.out_relu != 0, lds_frag, lds_wout, stage);
    wave_sync();  // the stage is rewritten by the next group
    if (valid) {
      if constexpr (MODE == 0) {
        out[slot] = yv;
      } else {
        const double d = (double)yv - (double)load_vox<VT>(vol, (size_t)s);
        err += d * d;
      }
    }
  }
  if constexpr (MODE == 1) {
    err = wave_sum(err);
    if (lane == 0 && err != 0.0) atomicAdd(sq_sum, err);
  }
}

// ---------------------------------------------------------------------------
// Standalone MLP on given features ([n][n_in], FP32 or BF16).  DIRECT: the
// features are stored in the operand type with n_in = KIN, so a lane's
// operand block is one 16-byte load; otherwise they are converted element by
// element (zero beyond n_in).  The two loaders are separate instantiations,
// so the direct kernel carries none of the element-wise code.
// ---------------------------------------------------------------------------
template <int P, int KIN, int W, typename IT, int NHC, bool DIRECT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(mlp_waves_per_eu(P, KIN, NHC))))
k_mlp_fwd(ModelDesc md, const float* __restrict__ mlp,
                                                 const IT* __restrict__ feat, int64_t n, float* __restrict__ out) {
  // NB tiles (16 samples each) per wave and group: the weight fragments are
  // read once per group (with NHC = 2 hidden layers fixed at compile time
  // the kernel keeps all of them in registers), and the next group's
  // features are loaded while this one is evaluated.
  constexpr int NB = 2;
  constexpr int CH0 = InChunks<P, KIN>::n;
  typedef typename Prec<P>::Frag Frag;
  typedef WeightLayout<P, KIN, W> WL;
  extern __shared__ __align__(16) unsigned char smem[];
  Frag* lds_frag = reinterpret_cast<Frag*>(smem);
  float* lds_wout = reinterpret_cast<float*>(smem + (size_t)WL::frags(md.n_hidden, false) * 64 * sizeof(Frag));
  stage_weights<P, KIN, W>(md, mlp, lds_frag, lds_wout, false);
  __syncthreads();
  const int lane = threadIdx.x & 63, nl = lane & 15, g = lane >> 4;
  const int n_in = md.n_in;
  const int64_t n_groups = (n + 16 * NB - 1) / (16 * NB);
  TileIter it(n_groups);
  auto row = [&](int64_t grp, int nb) -> int64_t {
    const int64_t s = (grp * NB + nb) * 16 + nl;
    return s < n ? s : n - 1;
  };
  auto st = [&](int64_t grp, int nb, float y, const auto&) {
    const int64_t s = (grp * NB + nb) * 16 + nl;
    if (s < n && g == 0) out[s] = y;
  };
  if constexpr (DIRECT) {
    static_assert(P != 0 && std::is_same<IT, typename Prec<P>::T>::value, "direct loads need operand-typed features");
    {
      // the stored 16-bit features are the operand: one 16-byte load per lane per block
      struct Raw {
        Frag f[NB][KIN / 32];
      };
      mlp_stream<P, KIN, W, NB, Raw, NHC>(
          md.n_hidden, md.out_relu != 0, lds_frag, lds_wout, it.next, it.step, it.end,
          [&](int64_t grp, Raw& r) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
              for (int b = 0; b < KIN / 32; ++b)
                r.f[nb][b] = *reinterpret_cast<const Frag*>(feat + row(grp, nb) * KIN + 32 * b + 8 * g);
          },
          [&](const Raw& r, Frag (*in)[CH0]) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
              for (int b = 0; b < KIN / 32; ++b) in[nb][b] = r.f[nb][b];
          },
          st);
    }
  } else {
    struct Raw {
      IT v[NB][KIN / 32][8];
    };
    mlp_stream<P, KIN, W, NB, Raw, NHC>(
        md.n_hidden, md.out_relu != 0, lds_frag, lds_wout, it.next, it.step, it.end,
        [&](int64_t grp, Raw& r) {
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const int64_t sc = row(grp, nb);
#pragma unroll
            for (int b = 0; b < KIN / 32; ++b)
#pragma unroll
              for (int jj = 0; jj < 8; ++jj) {
                const int k = 32 * b + 8 * g + jj;
                r.v[nb][b][jj] = k < n_in ? feat[sc * n_in + k] : (IT)0.0f;
              }
          }
        },
        [&](const Raw& r, Frag (*in)[CH0]) {
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            float f[KIN / 32][8];
#pragma unroll
            for (int b = 0; b < KIN / 32; ++b)
#pragma unroll
              for (int jj = 0; jj < 8; ++jj) f[b][jj] = (float)r.v[nb][b][jj];
            feat_to_frag<P, KIN>(f, in[nb]);
          }
        },
        st);
  }
}

// ---------------------------------------------------------------------------
// Sampling step alone.
// ---------------------------------------------------------------------------
template <typename VT>
__global__ void __launch_bounds__(256) k_sample_batch(BatchArgs ba, float* __restrict__ xyz, float* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ba.B) return;
  const int64_t bstep = ba.step_index();
  const float a = batch_coord(ba.seed, bstep, ba.B, i, 0);
  const float b = batch_coord(ba.seed, bstep, ba.B, i, 1);
  const float c = batch_coord(ba.seed, bstep, ba.B, i, 2);
  xyz[3 * i] = a;
  xyz[3 * i + 1] = b;
  xyz[3 * i + 2] = c;
  y[i] = volume_sample<VT>(reinterpret_cast<const VT*>(ba.volume), ba.dims[0], ba.dims[1], ba.dims[2], a, b, c);
}

// ---------------------------------------------------------------------------
// Host-side launchers.  This file is compiled once per MLP precision
// (NGV_PSEL = 0, 1, 2): each object holds the launchers of its precision,
// and the first also the precision-independent launchers and dispatchers.
// ---------------------------------------------------------------------------
template <int P, int W, int MODE, typename VT>
static hipError_t launch_infer_t(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const float* xyz,
                                 const float4* rec, int64_t n, float* out, const VT* vol, int dx, int dy, int dz,
                                 double* sq, hipStream_t st) {
  const ModelDesc& md = plan->md;
  const int64_t n_groups = (n + 63) / 64;  // 64 samples per wave
  const int waves = enc_waves(plan);
  const size_t lds = enc_lds_bytes(plan, waves);
  const int grid = grid_for(plan, n_groups, waves, 32 / waves);
  NGV_DISPATCH_F_KIN(md.F, plan->kin, {
    if (tp.f16)
      hipLaunchKernelGGL((k_infer<P, F, KIN, W, __half, MODE, VT>), dim3(grid), dim3(64 * waves), lds, st, md, tp, mlp,
                         xyz, rec, n, out, vol, dx, dy, dz, sq);
    else
      hipLaunchKernelGGL((k_infer<P, F, KIN, W, float, MODE, VT>), dim3(grid), dim3(64 * waves), lds, st, md, tp, mlp,
                         xyz, rec, n, out, vol, dx, dy, dz, sq);
  });
  return hipGetLastError();
}

template <int P, int W>
hipError_t launch_infer_p(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const float* xyz,
                          const float4* rec, int64_t n, float* out, hipStream_t st) {
  return launch_infer_t<P, W, 0, float>(plan, tp, mlp, xyz, rec, n, out, nullptr, 1, 1, 1, nullptr, st);
}

template <int P, int W>
hipError_t launch_sq_error_grid_p(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const void* vol, int dtype,
                                  const int32_t dims[3], double* sq, hipStream_t st) {
  const int64_t n = (int64_t)dims[0] * dims[1] * dims[2];
  if (dtype == NGVOL_DT_F16)
    return launch_infer_t<P, W, 1, __half>(plan, tp, mlp, nullptr, nullptr, n, nullptr,
                                        reinterpret_cast<const __half*>(vol), dims[0], dims[1], dims[2], sq, st);
  return launch_infer_t<P, W, 1, float>(plan, tp, mlp, nullptr, nullptr, n, nullptr,
                                     reinterpret_cast<const float*>(vol), dims[0], dims[1], dims[2], sq, st);
}

template <int P, int W>
hipError_t launch_mlp_fwd_p(const ngvol_plan* plan, const float* mlp, const void* feat, int dtype, int64_t n,
                            float* out, hipStream_t st) {
  const ModelDesc& md = plan->md;
  const int64_t n_tiles = (n + 31) / 32;  // 2-tile groups
  const size_t lds = fwd_lds_bytes(plan);
  const int grid = grid_for(plan, n_tiles, 4, 8);
#define NGV_MLPF(IT, NHC)                                                                                      \
  do {                                                                                                         \
    if constexpr (P != 0 && std::is_same<IT, typename Prec<P>::T>::value) {                                    \
      if (md.n_in == KIN) {                                                                                    \
        hipLaunchKernelGGL((k_mlp_fwd<P, KIN, W, IT, NHC, true>), dim3(grid), dim3(256), lds, st, md, mlp,     \
                           (const IT*)feat, n, out);                                                           \
        break;                                                                                                 \
      }                                                                                                        \
    }                                                                                                          \
    hipLaunchKernelGGL((k_mlp_fwd<P, KIN, W, IT, NHC, false>), dim3(grid), dim3(256), lds, st, md, mlp,        \
                       (const IT*)feat, n, out);                                                               \
  } while (0)
  NGV_DISPATCH_KIN(plan->kin, {
    if (md.n_hidden == 2) {
      if (dtype == NGVOL_DT_BF16) NGV_MLPF(__bf16, 2);
      else if (dtype == NGVOL_DT_F16) NGV_MLPF(_Float16, 2);
      else NGV_MLPF(float, 2);
    } else {
      if (dtype == NGVOL_DT_BF16) NGV_MLPF(__bf16, 0);
      else if (dtype == NGVOL_DT_F16) NGV_MLPF(_Float16, 0);
      else NGV_MLPF(float, 0);
    }
  });
#undef NGV_MLPF
  return hipGetLastError();
}

template hipError_t launch_infer_p<NGV_PSEL, NGV_WSEL>(const ngvol_plan*, TablePtrs, const float*, const float*, const float4*,
                                             int64_t, float*, hipStream_t);
template hipError_t launch_sq_error_grid_p<NGV_PSEL, NGV_WSEL>(const ngvol_plan*, TablePtrs, const float*, const void*, int,
                                                     const int32_t*, double*, hipStream_t);
template hipError_t launch_mlp_fwd_p<NGV_PSEL, NGV_WSEL>(const ngvol_plan*, const float*, const void*, int, int64_t, float*,
                                               hipStream_t);

#if NGV_PRIMARY
size_t mlp_weight_bytes(const ngvol_plan* plan) {
  const int P = plan->layout.precision, KIN = plan->kin, W = plan->layout.n_neurons, nh = plan->md.n_hidden;
  const int ch0 = P ? KIN / 32 : KIN / 4;
  const int chh = P ? (W + 31) / 32 : W / 4;
  const int frags = (W / 16) * ch0 + (nh - 1) * (W / 16) * chh;
  return (size_t)frags * 64 * (P ? 16 : 4);
}

size_t wout_bytes(const ngvol_plan* plan) {
  // W_out in FP32, then (16-bit operands) the output layer's fragments
  const int P = plan->layout.precision, W = plan->layout.n_neurons;
  return (size_t)W * 4 + (P ? (size_t)((W + 31) / 32) * 64 * 16 : 0);
}

size_t fwd_lds_bytes(const ngvol_plan* plan) { return mlp_weight_bytes(plan) + wout_bytes(plan); }

size_t enc_lds_bytes(const ngvol_plan* plan, int waves) {
  // staged weights, then one encoding stage of 64 rows per wave
  const int P = plan->layout.precision, KIN = plan->kin;
  const size_t esz = P ? 2 : 4;
  const size_t row = (size_t)(KIN + 16 / esz) * esz;
  return ((fwd_lds_bytes(plan) + 15) & ~(size_t)15) + (size_t)waves * 64 * row;
}

int enc_waves(const ngvol_plan* plan) {
  // 4 waves per workgroup unless the weights and stages would not fit
  for (int w = 4; w > 1; w >>= 1)
    if (enc_lds_bytes(plan, w) <= kLdsLimit) return w;
  return 1;
}

hipError_t launch_encode(const ngvol_plan* plan, TablePtrs tp, const float* xyz, int64_t n, float* feat,
                         hipStream_t st) {
  const ModelDesc& md = plan->md;
  const int64_t n_groups = (n + 63) / 64;  // 64 samples per wave
  const int grid = grid_for(plan, n_groups, 4, 8);
  NGV_DISPATCH_F_KIN(md.F, plan->kin, {
    if (tp.f16)
      hipLaunchKernelGGL((k_encode<F, KIN, __half>), dim3(grid), dim3(256), 0, st, md, tp, xyz, n, feat);
    else
      hipLaunchKernelGGL((k_encode<F, KIN, float>), dim3(grid), dim3(256), 0, st, md, tp, xyz, n, feat);
  });
  return hipGetLastError();
}

hipError_t launch_encode_debug(const ngvol_plan* plan, const float* xyz, int64_t n, uint32_t* idx, float* w,
                               hipStream_t st) {
  const int64_t total = n * plan->md.L;
  const int64_t grid = (total + 255) / 256;
  hipLaunchKernelGGL(k_encode_debug, dim3((unsigned)grid), dim3(256), 0, st, plan->md, xyz, n, idx, w);
  return hipGetLastError();
}

hipError_t launch_infer(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const float* xyz, const float4* rec,
                        int64_t n, float* out, hipStream_t st) {
  NGV_DISPATCH_P(plan->layout.precision, NGV_DISPATCH_W(plan->md.width, return launch_infer_p<P, W>(plan, tp, mlp, xyz, rec, n, out, st)));
  return hipErrorInvalidValue;
}

hipError_t launch_sq_error_grid(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const void* vol, int dtype,
                                const int32_t dims[3], double* sq, hipStream_t st) {
  NGV_DISPATCH_P(plan->layout.precision, NGV_DISPATCH_W(plan->md.width, return launch_sq_error_grid_p<P, W>(plan, tp, mlp, vol, dtype, dims, sq, st)));
  return hipErrorInvalidValue;
}

hipError_t launch_mlp_fwd(const ngvol_plan* plan, const float* mlp, const void* feat, int dtype, int64_t n,
                          float* out, hipStream_t st) {
  NGV_DISPATCH_P(plan->layout.precision, NGV_DISPATCH_W(plan->md.width, return launch_mlp_fwd_p<P, W>(plan, mlp, feat, dtype, n, out, st)));
  return hipErrorInvalidValue;
}

hipError_t launch_sample_batch(const BatchArgs& ba, float* xyz, float* y, hipStream_t st) {
  const int64_t grid = (ba.B + 255) / 256;
  if (ba.vdtype == NGVOL_DT_F16)
    hipLaunchKernelGGL(k_sample_batch<__half>, dim3((unsigned)grid), dim3(256), 0, st, ba, xyz, y);
  else
    hipLaunchKernelGGL(k_sample_batch<float>, dim3((unsigned)grid), dim3(256), 0, st, ba, xyz, y);
  return hipGetLastError();
}
#endif  // NGV_PRIMARY

}  // namespace ngvol
