// Backward kernels: MLP backward with activation recompute (MFMA), encoding
// scatter-add, partial-sum reduction, Adam and step bookkeeping.
#include "kernels.hpp"
#include "lds_add.hpp"
#include "mlp_tile.hpp"

namespace ngvol {

namespace {

constexpr int kBwdMaxWaves = 8;
constexpr int kPitch = 20;  // LDS row pitch (elements) of the per-wave transposed buffers

__device__ __forceinline__ bool finite(float v) { return __builtin_isfinite(v); }

}  // namespace

// dW of one layer over the 16 samples of a tile, accumulated in registers:
// acc[mo][mi] += dz^T[16mo.., s] a[s, 16mi..] with dz^T and a^T the wave's
// transposed LDS rows ([neuron][sample], pitch kPitch).  Each operand
// fragment is read once (one 8-byte load for 16-bit operands) and used for
// a whole row or column of blocks.  Output element j of lane (nl, g) is
// dW[16mo + 4g + j][16mi + nl].
template <int P, int NO, int NI>
__device__ __forceinline__ void dw_accumulate(const typename Prec<P>::T* dzT, const typename Prec<P>::T* aT,
                                              f32x4 (&acc)[NO][NI]) {
  const int lane = threadIdx.x & 63, nl = lane & 15, g = lane >> 4;
  if constexpr (P != 0) {
    typedef typename Prec<P>::Frag4 F4;
    F4 a[NO], b[NI];
#pragma unroll
    for (int mo = 0; mo < NO; ++mo)
      a[mo] = __builtin_bit_cast(F4, *reinterpret_cast<const uint2*>(dzT + (16 * mo + nl) * kPitch + 4 * g));
#pragma unroll
    for (int mi = 0; mi < NI; ++mi)
      b[mi] = __builtin_bit_cast(F4, *reinterpret_cast<const uint2*>(aT + (16 * mi + nl) * kPitch + 4 * g));
#pragma unroll
    for (int mo = 0; mo < NO; ++mo)
#pragma unroll
      for (int mi = 0; mi < NI; ++mi) acc[mo][mi] = mfma_k16(a[mo], b[mi], acc[mo][mi]);
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float a[NO], b[NI];
#pragma unroll
      for (int mo = 0; mo < NO; ++mo) a[mo] = dzT[(16 * mo + nl) * kPitch + 4 * q + g];
#pragma unroll
      for (int mi = 0; mi < NI; ++mi) b[mi] = aT[(16 * mi + nl) * kPitch + 4 * q + g];
#pragma unroll
      for (int mo = 0; mo < NO; ++mo)
#pragma unroll
        for (int mi = 0; mi < NI; ++mi) acc[mo][mi] = mfma(a[mo], b[mi], acc[mo][mi]);
    }
  }
}

// Adds register dW blocks into a row-major [out][in_dim] matrix (columns
// >= in_dim are padding and dropped), scaled by `scale`.
template <int NO, int NI>
__device__ __forceinline__ void dw_flush(const f32x4 (&acc)[NO][NI], float* dw, int in_dim, float scale) {
  const int lane = threadIdx.x & 63, nl = lane & 15, g = lane >> 4;
#pragma unroll
  for (int mo = 0; mo < NO; ++mo)
#pragma unroll
    for (int mi = 0; mi < NI; ++mi) {
      const int i = 16 * mi + nl;
      if (i < in_dim) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float* p = dw + (16 * mo + 4 * g + j) * in_dim + i;
          *p += acc[mo][mi][j] * scale;
        }
      }
    }
}

template <int P, int KIN, int W>
__host__ __device__ constexpr size_t bwd_wave_bytes(int nh) {
  // z of every hidden layer (f32x4 per lane per block) + dz^T and a^T
  return (size_t)nh * (W / 16) * 64 * 16 + 2 * (size_t)(KIN > W ? KIN : W) * kPitch * (P ? 2 : 4);
}

size_t bwd_lds_bytes(const ngvol_plan* plan, int waves, bool gdw) {
  const int P = plan->layout.precision, KIN = plan->kin, W = plan->layout.n_neurons, nh = plan->md.n_hidden;
  const int ch0 = P ? KIN / 32 : KIN / 4;
  const int chh = P ? (W + 31) / 32 : W / 4;
  const int frags = (W / 16) * ch0 + (nh - 1) * (W / 16) * chh + (KIN / 16) * chh + (nh - 1) * (W / 16) * chh;
  size_t b = (size_t)frags * 64 * (P ? 16 : 4) + (size_t)W * 4;
  if (!gdw) b += ((size_t)plan->md.n_mlp * 4 + 15) / 16 * 16;
  const size_t wave = (size_t)nh * (W / 16) * 64 * 16 + 2 * (size_t)(KIN > W ? KIN : W) * kPitch * (P ? 2 : 4);
  return b + wave * waves;
}

// ---------------------------------------------------------------------------
// MLP backward: dW (per-block partial sums) and dL/dfeature written to dfeat.
// MODE 0 reads the training forward's stored encoding ([B][KIN], 16-bit or
// FP32), MODE 1 caller features ([n][n_in] FP32).  The table scatter of
// dfeat is a separate pass (bucketed, see kernels_scatter.hip).  The
// workgroup's dW sum lives in LDS, or with GDW (networks whose LDS dW would
// leave room for fewer than four waves) directly in the workgroup's own row
// of `partial`, which then lives in L2.  With NHC = 2 (two hidden layers,
// fixed at compile time) every wave keeps its dW in MFMA accumulators over
// all its tiles and the waves add them into the workgroup sum in turn at the
// end, in a fixed order and without atomics; otherwise each tile adds its
// 16-sample products into the sum with LDS (or L2) atomics.
// ---------------------------------------------------------------------------
template <int P, int KIN, int W, int MODE, bool GDW, int NHC>
__global__ void __launch_bounds__(64 * kBwdMaxWaves) k_bwd(ModelDesc md, const float* __restrict__ mlp,
                                             const void* __restrict__ e_buf, const float* __restrict__ g_buf,
                                             BatchArgs ba, float* __restrict__ grad, float* __restrict__ dfeat,
                                             float* __restrict__ partial, int32_t* __restrict__ nonfinite,
                                             float bscale) {
  typedef typename Prec<P>::Frag Frag;
  typedef WeightLayout<P, KIN, W> WL;
  typedef typename Prec<P>::T T;
  // 16-bit operands of the backward carry dz * bscale (a power of two chosen
  // on the host so loss-scaled gradients stay in the normal range); products
  // are multiplied back by 1/bscale, which is exact.
  const float ibscale = 1.0f / bscale;
  constexpr int MB = W / 16;
  constexpr int MBI = KIN / 16;
  constexpr int RT = KIN > W ? KIN : W;
  const int nh = NHC > 0 ? NHC : md.n_hidden;
  const int n_in = md.n_in;

  extern __shared__ __align__(16) unsigned char smem[];
  const int fwd_frags = WL::frags(nh, false);
  const int all_frags = WL::frags(nh, true);
  Frag* lds_frag = reinterpret_cast<Frag*>(smem);
  size_t off = (size_t)all_frags * 64 * sizeof(Frag);
  float* lds_wout = reinterpret_cast<float*>(smem + off);
  off += W * 4;
  float* lds_dw;
  if constexpr (GDW) {
    lds_dw = partial + (size_t)blockIdx.x * md.n_mlp;
  } else {
    lds_dw = reinterpret_cast<float*>(smem + off);
    off += ((size_t)md.n_mlp * 4 + 15) / 16 * 16;
  }
  const int wave = threadIdx.x >> 6;
  unsigned char* wbase = smem + off + (size_t)wave * bwd_wave_bytes<P, KIN, W>(nh);
  f32x4* zbuf = reinterpret_cast<f32x4*>(wbase);
  T* dzT = reinterpret_cast<T*>(wbase + (size_t)nh * MB * 64 * 16);
  T* aT = dzT + RT * kPitch;

  for (int t = threadIdx.x; t < md.n_mlp; t += blockDim.x) lds_dw[t] = 0.0f;
  stage_weights<P, KIN, W>(md, mlp, lds_frag, lds_wout, true);
  __syncthreads();

  const int lane = threadIdx.x & 63, nl = lane & 15, g = lane >> 4;
  const int64_t B = ba.B;
  float dwo[MB][4];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int j = 0; j < 4; ++j) dwo[mb][j] = 0.0f;
  bool bad = false;
  // NHC == 2: the wave's dW of layers 1 and 0 over all its tiles
  f32x4 dacc1[NHC == 2 ? MB : 1][NHC == 2 ? MB : 1];
  f32x4 dacc0[NHC == 2 ? MB : 1][NHC == 2 ? MBI : 1];
  if constexpr (NHC == 2) {
#pragma unroll
    for (int mo = 0; mo < MB; ++mo) {
#pragma unroll
      for (int mi = 0; mi < MB; ++mi) dacc1[mo][mi] = zero4();
#pragma unroll
      for (int mi = 0; mi < MBI; ++mi) dacc0[mo][mi] = zero4();
    }
  }

  const int64_t n_tiles = (B + 15) >> 4;
  TileIter it(n_tiles);
  for (int64_t t = it.next; t < it.end; t += it.step) {
    const int64_t s = t * 16 + nl;
    const bool valid = s < B;
    const int64_t sc = valid ? s : B - 1;
    // ---- stored encoding -> layer-0 operands
    float f[KIN / 32][8];
    if constexpr (MODE == 0) {  // stored encoding of the training forward
      if constexpr (P) {
#pragma unroll
        for (int b = 0; b < KIN / 32; ++b) {
          const Frag v = *reinterpret_cast<const Frag*>(reinterpret_cast<const T*>(e_buf) + sc * KIN + 32 * b + 8 * g);
#pragma unroll
          for (int jj = 0; jj < 8; ++jj) f[b][jj] = (float)v[jj];
        }
      } else {
#pragma unroll
        for (int b = 0; b < KIN / 32; ++b) {
          const float* src = reinterpret_cast<const float*>(e_buf) + sc * KIN + 32 * b + 8 * g;
          const float4 u = *reinterpret_cast<const float4*>(src);
          const float4 w4 = *reinterpret_cast<const float4*>(src + 4);
          f[b][0] = u.x; f[b][1] = u.y; f[b][2] = u.z; f[b][3] = u.w;
          f[b][4] = w4.x; f[b][5] = w4.y; f[b][6] = w4.z; f[b][7] = w4.w;
        }
      }
    } else {
      const float* fe = reinterpret_cast<const float*>(e_buf);
#pragma unroll
      for (int b = 0; b < KIN / 32; ++b)
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
          const int k = 32 * b + 8 * g + jj;
          f[b][jj] = k < n_in ? fe[sc * n_in + k] : 0.0f;
        }
    }
    if constexpr (P) {
      // the forward saw 16-bit rounded inputs; use the same values here
#pragma unroll
      for (int b = 0; b < KIN / 32; ++b)
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) f[b][jj] = (float)(T)f[b][jj];
    }
    Frag in[InChunks<P, KIN>::n];
    feat_to_frag<P, KIN>(f, in);

    // ---- forward recompute, z of every hidden layer kept in LDS
    f32x4 act[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      f32x4 acc = zero4();
#pragma unroll
      for (int c = 0; c < WL::CH0; ++c) acc = mfma(lds_frag[(mb * WL::CH0 + c) * 64 + lane], in[c], acc);
      act[mb] = acc;
      zbuf[mb * 64 + lane] = acc;
    }
    auto fwd_layer = [&](int li) {
      Frag bfr[WL::CHH];
      pack_hidden<P, W>(act, bfr, true);
      const Frag* base = lds_frag + (WL::FR0 + (li - 1) * WL::FRH) * 64;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        f32x4 acc = zero4();
#pragma unroll
        for (int c = 0; c < WL::CHH; ++c) acc = mfma(base[(mb * WL::CHH + c) * 64 + lane], bfr[c], acc);
        act[mb] = acc;
        zbuf[(li * MB + mb) * 64 + lane] = acc;
      }
    };
    if constexpr (NHC > 0) {
#pragma unroll
      for (int li = 1; li < NHC; ++li) fwd_layer(li);
    } else {
      for (int li = 1; li < nh; ++li) fwd_layer(li);
    }

    // ---- output layer
    float gv = valid ? g_buf[sc] : 0.0f;
    if constexpr (MODE == 1) {
      // an output ReLU passes d_out only where its input was positive (the
      // training forward has already applied this to its gradient)
      if (md.out_relu) {
        float zo = 0.0f;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int j = 0; j < 4; ++j) zo = __builtin_fmaf(lds_wout[16 * mb + 4 * g + j], relu_bits(act[mb][j]), zo);
        zo += __shfl_xor(zo, 16, 64);
        zo += __shfl_xor(zo, 32, 64);
        if (!(zo > 0.0f)) gv = 0.0f;
      }
    }
    if (!finite(gv)) bad = true;
    f32x4 dz[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float zz = act[mb][j];
        const float h = relu_bits(zz);
        dwo[mb][j] = __builtin_fmaf(gv, h, dwo[mb][j]);
        dz[mb][j] = zz > 0.0f ? lds_wout[16 * mb + 4 * g + j] * gv : 0.0f;
      }

    // ---- hidden layers, last to first
    f32x4 de[MBI];
    auto bwd_layer = [&](int li) {
      const int in_dim = li == 0 ? n_in : W;
      // dz^T and a^T of this layer into the wave's LDS buffers
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int j = 0; j < 4; ++j) dzT[(16 * mb + 4 * g + j) * kPitch + nl] = (T)(dz[mb][j] * bscale);
      if (li > 0) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const f32x4 zp = zbuf[((li - 1) * MB + mb) * 64 + lane];
#pragma unroll
          for (int j = 0; j < 4; ++j) aT[(16 * mb + 4 * g + j) * kPitch + nl] = (T)relu_bits(zp[j]);
        }
      } else {
#pragma unroll
        for (int b = 0; b < KIN / 32; ++b)
#pragma unroll
          for (int jj = 0; jj < 8; ++jj) aT[(32 * b + 8 * g + jj) * kPitch + nl] = (T)f[b][jj];
      }
      wave_sync();
      // dW_li[o][i] += sum_s dz[s][o] a[s][i]
      if constexpr (NHC == 2) {
        if (li == 1) dw_accumulate<P, MB, MB>(dzT, aT, dacc1);
        else dw_accumulate<P, MB, MBI>(dzT, aT, dacc0);
      } else {
      float* dw = lds_dw + md.w_off[li];
      const int mbi_n = li == 0 ? MBI : MB;
#pragma unroll
      for (int mo = 0; mo < MB; ++mo) {
        for (int mi = 0; mi < mbi_n; ++mi) {
          f32x4 acc = zero4();
          if constexpr (P) {
            const T* pa = dzT + (16 * mo + nl) * kPitch + 4 * g;
            const T* pb = aT + (16 * mi + nl) * kPitch + 4 * g;
            typename Prec<P>::Frag4 a4, b4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              a4[q] = pa[q];
              b4[q] = pb[q];
            }
            acc = mfma_k16(a4, b4, acc);
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              acc = mfma((float)dzT[(16 * mo + nl) * kPitch + 4 * q + g], (float)aT[(16 * mi + nl) * kPitch + 4 * q + g],
                         acc);
          }
          const int i = 16 * mi + nl;
          if (i < in_dim) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int o = 16 * mo + 4 * g + j;
              if (acc[j] != 0.0f) {
                if constexpr (GDW) atomicAdd(dw + o * in_dim + i, acc[j] * ibscale);  // L2
                else lds_add_f32(dw + o * in_dim + i, acc[j] * ibscale);
              }
            }
          }
        }
      }
      }
      wave_sync();
      // dh = W_li^T dz
      Frag dzf[WL::CHH];
      {
        f32x4 dzs[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int j = 0; j < 4; ++j) dzs[mb][j] = dz[mb][j] * bscale;
        pack_hidden<P, W>(dzs, dzf, false);
      }
      if (li > 0) {
        const Frag* base = lds_frag + (fwd_frags + WL::FR0T + (li - 1) * WL::FRHT) * 64;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          f32x4 acc = zero4();
#pragma unroll
          for (int c = 0; c < WL::CHH; ++c) acc = mfma(base[(mb * WL::CHH + c) * 64 + lane], dzf[c], acc);
          const f32x4 zp = zbuf[((li - 1) * MB + mb) * 64 + lane];
#pragma unroll
          for (int j = 0; j < 4; ++j) dz[mb][j] = zp[j] > 0.0f ? acc[j] * ibscale : 0.0f;
        }
      } else {
        const Frag* base = lds_frag + fwd_frags * 64;
#pragma unroll
        for (int mb = 0; mb < MBI; ++mb) {
          f32x4 acc = zero4();
#pragma unroll
          for (int c = 0; c < WL::CHH; ++c) acc = mfma(base[(mb * WL::CHH + c) * 64 + lane], dzf[c], acc);
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[j] *= ibscale;
          de[mb] = acc;
        }
      }
    };
    if constexpr (NHC > 0) {
#pragma unroll
      for (int li = NHC - 1; li >= 0; --li) bwd_layer(li);
    } else {
      for (int li = nh - 1; li >= 0; --li) bwd_layer(li);
    }

    // ---- dL/dfeature: lane holds features 16m + 4g + j
    if (valid) {
#pragma unroll
      for (int m = 0; m < MBI; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (!finite(de[m][j])) bad = true;
      if (dfeat) {
#pragma unroll
        for (int m = 0; m < MBI; ++m)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int k = 16 * m + 4 * g + j;
            if (k < n_in) dfeat[sc * n_in + k] = de[m][j];
          }
      }
    }
  }

  // ---- output-layer gradient: reduce over the 16 samples of each lane group
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float v = dwo[mb][j];
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      dwo[mb][j] = v;
    }
  if (bad) *nonfinite = 1;
  // ---- the waves add their sums into the workgroup's dW one after another
  // (every lane owns distinct elements, so a turn needs no atomics)
  const int wpb = blockDim.x >> 6;
  for (int w = 0; w < wpb; ++w) {
    __syncthreads();
    if (wave == w) {
      if constexpr (NHC == 2) {
        dw_flush<MB, MB>(dacc1, lds_dw + md.w_off[1], W, ibscale);
        dw_flush<MB, MBI>(dacc0, lds_dw + md.w_off[0], n_in, ibscale);
      }
      if (nl == 0) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int j = 0; j < 4; ++j) lds_dw[md.w_off[nh] + 16 * mb + 4 * g + j] += dwo[mb][j];
      }
    }
  }
  if constexpr (!GDW) {
    __syncthreads();
    float* dst = partial + (size_t)blockIdx.x * md.n_mlp;
    for (int t = threadIdx.x; t < md.n_mlp; t += blockDim.x) dst[t] = lds_dw[t];
  }
}

// grad_mlp[k] += sum over blocks of partial[b][k], in a fixed order: a
// workgroup covers 64 columns; its 16 thread rows each sum every 16th
// partial, then the 16 row sums are added in LDS.
__global__ void __launch_bounds__(1024) k_reduce_partials(const float* __restrict__ partial, int blocks, int n_mlp,
                                                          float* __restrict__ grad_mlp,
                                                          int32_t* __restrict__ nonfinite) {
  __shared__ float part[16][65];
  const int col = threadIdx.x & 63, row = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + col;
  float s = 0.0f;
  if (k < n_mlp)
    for (int b = row; b < blocks; b += 16) s += partial[(size_t)b * n_mlp + k];
  part[row][col] = s;
  __syncthreads();
  if (row == 0 && k < n_mlp) {
    float t = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) t += part[r][col];
    const float v = grad_mlp[k] + t;
    grad_mlp[k] = v;
    if (!finite(v)) *nonfinite = 1;
  }
}

// Encoding backward alone: one thread per (sample, level).
template <int F>
__global__ void __launch_bounds__(256) k_encode_bwd(ModelDesc md, const float* __restrict__ xyz, int64_t n,
                                                    const float* __restrict__ dfeat, float* __restrict__ grad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * md.L) return;
  const int64_t s = t / md.L;
  const int l = (int)(t % md.L);
  Corners cr;
  level_corners(md.lv[l], clamp01(xyz[3 * s]), clamp01(xyz[3 * s + 1]), clamp01(xyz[3 * s + 2]), cr);
  float d[F];
#pragma unroll
  for (int f = 0; f < F; ++f) d[f] = dfeat[s * md.n_in + l * F + f];
  scatter_level<F>(cr, grad, d);
}

// ---------------------------------------------------------------------------
// Adam over all parameters; skipped (gradient only cleared) when a
// non-finite contribution was seen.  t = step + 1; c1 = 1 - b1^t and
// c2 = 1 - b2^t in FP64; the step's learning rate follows the exponential
// decay schedule of the arguments, and l2_reg * w joins the gradient of the
// MLP weights (indices >= n_table).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_adam(int64_t n, int64_t n_table, float* __restrict__ params,
                                              __half* __restrict__ table_f16, float* __restrict__ grad,
                                              float* __restrict__ m, float* __restrict__ v,
                                              const int64_t* __restrict__ step, const int32_t* __restrict__ nonfinite,
                                              AdamArgs a) {
  __shared__ float coef[3];
  const bool skip = *nonfinite != 0;
  if (threadIdx.x == 0) {
    const int64_t k = *step;
    double lr = a.lr;
    if (a.decay_interval > 0 && k >= a.decay_start)
      lr *= pow(a.decay_base, (double)((k - a.decay_start) / a.decay_interval));
    const double t = (double)(k + 1);
    const double c1 = 1.0 - pow(a.b1, t);
    const double c2 = 1.0 - pow(a.b2, t);
    coef[0] = (float)(lr / c1);   // lr_k / c1
    coef[1] = (float)(1.0 / c2);  // 1 / c2
    coef[2] = (float)a.l2_reg;
  }
  __syncthreads();
  const float lr_c1 = coef[0], inv_c2 = coef[1], l2 = coef[2];
  const float b1 = (float)a.b1, b2 = (float)a.b2, eps = (float)a.eps;
  const float omb1 = (float)(1.0 - a.b1), omb2 = (float)(1.0 - a.b2);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    float gr = grad[i] * a.inv_scale;
    grad[i] = 0.0f;
    if (skip) continue;
    const float w = params[i];
    if (i >= n_table) gr = __builtin_fmaf(l2, w, gr);
    const float mi = __builtin_fmaf(b1, m[i], omb1 * gr);
    const float vi = __builtin_fmaf(b2, v[i], omb2 * gr * gr);
    m[i] = mi;
    v[i] = vi;
    const float p = w - lr_c1 * mi / (sqrtf(vi * inv_c2) + eps);
    params[i] = p;
    if (table_f16 && i < n_table) table_f16[i] = __float2half_rn(p);
  }
}

__global__ void k_step_begin(double* loss_acc, int32_t* nonfinite) {
  *loss_acc = 0.0;
  *nonfinite = 0;
}

__global__ void k_step_end(const double* loss_acc, int32_t* nonfinite, int64_t* step, int64_t* draws,
                           int32_t* skipped, double* loss_out, double inv_b) {
  const int32_t bad = *nonfinite;
  if (!bad) *step += 1;
  if (draws) *draws += 1;
  if (skipped) *skipped = bad;
  if (loss_out) *loss_out = *loss_acc * inv_b;
}

__global__ void k_zero_f64(double* p) { *p = 0.0; }

// MSE = sum * inv_n; PSNR = -10 log10(MSE) (peak 1), both in FP64
__global__ void k_psnr_finish(double* mse, double inv_n, double* psnr) {
  const double m = *mse * inv_n;
  *mse = m;
  if (psnr) *psnr = -10.0 * log10(m);
}

__global__ void __launch_bounds__(256) k_make_f16(const float* __restrict__ p, __half* __restrict__ o, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) o[i] = __float2half_rn(p[i]);
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
BwdConfig bwd_config(const ngvol_plan* plan) {
  // as many waves per workgroup (up to 8) as the LDS holds: one workgroup
  // per CU accumulates dW, so its waves are the CU's latency hiding.  dW
  // moves out of LDS when that buys more waves than the LDS form's (< 4).
  auto most = [&](bool gdw) {
    for (int w = kBwdMaxWaves; w >= 1; w >>= 1)
      if (bwd_lds_bytes(plan, w, gdw) <= kLdsLimit) return w;
    return 0;
  };
  const int wl = most(false), wg = most(true);
  if (wl >= 4 || wl >= wg) return BwdConfig{wl > 0 ? wl : 1, false};
  return BwdConfig{wg, true};
}

int bwd_waves(const ngvol_plan* plan) { return bwd_config(plan).waves; }

int bwd_grid(const ngvol_plan* plan, int64_t n) {
  const int64_t n_tiles = (n + 15) / 16;
  const int waves = bwd_waves(plan);
  int64_t need = (n_tiles + waves - 1) / waves;
  const int64_t cap = (int64_t)plan->cus;
  if (need > cap) need = cap;
  if (need < 1) need = 1;
  return (int)need;
}

hipError_t launch_bwd(const ngvol_plan* plan, int mode, const float* mlp, const void* e_buf, const float* g_buf,
                      const BatchArgs& ba, float* grad, float* dfeat, float* partial, int grid, int32_t* nonfinite,
                      float bscale, hipStream_t st) {
  const ModelDesc& md = plan->md;
  const BwdConfig bc = bwd_config(plan);
  const int waves = bc.waves;
  const size_t lds = bwd_lds_bytes(plan, waves, bc.gdw);
  const int P_ = plan->layout.precision;
#define NGV_BWD_GO(P, KIN, W, M, G)                                                                                \
  do {                                                                                                         \
    if (md.n_hidden == 2)                                                                                      \
      hipLaunchKernelGGL((k_bwd<P, KIN, W, M, G, 2>), dim3(grid), dim3(64 * waves), lds, st, md, mlp, e_buf,   \
                         g_buf, ba, grad, dfeat, partial, nonfinite, bscale);                                  \
    else                                                                                                       \
      hipLaunchKernelGGL((k_bwd<P, KIN, W, M, G, 0>), dim3(grid), dim3(64 * waves), lds, st, md, mlp, e_buf,   \
                         g_buf, ba, grad, dfeat, partial, nonfinite, bscale);                                  \
  } while (0)
#define NGV_BWD_LAUNCH(P, KIN, W)                          \
  do {                                                    \
    if (mode == 0) {                                      \
      if (bc.gdw) NGV_BWD_GO(P, KIN, W, 0, true);         \
      else NGV_BWD_GO(P, KIN, W, 0, false);               \
    } else {                                              \
      if (bc.gdw) NGV_BWD_GO(P, KIN, W, 1, true);         \
      else NGV_BWD_GO(P, KIN, W, 1, false);               \
    }                                                     \
  } while (0)
#define NGV_BWD_W(P, KIN)                                      \
  do {                                                         \
    if (md.width == 32) NGV_BWD_LAUNCH(P, KIN, 32);             \
    else if (md.width == 64) NGV_BWD_LAUNCH(P, KIN, 64);        \
    else return hipErrorInvalidValue;                          \
  } while (0)
#define NGV_BWD_K(P)                                                    \
  do {                                                                  \
    if (plan->kin == 32) NGV_BWD_W(P, 32);                              \
    else if (plan->kin == 64) NGV_BWD_W(P, 64);                         \
    else return hipErrorInvalidValue;                                   \
  } while (0)
  if (P_ == 1) NGV_BWD_K(1);
  else if (P_ == 2) NGV_BWD_K(2);
  else NGV_BWD_K(0);
#undef NGV_BWD_K
#undef NGV_BWD_W
#undef NGV_BWD_LAUNCH
#undef NGV_BWD_GO
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const ngvol_plan* plan, const float* partial, int grid, float* grad,
                                  int32_t* nonfinite, hipStream_t st) {
  const int n = plan->md.n_mlp;
  hipLaunchKernelGGL(k_reduce_partials, dim3((n + 63) / 64), dim3(1024), 0, st, partial, grid, n,
                     grad + plan->md.n_table, nonfinite);
  return hipGetLastError();
}

hipError_t launch_encode_bwd(const ngvol_plan* plan, const float* xyz, int64_t n, const float* dfeat, float* grad,
                             hipStream_t st) {
  const ModelDesc& md = plan->md;
  const int64_t total = n * md.L;
  const unsigned grid = (unsigned)((total + 255) / 256);
  switch (md.F) {
    case 1: hipLaunchKernelGGL(k_encode_bwd<1>, dim3(grid), dim3(256), 0, st, md, xyz, n, dfeat, grad); break;
    case 2: hipLaunchKernelGGL(k_encode_bwd<2>, dim3(grid), dim3(256), 0, st, md, xyz, n, dfeat, grad); break;
    case 4: hipLaunchKernelGGL(k_encode_bwd<4>, dim3(grid), dim3(256), 0, st, md, xyz, n, dfeat, grad); break;
    case 8: hipLaunchKernelGGL(k_encode_bwd<8>, dim3(grid), dim3(256), 0, st, md, xyz, n, dfeat, grad); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_adam(const ngvol_plan* plan, float* params, __half* table_f16, float* grad, float* m, float* v,
                       int64_t* step, const int32_t* nonfinite, const AdamArgs& a, hipStream_t st) {
  const int64_t n = plan->md.n_params;
  int64_t grid = (n + 255) / 256;
  const int64_t cap = (int64_t)plan->cus * 16;
  if (grid > cap) grid = cap;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)grid), dim3(256), 0, st, n, plan->md.n_table, params, table_f16, grad, m,
                     v, step, nonfinite, a);
  return hipGetLastError();
}

hipError_t launch_step_begin(double* loss_acc, int32_t* nonfinite, hipStream_t st) {
  hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(1), 0, st, loss_acc, nonfinite);
  return hipGetLastError();
}

hipError_t launch_step_end(const double* loss_acc, int32_t* nonfinite, int64_t* step, int64_t* draws,
                           int32_t* skipped, double* loss_out, double inv_b, hipStream_t st) {
  hipLaunchKernelGGL(k_step_end, dim3(1), dim3(1), 0, st, loss_acc, nonfinite, step, draws, skipped, loss_out,
                     inv_b);
  return hipGetLastError();
}

hipError_t launch_zero_f64(double* p, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(1), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_psnr_finish(double* mse, double inv_n, double* psnr, hipStream_t st) {
  hipLaunchKernelGGL(k_psnr_finish, dim3(1), dim3(1), 0, st, mse, inv_n, psnr);
  return hipGetLastError();
}

hipError_t launch_make_f16(const float* params, __half* out, int64_t n, hipStream_t st) {
  int64_t grid = (n + 255) / 256;
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_make_f16, dim3((unsigned)grid), dim3(256), 0, st, params, out, n);
  return hipGetLastError();
}

}  // namespace ngvol
