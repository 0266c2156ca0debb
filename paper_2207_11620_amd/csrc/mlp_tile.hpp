// Wavefront-tile MLP on the matrix cores (gfx950).
//
// A wave evaluates the network on tiles of 16 samples.  Activations live in
// the MFMA accumulator layout, transposed: for a layer of width Wd the lane
// (n = lane%16, g = lane/16) holds, for each 16-neuron block m, the values of
// neurons 16m + 4g + j (j = 0..3) of sample n.  The next layer contracts over
// neurons, and since the order of a contraction is free, its K chunks are
// formed directly from the registers a lane already holds; the matching
// permutation is applied to the weights once, when a workgroup stages them in
// LDS.  No shuffles are needed between layers.
//
// Two precisions share this structure:
//   P = 1: BF16 operands, v_mfma_f32_16x16x32_bf16 (K = 32 per instruction);
//   P = 2: FP16 operands, v_mfma_f32_16x16x32_f16 (K = 32, same lane layout);
//   P = 0: FP32 operands, v_mfma_f32_16x16x4_f32 (K = 4 per instruction).
// Both accumulate in FP32.
//
// The output neuron (W_out, one row) is a VALU dot product for P = 0.  For
// 16-bit operands it is one more MFMA per K chunk: its A operand holds W_out
// in rows 0, 4, 8 and 12 and zeros elsewhere, so that accumulator element 0
// of every lane (n, g) is the output of sample n - each lane receives its
// sample's output without a shuffle.  An optional ReLU follows it.
//
// Encoded inputs enter as B operands in which, for every 32-feature block b,
// lane group g holds features 32b + 8g + jj (jj = 0..7) of sample n.  They
// are produced with one sample per lane (all lanes on the same level) and
// redistributed through a per-wave LDS stage.
#pragma once

#include "device_common.hpp"

namespace ngvol {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma(const f16x8& a, const f16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma(float a, float b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// K = 16 BF16 product, used where the contraction runs over the 16 samples of a tile.
__device__ __forceinline__ f32x4 mfma_k16(const bf16x4& a, const bf16x4& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_k16(const f16x4& a, const f16x4& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 zero4() { return f32x4{0.0f, 0.0f, 0.0f, 0.0f}; }

template <int P>
struct Prec;

template <>
struct Prec<1> {
  typedef __bf16 T;
  typedef bf16x8 Frag;
  typedef bf16x4 Frag4;
  static constexpr int K = 32;
  static __device__ __forceinline__ Frag zero() {
    Frag f;
#pragma unroll
    for (int i = 0; i < 8; ++i) f[i] = (T)0.0f;
    return f;
  }
};

template <>
struct Prec<2> {
  typedef _Float16 T;
  typedef f16x8 Frag;
  typedef f16x4 Frag4;
  static constexpr int K = 32;
  static __device__ __forceinline__ Frag zero() {
    Frag f;
#pragma unroll
    for (int i = 0; i < 8; ++i) f[i] = (T)0.0f;
    return f;
  }
};

template <>
struct Prec<0> {
  typedef float T;
  typedef float Frag;
  static constexpr int K = 4;
  static __device__ __forceinline__ Frag zero() { return 0.0f; }
};

// Number of K chunks of a layer's input.
//   encoded input of KIN features: P1: KIN/32, P0: KIN/4
//   hidden input of width W:       P1: ceil(W/32), P0: W/4
template <int P, int KIN>
struct InChunks {
  static constexpr int n = P ? KIN / 32 : KIN / 4;
};
template <int P, int W>
struct HidChunks {
  static constexpr int n = P ? (W + 31) / 32 : W / 4;
};

// Input feature (column) that lane group g feeds at position jj of chunk c.
template <int P>
__device__ __forceinline__ int enc_col(int c, int g, int jj) {
  if constexpr (P) return 32 * c + 8 * g + jj;
  else return 32 * (c >> 3) + 8 * g + (c & 7);
}
template <int P>
__device__ __forceinline__ int hid_col(int c, int g, int jj) {
  if constexpr (P) return 16 * (2 * c + (jj >> 2)) + 4 * g + (jj & 3);
  else return 16 * (c >> 2) + 4 * g + (c & 3);
}

// ---------------------------------------------------------------------------
// Weight staging.  Layer li's fragments for output block mb and chunk c are
// stored at frag index (layer_base[li] + mb * chunks[li] + c) * 64 + lane.
// Entries whose row or column falls outside the matrix are zero.
// ---------------------------------------------------------------------------
template <int P, int KIN, int W>
struct WeightLayout {
  static constexpr int CH0 = InChunks<P, KIN>::n;
  static constexpr int CHH = HidChunks<P, W>::n;
  static constexpr int MB = W / 16;
  static constexpr int FR0 = MB * CH0;  // fragments of the input layer
  static constexpr int FRH = MB * CHH;  // fragments of each hidden layer
  // fragments of the transposed matrices (backward): input dim becomes the M side
  static constexpr int MB0T = KIN / 16;  // blocks of W0^T rows
  static constexpr int FR0T = MB0T * CHH;
  static constexpr int FRHT = MB * CHH;
  __host__ __device__ static constexpr int frags(int n_hidden, bool bwd) {
    return FR0 + (n_hidden - 1) * FRH + (bwd ? FR0T + (n_hidden - 1) * FRHT : 0);
  }
};

// The region behind the staged matrices: W_out in FP32 (W floats) and, for
// 16-bit operands in the forward, the output layer's A fragments.
template <int P, int W>
__host__ __device__ constexpr size_t wout_region_bytes() {
  return (size_t)W * 4 + (P != 0 ? (size_t)HidChunks<P, W>::n * 64 * sizeof(typename Prec<P>::Frag) : 0);
}
template <int P, int W>
__device__ __forceinline__ typename Prec<P>::Frag* out_frags(float* lds_wout) {
  return reinterpret_cast<typename Prec<P>::Frag*>(lds_wout + W);
}
template <int P, int W>
__device__ __forceinline__ const typename Prec<P>::Frag* out_frags(const float* lds_wout) {
  return reinterpret_cast<const typename Prec<P>::Frag*>(lds_wout + W);
}

// Stage W0..W_{h-1} (and, for the backward, their transposes) into LDS in
// fragment order, plus W_out in FP32 and (forward, 16-bit operands) as
// output-layer fragments.  Called by the whole workgroup.
// colmap (optional, LDS): input feature of each first-layer operand column
// (-1: none), for kernels whose encoded inputs arrive in another order.
template <int P, int KIN, int W>
__device__ void stage_weights(const ModelDesc& md, const float* __restrict__ mlp, typename Prec<P>::Frag* lds_frag,
                              float* lds_wout, bool bwd, const int8_t* colmap = nullptr) {
  typedef WeightLayout<P, KIN, W> WL;
  typedef typename Prec<P>::Frag Frag;
  constexpr int EPF = P ? 8 : 1;  // elements per fragment
  constexpr int U = P ? 4 : 16;   // fragments per thread per round: their loads are in flight together
  const int nh = md.n_hidden;
  const int n_in = md.n_in;
  const int total = WL::frags(nh, bwd) * 64;
  const int fw = WL::FR0 + (nh - 1) * WL::FRH;
  for (int t0 = threadIdx.x; t0 < total; t0 += blockDim.x * U) {
    float x[U][EPF];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * (int)blockDim.x;
      const int lane = t & 63;
      int fr = t >> 6;
      const int i = lane & 15, g = lane >> 4;
      // which matrix
      int li, mb, c;
      bool trans = false;
      if (fr >= fw) {
        trans = true;
        fr -= fw;
        if (fr < WL::FR0T) {
          li = 0;
          mb = fr / WL::CHH;
          c = fr % WL::CHH;
        } else {
          fr -= WL::FR0T;
          li = 1 + fr / WL::FRHT;
          fr %= WL::FRHT;
          mb = fr / WL::CHH;
          c = fr % WL::CHH;
        }
      } else if (fr < WL::FR0) {
        li = 0;
        mb = fr / WL::CH0;
        c = fr % WL::CH0;
      } else {
        fr -= WL::FR0;
        li = 1 + fr / WL::FRH;
        fr %= WL::FRH;
        mb = fr / WL::CHH;
        c = fr % WL::CHH;
      }
      const bool live = t < total;
      if (!live) li = 0;
      // matrix offset by selects over the (uniform) offsets, not an indexed load
      int off = md.w_off[0];
#pragma unroll
      for (int q = 1; q < NGVOL_MAX_LAYERS; ++q) off = li == q ? md.w_off[q] : off;
      const int in_dim = li == 0 ? n_in : W;
#pragma unroll
      for (int jj = 0; jj < EPF; ++jj) {
        int idx = -1;
        const int row = 16 * mb + i;
        if (!trans) {
          // forward: A[row = 16mb + i][k] = W[row][col(k)]
          int col = li == 0 ? enc_col<P>(c, g, jj) : hid_col<P>(c, g, jj);
          if (li == 0 && colmap) col = col < KIN ? colmap[col] : -1;
          if (row < W && col >= 0 && col < in_dim) idx = row * in_dim + col;
        } else {
          // backward: A[row = 16mb + i][k] = W^T[row][col(k)] = W[col][row], contracting over W's rows
          const int col = hid_col<P>(c, g, jj);
          if (row < in_dim && col < W) idx = col * in_dim + row;
        }
        // every lane loads (an in-range element when its own is absent), so
        // that the loads of the round are issued together; zeros are selected after
        const bool use = live && idx >= 0;
        x[u][jj] = mlp[use ? off + idx : 0];
        if (!use) x[u][jj] = 0.0f;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * (int)blockDim.x;
      if (t < total) {
        Frag val;
        if constexpr (P) {
#pragma unroll
          for (int jj = 0; jj < EPF; ++jj) val[jj] = (typename Prec<P>::T)x[u][jj];
        } else {
          val = x[u][0];
        }
        lds_frag[t] = val;
      }
    }
  }
  const float* wo = mlp + md.w_off[nh];
  for (int t = threadIdx.x; t < W; t += blockDim.x) lds_wout[t] = wo[t];
  if constexpr (P != 0) {
    // forward: the output layer's A operands (W_out in rows 0, 4, 8, 12)
    if (!bwd) {
      Frag* ofrag = out_frags<P, W>(lds_wout);
      for (int t = threadIdx.x; t < HidChunks<P, W>::n * 64; t += blockDim.x) {
        const int lane = t & 63, c = t >> 6, i = lane & 15, g = lane >> 4;
        Frag val;
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
          const int col = hid_col<P>(c, g, jj);
          val[jj] = (typename Prec<P>::T)((i & 3) == 0 && col < W ? wo[col] : 0.0f);
        }
        ofrag[t] = val;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Forward through the hidden layers.
//   in_frag[c]   : B operands of the encoded input (chunks of layer 0)
//   z[li][mb]    : pre-activations kept for the backward (optional)
//   returns the last hidden activation in act[mb] (FP32, accumulator layout)
// ---------------------------------------------------------------------------
// ReLU on the bit pattern: a float with the sign bit set is a negative
// integer, so max(bits, 0) is max(x, 0) in one integer instruction (the float
// max would first quiet its matrix-core input).  A NaN with the sign bit set
// becomes 0.
__device__ __forceinline__ float relu_bits(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

typedef short short8 __attribute__((ext_vector_type(8)));

// Two FP32 values to a BF16 pair with round-to-nearest-even.  A two-wide
// vector conversion becomes one v_cvt_pk_bf16_f32 (element-wise conversions
// are converted one value at a time and then merged), and the compiler sees
// it, so it keeps the wait states a read of a matrix-core result needs.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t cvt_pk_bf16(float lo, float hi) {
  const f32x2 v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

// Hidden activations (accumulator layout) to the B operands of the next
// layer: chunk c takes blocks 2c and 2c+1 (16-bit operands) or element c&3
// of block c>>2 (FP32).  relu: clamp at zero, done on the 16-bit values two
// per instruction (rounding then clamping equals clamping then rounding).
template <int P, int W>
__device__ __forceinline__ void pack_hidden(const f32x4 act[W / 16], typename Prec<P>::Frag out[HidChunks<P, W>::n],
                                            bool relu) {
  constexpr int CHH = HidChunks<P, W>::n;
#pragma unroll
  for (int c = 0; c < CHH; ++c) {
    if constexpr (P == 1) {
      uint32_t w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = 2 * c + (q >> 1);
        w[q] = (m < W / 16) ? cvt_pk_bf16(act[m < W / 16 ? m : 0][2 * (q & 1)], act[m < W / 16 ? m : 0][2 * (q & 1) + 1])
                            : 0u;
      }
      short8 h = __builtin_bit_cast(short8, w);
      if (relu) h = __builtin_elementwise_max(h, (short8)0);
      out[c] = __builtin_bit_cast(typename Prec<P>::Frag, h);
    } else if constexpr (P == 2) {
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        const int m = 2 * c + (jj >> 2);
        const float v = (m < W / 16) ? act[m < W / 16 ? m : 0][jj & 3] : 0.0f;
        out[c][jj] = (typename Prec<P>::T)v;
      }
      if (relu) {
        short8 h = __builtin_bit_cast(short8, out[c]);
        h = __builtin_elementwise_max(h, (short8)0);
        out[c] = __builtin_bit_cast(typename Prec<P>::Frag, h);
      }
    } else {
      const float v = act[c >> 2][c & 3];
      out[c] = relu ? relu_bits(v) : v;
    }
  }
}

// Occupancy target (waves per SIMD) of the streaming MLP kernels: 4 for
// 16-bit operands and 32 inputs (their registers fit), 2 when the depth is
// fixed at compile time (the kernel then keeps every weight fragment in
// registers next to two tiles' activations), else no target.
__host__ __device__ constexpr int mlp_waves_per_eu(int P, int KIN, int NHC) {
  return P != 0 && NHC > 0 ? 2 : (P != 0 && KIN == 32 ? 4 : 1);
}

// Forward through the hidden layers over NB tiles at once: each weight
// fragment is read once for all NB tiles, and the NB accumulator chains are
// independent.  in[nb][c]: B operands of the encoded input; returns the last
// hidden pre-activations in act[nb][mb] (FP32, accumulator layout).  NHC > 0
// fixes the number of hidden layers at compile time (the layer loop unrolls
// and a kernel that never writes LDS can keep every weight in registers);
// NHC = 0 takes n_hidden.
template <int P, int KIN, int W, int NB, int NHC = 0>
__device__ __forceinline__ void mlp_hidden_fwd_nb(int n_hidden, const typename Prec<P>::Frag* __restrict__ lds_frag,
                                                  const typename Prec<P>::Frag in[NB][InChunks<P, KIN>::n],
                                                  f32x4 act[NB][W / 16]) {
  typedef WeightLayout<P, KIN, W> WL;
  typedef typename Prec<P>::Frag Frag;
  constexpr int MB = W / 16;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    f32x4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = zero4();
#pragma unroll
    for (int c = 0; c < WL::CH0; ++c) {
      const Frag a = lds_frag[(mb * WL::CH0 + c) * 64 + lane];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma(a, in[nb][c], acc[nb]);
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) act[nb][mb] = acc[nb];
  }
  auto layer = [&](int li) {
    Frag b[NB][WL::CHH];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) pack_hidden<P, W>(act[nb], b[nb], true);
    const Frag* base = lds_frag + (WL::FR0 + (li - 1) * WL::FRH) * 64;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      f32x4 acc[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = zero4();
#pragma unroll
      for (int c = 0; c < WL::CHH; ++c) {
        const Frag a = base[(mb * WL::CHH + c) * 64 + lane];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma(a, b[nb][c], acc[nb]);
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) act[nb][mb] = acc[nb];
    }
  };
  if constexpr (NHC > 0) {
#pragma unroll
    for (int li = 1; li < NHC; ++li) layer(li);
  } else {
    for (int li = 1; li < n_hidden; ++li) layer(li);
  }
}

// Output neuron: y = w_out . relu(z_last), then ReLU if relu_out; every lane
// of the sample gets y.  P = 0: FP32 dot product over the lane's neurons and
// a sum over the four lane groups; 16-bit operands: the output MFMA.
template <int P, int W>
__device__ __forceinline__ float mlp_output(const f32x4 zlast[W / 16], const float* __restrict__ lds_wout,
                                            bool relu_out) {
  float y;
  if constexpr (P == 0) {
    const int g = (threadIdx.x & 63) >> 4;
    float s = 0.0f;
#pragma unroll
    for (int mb = 0; mb < W / 16; ++mb)
#pragma unroll
      for (int j = 0; j < 4; ++j) s = __builtin_fmaf(lds_wout[16 * mb + 4 * g + j], relu_bits(zlast[mb][j]), s);
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    y = s;
  } else {
    typedef typename Prec<P>::Frag Frag;
    constexpr int CHH = HidChunks<P, W>::n;
    const int lane = threadIdx.x & 63;
    Frag b[CHH];
    pack_hidden<P, W>(zlast, b, true);
    const Frag* of = out_frags<P, W>(lds_wout);
    f32x4 acc = zero4();
#pragma unroll
    for (int c = 0; c < CHH; ++c) acc = mfma(of[c * 64 + lane], b[c], acc);
    y = acc[0];
  }
  return relu_out ? relu_bits(y) : y;
}

// ---------------------------------------------------------------------------
// Streaming evaluation: the wave walks groups of NB tiles; the inputs of the
// next group are loaded (ld) while the current group runs through the
// network, with two register buffers used in turn so that the loads stay in
// flight during the MFMA work.  cv turns loaded data into B operands; st
// receives y for (group, tile, lane) together with the group's loaded data.
// ---------------------------------------------------------------------------
template <int P, int KIN, int W, int NB, typename Raw, int NHC, class Ld, class Cv, class St>
__device__ __forceinline__ void mlp_stream(int n_hidden, bool relu_out, const typename Prec<P>::Frag* __restrict__ lds_frag,
                                           const float* __restrict__ lds_wout, int64_t t, int64_t step, int64_t end,
                                           Ld ld, Cv cv, St st) {
  typedef typename Prec<P>::Frag Frag;
  auto run = [&](int64_t grp, const Raw& r) {
    Frag in[NB][InChunks<P, KIN>::n];
    cv(r, in);
    f32x4 act[NB][W / 16];
    mlp_hidden_fwd_nb<P, KIN, W, NB, NHC>(n_hidden, lds_frag, in, act);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) st(grp, nb, mlp_output<P, W>(act[nb], lds_wout, relu_out), r);
  };
  if (t >= end) return;
  Raw a, b;
  ld(t, a);
  while (true) {
    int64_t tn = t + step;
    if (tn < end) ld(tn, b);
    run(t, a);
    t = tn;
    if (t >= end) break;
    tn = t + step;
    if (tn < end) ld(tn, a);
    run(t, b);
    t = tn;
    if (t >= end) break;
  }
}

// ---------------------------------------------------------------------------
// Encoding with one sample per lane (64 per wave).  All lanes work on the
// same level at a time, so the level's descriptor is uniform (scalar loads)
// and so is the dense/hashed choice.  Each lane writes its features, in the
// operand type, to its row of a per-wave LDS stage [64][pitch]; after
// wave_sync, stage_frags gives lane (n, g) the B operands of tile t (samples
// 16t..16t+15 of the wave's 64): features 32b + 8g + jj of sample 16t + n.
// The conversion to the operand type is the one feat_to_frag applies.
// ---------------------------------------------------------------------------
template <int P, int KIN>
struct Stage {
  typedef typename Prec<P>::T T;
  static constexpr int pitch = KIN + (int)(16 / sizeof(T));  // rows stay 16-byte aligned
  static constexpr size_t wave_bytes = (size_t)64 * pitch * sizeof(T);
};

// 8 consecutive operands of one row, as stored in LDS and in memory.
template <int P>
struct alignas(16) Oct {
  typename Prec<P>::T v[8];
};

// Encodes the lane's sample into its stage row; sink(sb, oct) also receives
// every 8-feature block (sb = block index), e.g. to store the encoding.
template <int P, int F, int KIN, typename TT, class Sink>
__device__ __forceinline__ void encode_row(const ModelDesc& md, const TT* __restrict__ table, float x, float y,
                                           float z, typename Prec<P>::T* row, Sink sink) {
  typedef typename Prec<P>::T T;
  constexpr int LPS = 8 / F;  // levels per 8-feature block
#pragma unroll
  for (int sb = 0; sb < KIN / 8; ++sb) {
    float v[8];
#pragma unroll
    for (int q = 0; q < LPS; ++q) {
      const int l = sb * LPS + q;
      float acc[F];
      if (l < md.L) {
        Corners cr;
        level_corners(md.lv[l], x, y, z, cr);
        gather_level<F>(cr, table, (uint32_t)(md.n_table / F), acc);
      } else {
#pragma unroll
        for (int f = 0; f < F; ++f) acc[f] = 0.0f;
      }
#pragma unroll
      for (int f = 0; f < F; ++f) v[q * F + f] = acc[f];
    }
    Oct<P> o;
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) o.v[jj] = (T)v[jj];
    *reinterpret_cast<Oct<P>*>(row + 8 * sb) = o;
    sink(sb, o);
  }
}

template <int P, int KIN>
__device__ __forceinline__ void stage_frags(const typename Prec<P>::T* stage, int t,
                                            typename Prec<P>::Frag in[InChunks<P, KIN>::n]) {
  typedef typename Prec<P>::Frag Frag;
  const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
  const typename Prec<P>::T* row = stage + (16 * t + n) * Stage<P, KIN>::pitch;
#pragma unroll
  for (int b = 0; b < KIN / 32; ++b) {
    const Oct<P> o = *reinterpret_cast<const Oct<P>*>(row + 32 * b + 8 * g);
    if constexpr (P) {
      in[b] = __builtin_bit_cast(Frag, o);
    } else {
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) in[8 * b + jj] = o.v[jj];
    }
  }
}

// Byte offset of the per-wave encoding stages behind the staged weights.
template <int P, int W>
__device__ __forceinline__ size_t stage_offset(size_t weight_bytes) {
  return (weight_bytes + wout_region_bytes<P, W>() + 15) & ~(size_t)15;
}

// The network on the wave's 64 staged samples (4 tiles, NB at a time); the
// lane receives y of its own sample (tile g, column n).
template <int P, int KIN, int W, int NB = 1>
__device__ __forceinline__ float mlp_wave64(int n_hidden, bool relu_out, const typename Prec<P>::Frag* __restrict__ lds_frag,
                                            const float* __restrict__ lds_wout, const typename Prec<P>::T* stage) {
  typedef typename Prec<P>::Frag Frag;
  const int g = (threadIdx.x & 63) >> 4;
  float yo = 0.0f;
#pragma unroll
  for (int h = 0; h < 4 / NB; ++h) {
    Frag in[NB][InChunks<P, KIN>::n];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) stage_frags<P, KIN>(stage, NB * h + nb, in[nb]);
    f32x4 act[NB][W / 16];
    mlp_hidden_fwd_nb<P, KIN, W, NB>(n_hidden, lds_frag, in, act);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const float y = mlp_output<P, W>(act[nb], lds_wout, relu_out);
      if (g == NB * h + nb) yo = y;
    }
  }
  return yo;
}

template <int P, int KIN>
__device__ __forceinline__ void feat_to_frag(const float feat[KIN / 32][8],
                                             typename Prec<P>::Frag out[InChunks<P, KIN>::n]) {
#pragma unroll
  for (int b = 0; b < KIN / 32; ++b) {
    if constexpr (P) {
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) out[b][jj] = (typename Prec<P>::T)feat[b][jj];
    } else {
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) out[8 * b + jj] = feat[b][jj];
    }
  }
}

}  // namespace ngvol
