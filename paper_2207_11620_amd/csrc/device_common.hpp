// Device-side building blocks shared by the ngvol kernels (gfx950).
//
// Everything here is compiled with -ffp-contract=off: every fused multiply-add
// is written out with __builtin_fmaf, so the binary32 geometry and the exact
// level floor below are reproducible operation by operation.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "plan.hpp"

namespace ngvol {

// ---------------------------------------------------------------------------
// Counter-based SplitMix64 (Steele, Lea and Flood 2014): output n of stream
// (seed, stream) is the n-th output of the generator started from state
// seed ^ (stream << 56).  Uniforms keep the top 24 bits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ float rng_u01(uint64_t seed, uint32_t stream, uint64_t index) {
  uint64_t s0 = seed ^ ((uint64_t)stream << 56);
  uint64_t r = sm64_mix(s0 + (index + 1ull) * 0x9E3779B97F4A7C15ull);
  return (float)(uint32_t)(r >> 40) * 0x1p-24f;
}

// Coordinate axis a of training sample i of step s (stream 3).
__device__ __forceinline__ float batch_coord(uint64_t seed, int64_t step, int64_t B, int64_t i, int a) {
  return rng_u01(seed, 3u, (uint64_t)(step * B * 3 + i * 3 + a));
}

__device__ __forceinline__ float clamp01(float x) { return fminf(fmaxf(x, 0.0f), 1.0f); }

// ---------------------------------------------------------------------------
// Level geometry along one axis (Section 3.1): p = x (N-1); the cell is
// c = min(floor(p), N-2) taken on the exact product, and w = p - c.
// In binary32: floor the rounded product, then use the exact sign of the
// fma residual x*s - c to step back when the product rounded up onto an
// integer; w = fma(x, s, -c) is the correctly rounded exact weight.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void level_axis(float x, float s, float cmax, int& c, float& w) {
  float p = x * s;
  float cf = floorf(p);
  float r = __builtin_fmaf(x, s, -cf);
  if (r < 0.0f) cf -= 1.0f;
  cf = fminf(cf, cmax);
  w = __builtin_fmaf(x, s, -cf);
  c = (int)cf;
}

// Slot of vertex v at a level: dense row-major when the level is dense, else
// the spatial hash (primes 1, 2654435761, 805459861) modulo the table size.
__device__ __forceinline__ uint32_t level_slot(const LevelDesc& lv, uint32_t vx, uint32_t vy, uint32_t vz) {
  if (lv.dense) return vx + (uint32_t)lv.N * (vy + (uint32_t)lv.N * vz);
  return (vx ^ (vy * 2654435761u) ^ (vz * 805459861u)) & lv.mask;
}

// Cell of a point at one level: the corner vertex c (lowest corner) per
// axis and the trilinear weights of the 8 corners, corner k = (k&1, (k>>1)&1,
// (k>>2)&1).
struct Cell {
  int c[3];
  float w[8];
};

__device__ __forceinline__ void level_cell(const LevelDesc& lv, float x, float y, float z, Cell& cl) {
  const float s = (float)(lv.N - 1);
  const float cmax = (float)(lv.N - 2);
  float wx, wy, wz;
  level_axis(x, s, cmax, cl.c[0], wx);
  level_axis(y, s, cmax, cl.c[1], wy);
  level_axis(z, s, cmax, cl.c[2], wz);
  const float ox = 1.0f - wx, oy = 1.0f - wy, oz = 1.0f - wz;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
    cl.w[k] = ((dx ? wx : ox) * (dy ? wy : oy)) * (dz ? wz : oz);
  }
}

struct Corners {
  uint32_t slot[8];  // with level offset
  float w[8];
};

__device__ __forceinline__ void level_corners(const LevelDesc& lv, float x, float y, float z, Corners& cr) {
  Cell cl;
  level_cell(lv, x, y, z, cl);
  const int cx = cl.c[0], cy = cl.c[1], cz = cl.c[2];
  // the slots of the 8 corners differ from the first by constants (dense) or
  // by the hash terms of y+1 and z+1, (v+1)*p = v*p + p (mod 2^32)
  if (lv.dense) {
    const uint32_t N = (uint32_t)lv.N, NN = N * N;
    const uint32_t b = lv.offset + (uint32_t)cx + N * ((uint32_t)cy + N * (uint32_t)cz);
#pragma unroll
    for (int k = 0; k < 8; ++k) cr.slot[k] = b + (k & 1) + ((k >> 1) & 1) * N + ((k >> 2) & 1) * NN;
  } else {
    const uint32_t hy0 = (uint32_t)cy * 2654435761u, hz0 = (uint32_t)cz * 805459861u;
    const uint32_t hy1 = hy0 + 2654435761u, hz1 = hz0 + 805459861u;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t vx = (uint32_t)cx + (k & 1);
      const uint32_t hy = (k & 2) ? hy1 : hy0, hz = (k & 4) ? hz1 : hz0;
      cr.slot[k] = lv.offset + ((vx ^ hy ^ hz) & lv.mask);
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) cr.w[k] = cl.w[k];
}

// Element at a 32-bit byte offset from a table base (tables are below 4 GB):
// the load takes the base in scalar registers and the offset in one vector
// register.
template <typename T>
__device__ __forceinline__ T load_at(const void* base, uint32_t off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}

// Raw table entries: F features of type TT, ED dwords.
template <int F, typename TT>
struct Entry {
  static constexpr int ED = F * (int)sizeof(TT) / 4;
};

template <int F, typename TT>
__device__ __forceinline__ void entry_values(const uint32_t* d, float v[F]) {
  if constexpr (std::is_same<TT, __half>::value) {
#pragma unroll
    for (int q = 0; q < F / 2; ++q) {
      const float2 u = __half22float2(__builtin_bit_cast(__half2, d[q]));
      v[2 * q] = u.x;
      v[2 * q + 1] = u.y;
    }
  } else {
#pragma unroll
    for (int f = 0; f < F; ++f) v[f] = __uint_as_float(d[f]);
  }
}

template <int ED>
__device__ __forceinline__ void load_entry(const void* __restrict__ base, uint32_t slot, uint32_t d[ED]) {
  const uint32_t off = slot * (uint32_t)(ED * 4);
  if constexpr (ED == 1) {
    d[0] = load_at<uint32_t>(base, off);
  } else if constexpr (ED == 2) {
    const uint2 t = load_at<uint2>(base, off);
    d[0] = t.x;
    d[1] = t.y;
  } else {
#pragma unroll
    for (int q = 0; q < ED; q += 4) {
      const uint4 t = load_at<uint4>(base, off + 4 * q);
      d[q] = t.x;
      d[q + 1] = t.y;
      d[q + 2] = t.z;
      d[q + 3] = t.w;
    }
  }
}

// Gather and interpolate the F features of one level:
// acc[f] = sum over corners k = 0..7, in that order, of w_k * entry_k[f].
// Corners 2p and 2p+1 differ only in x.  Their slots usually share an
// aligned 16-byte block: for dense levels they are adjacent, and since the
// x prime of the hash is 1, x and x+1 hash to slots that differ only in the
// low bits flipped by the increment.  When entries are at most 8 bytes each
// pair is read as that one block (one cache-line lookup instead of two) and
// only partners outside their block are loaded on their own, by the lanes
// that need them.  All loads are issued before any is used.  n_ent (entries
// of the whole table) keeps block reads inside the table: a wave with a
// block past the end takes the plain path.
template <int F, typename TT>
__device__ __forceinline__ void gather_level(const Corners& cr, const TT* __restrict__ table, uint32_t n_ent,
                                             float acc[F]) {
  constexpr int ED = Entry<F, TT>::ED;
  const void* base = table;
  float v[8][F];
  bool plain = true;
  if constexpr (ED <= 2) {
    constexpr uint32_t E = 4 / ED;  // entries per 16-byte block
    uint32_t b0[4];
    bool same[4];
    bool inside = true;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      b0[p] = cr.slot[2 * p] & ~(E - 1);
      same[p] = ((cr.slot[2 * p + 1] ^ cr.slot[2 * p]) & ~(E - 1)) == 0u;
    }
    if ((n_ent & (E - 1)) != 0) {  // only then can a block reach past the table's end
#pragma unroll
      for (int p = 0; p < 4; ++p) inside = inside && b0[p] + E <= n_ent;
    }
    if (__all(inside)) {
      plain = false;
      uint4 blk[4];
      uint32_t d1[4][ED];
#pragma unroll
      for (int p = 0; p < 4; ++p) blk[p] = load_at<uint4>(base, b0[p] * (uint32_t)(ED * 4));
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        if (!same[p]) {
          load_entry<ED>(base, cr.slot[2 * p + 1], d1[p]);
        } else {
#pragma unroll
          for (int q = 0; q < ED; ++q) d1[p][q] = 0u;
        }
      }
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        // words of the block by two bit tests of the entry's position (no
        // indexing, no branches)
        const uint32_t j0 = (cr.slot[2 * p] - b0[p]) * ED, j1 = (cr.slot[2 * p + 1] - b0[p]) * ED;
        uint32_t d0[ED], dd[ED];
        if constexpr (ED == 1) {
          const uint32_t l0 = (j0 & 1) ? blk[p].y : blk[p].x, h0 = (j0 & 1) ? blk[p].w : blk[p].z;
          const uint32_t l1 = (j1 & 1) ? blk[p].y : blk[p].x, h1 = (j1 & 1) ? blk[p].w : blk[p].z;
          d0[0] = (j0 & 2) ? h0 : l0;
          dd[0] = same[p] ? ((j1 & 2) ? h1 : l1) : d1[p][0];
        } else {
          d0[0] = j0 ? blk[p].z : blk[p].x;
          d0[1] = j0 ? blk[p].w : blk[p].y;
          dd[0] = same[p] ? (j1 ? blk[p].z : blk[p].x) : d1[p][0];
          dd[1] = same[p] ? (j1 ? blk[p].w : blk[p].y) : d1[p][1];
        }
        entry_values<F, TT>(d0, v[2 * p]);
        entry_values<F, TT>(dd, v[2 * p + 1]);
      }
    }
  }
  if (plain) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      uint32_t d[ED];
      load_entry<ED>(base, cr.slot[k], d);
      entry_values<F, TT>(d, v[k]);
    }
  }
#pragma unroll
  for (int f = 0; f < F; ++f) acc[f] = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int f = 0; f < F; ++f) acc[f] = __builtin_fmaf(cr.w[k], v[k][f], acc[f]);
}

// Scatter dL/dfeature of one level into the FP32 gradient of its table.
template <int F>
__device__ __forceinline__ void scatter_level(const Corners& cr, float* __restrict__ grad, const float d[F]) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
#pragma unroll
    for (int f = 0; f < F; ++f) {
      float v = cr.w[k] * d[f];
      if (v != 0.0f) atomicAdd(grad + (size_t)cr.slot[k] * F + f, v);
    }
  }
}

// Cell-centred trilinear sample with clamp-to-edge of a volume (x fastest).
template <typename T>
__device__ __forceinline__ float load_vox(const T* v, size_t i);
template <>
__device__ __forceinline__ float load_vox<float>(const float* v, size_t i) { return v[i]; }
template <>
__device__ __forceinline__ float load_vox<__half>(const __half* v, size_t i) { return __half2float(v[i]); }

template <typename T>
__device__ __forceinline__ float volume_sample(const T* __restrict__ vol, int dx, int dy, int dz, float x, float y,
                                               float z) {
  const float p[3] = {x, y, z};
  const int D[3] = {dx, dy, dz};
  int i0[3];
  float t[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float u = p[a] * (float)D[a] - 0.5f;
    float fl = floorf(u);
    fl = fminf(fmaxf(fl, 0.0f), (float)(D[a] - 2));
    t[a] = fminf(fmaxf(u - fl, 0.0f), 1.0f);
    i0[a] = (int)fl;
  }
  const size_t sy = (size_t)dx, sz = (size_t)dx * (size_t)dy;
  const size_t base = (size_t)i0[0] + sy * (size_t)i0[1] + sz * (size_t)i0[2];
  float c[8];
#pragma unroll
  for (int k = 0; k < 8; ++k)
    c[k] = load_vox<T>(vol, base + (size_t)(k & 1) + sy * (size_t)((k >> 1) & 1) + sz * (size_t)((k >> 2) & 1));
  // x, then y, then z
  float c00 = __builtin_fmaf(t[0], c[1] - c[0], c[0]);
  float c10 = __builtin_fmaf(t[0], c[3] - c[2], c[2]);
  float c01 = __builtin_fmaf(t[0], c[5] - c[4], c[4]);
  float c11 = __builtin_fmaf(t[0], c[7] - c[6], c[6]);
  float c0 = __builtin_fmaf(t[1], c10 - c00, c00);
  float c1 = __builtin_fmaf(t[1], c11 - c01, c01);
  return __builtin_fmaf(t[2], c1 - c0, c0);
}

// Orders a wave's LDS writes before its following LDS reads by other lanes
// of the same wave (no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave-wide sums (64 lanes).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace ngvol
