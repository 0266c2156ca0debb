// Device-side building blocks shared by the ngvol kernels (gfx950).
//
// Everything here is compiled with -ffp-contract=off: every fused multiply-add
// is written out with __builtin_fmaf, so the binary32 geometry and the exact
// level floor below are reproducible operation by operation.
#pragma once

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

struct Corners {
  uint32_t slot[8];  // with level offset
  float w[8];
};

__device__ __forceinline__ void level_corners(const LevelDesc& lv, float x, float y, float z, Corners& cr) {
  const float s = (float)(lv.N - 1);
  const float cmax = (float)(lv.N - 2);
  int cx, cy, cz;
  float wx, wy, wz;
  level_axis(x, s, cmax, cx, wx);
  level_axis(y, s, cmax, cy, wy);
  level_axis(z, s, cmax, cz, wz);
  const float ox = 1.0f - wx, oy = 1.0f - wy, oz = 1.0f - wz;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
    cr.slot[k] = lv.offset + level_slot(lv, (uint32_t)(cx + dx), (uint32_t)(cy + dy), (uint32_t)(cz + dz));
    cr.w[k] = ((dx ? wx : ox) * (dy ? wy : oy)) * (dz ? wz : oz);
  }
}

// Gather and interpolate the F features of one level.
template <int F>
__device__ __forceinline__ void gather_level(const Corners& cr, const float* __restrict__ table, float acc[F]) {
#pragma unroll
  for (int f = 0; f < F; ++f) acc[f] = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float* e = table + (size_t)cr.slot[k] * F;
    float v[F];
    if constexpr (F == 1) {
      v[0] = e[0];
    } else if constexpr (F == 2) {
      float2 t = *reinterpret_cast<const float2*>(e);
      v[0] = t.x;
      v[1] = t.y;
    } else {
#pragma unroll
      for (int q = 0; q < F; q += 4) {
        float4 t = *reinterpret_cast<const float4*>(e + q);
        v[q] = t.x;
        v[q + 1] = t.y;
        v[q + 2] = t.z;
        v[q + 3] = t.w;
      }
    }
#pragma unroll
    for (int f = 0; f < F; ++f) acc[f] = __builtin_fmaf(cr.w[k], v[f], acc[f]);
  }
}

template <int F>
__device__ __forceinline__ void gather_level(const Corners& cr, const __half* __restrict__ table, float acc[F]) {
#pragma unroll
  for (int f = 0; f < F; ++f) acc[f] = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const __half* e = table + (size_t)cr.slot[k] * F;
    float v[F];
    if constexpr (F == 1) {
      v[0] = __half2float(e[0]);
    } else if constexpr (F == 2) {
      __half2 t = *reinterpret_cast<const __half2*>(e);
      float2 u = __half22float2(t);
      v[0] = u.x;
      v[1] = u.y;
    } else {
#pragma unroll
      for (int q = 0; q < F; q += 4) {
        uint2 raw = *reinterpret_cast<const uint2*>(e + q);
        __half2 a = *reinterpret_cast<__half2*>(&raw.x);
        __half2 b = *reinterpret_cast<__half2*>(&raw.y);
        float2 ua = __half22float2(a), ub = __half22float2(b);
        v[q] = ua.x;
        v[q + 1] = ua.y;
        v[q + 2] = ub.x;
        v[q + 3] = ub.y;
      }
    }
#pragma unroll
    for (int f = 0; f < F; ++f) acc[f] = __builtin_fmaf(cr.w[k], v[f], acc[f]);
  }
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
