// Ray geometry shared by the renderers, in binary32 with one rounding per
// operation (no FMA), so that sample positions are reproducible bit for bit.
#pragma once

#include "device_common.hpp"
#include "kernels.hpp"

namespace ngvol {

struct RayGeom {
  float o[3], d[3], t0, j;
  uint32_t n;
};

// Unit direction v / |v|, |v| = sqrt((v0^2 + v1^2) + v2^2).
__device__ __forceinline__ void unit3(const float v[3], float out[3]) {
  const float n2 = __fadd_rn(__fadd_rn(__fmul_rn(v[0], v[0]), __fmul_rn(v[1], v[1])), __fmul_rn(v[2], v[2]));
  const float nrm = __fsqrt_rn(n2);
#pragma unroll
  for (int a = 0; a < 3; ++a) out[a] = __fdiv_rn(v[a], nrm);
}

// Unit direction of the camera ray through the centre of pixel (px, py):
// W + (px + 1/2) U + (py + 1/2) V, normalised.  cam = {o, U, V, W}.
__device__ __forceinline__ void camera_dir(const float* cam, int px, int py, float d[3]) {
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  float dir[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float t1 = __fmul_rn(fx, cam[3 + a]);
    const float t2 = __fadd_rn(cam[9 + a], t1);
    const float t3 = __fmul_rn(fy, cam[6 + a]);
    dir[a] = __fadd_rn(t2, t3);
  }
  unit3(dir, d);
}

// Slab test of o + t d against [0,1]^3: t_near = max(t_min, 0) and t_far.
__device__ __forceinline__ void slab(const float o[3], const float d[3], float& tn, float& tf) {
  float tmin = -INFINITY, tmax = INFINITY;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float inv = __fdiv_rn(1.0f, d[a]);
    const float ta = __fmul_rn(__fsub_rn(0.0f, o[a]), inv);
    const float tb = __fmul_rn(__fsub_rn(1.0f, o[a]), inv);
    tmin = fmaxf(tmin, fminf(ta, tb));
    tmax = fminf(tmax, fmaxf(ta, tb));
  }
  tn = fmaxf(tmin, 0.0f);
  tf = tmax;
}

// Ray from o along the unit direction d with jitter j: samples
// t_k = t_near + (k + j) dt for k < n = max(0, ceil((t_far - t_near)/dt - j)).
__device__ __forceinline__ RayGeom ray_from(const float o[3], const float d[3], float j, float dt) {
  RayGeom r;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r.o[a] = o[a];
    r.d[a] = d[a];
  }
  float tn, tf;
  slab(o, d, tn, tf);
  r.t0 = tn;
  r.j = j;
  r.n = 0;
  if (tn < tf) {
    const float q = __fdiv_rn(__fsub_rn(tf, tn), dt);
    // a unit-cube chord is at most sqrt(3) long; more than 2^24 steps (or a
    // NaN span) means a degenerate ray, which gets no samples
    if (q <= 16777216.0f) {
      const float c = ceilf(__fsub_rn(q, j));
      if (c > 0.0f) r.n = (uint32_t)c;
    }
  }
  return r;
}

// Camera ray of pixel (px, py), jittered by stream 5 of the counter generator.
__device__ __forceinline__ RayGeom make_ray(const float* cam, int W, int px, int py, uint32_t seed, float dt) {
  float d[3];
  camera_dir(cam, px, py, d);
  const float j = rng_u01((uint64_t)seed, 5u, (uint64_t)py * (uint64_t)W + (uint64_t)px);
  return ray_from(cam, d, j, dt);
}

__device__ __forceinline__ void ray_point(const RayGeom& r, uint32_t k, float dt, float& x, float& y, float& z) {
  const float kj = __fadd_rn((float)k, r.j);
  const float t = __fadd_rn(r.t0, __fmul_rn(kj, dt));
  x = __fadd_rn(r.o[0], __fmul_rn(t, r.d[0]));
  y = __fadd_rn(r.o[1], __fmul_rn(t, r.d[1]));
  z = __fadd_rn(r.o[2], __fmul_rn(t, r.d[2]));
}

__device__ __forceinline__ uint32_t sample_cell(const RayGeom& r, uint32_t k, float dt, const McGeom& g) {
  float x, y, z;
  ray_point(r, k, dt, x, y, z);
  return mc_index(g, clamp01(x), clamp01(y), clamp01(z));
}

// Transfer function at the network value y: v = clamp(y, 0, 1), u = 255 v,
// i = min(floor(u), 254), linear blend of table rows i and i + 1.
__device__ __forceinline__ void tf_lookup(const float* lut, float y, float c4[4]) {
  const float val = fminf(fmaxf(y, 0.0f), 1.0f);
  const float u = 255.0f * val;
  const float fi = fminf(floorf(u), 254.0f);
  const int i0 = (int)fi;
  const float fr = u - fi;
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) c4[ch] = __builtin_fmaf(fr, lut[4 * (i0 + 1) + ch] - lut[4 * i0 + ch], lut[4 * i0 + ch]);
}

// Work queue of the persistent renderers: the frame is cut into kBands
// bands of pixels, one per XCD; workgroups take pixels from the band of
// their XCD (workgroup id mod 8) and steal from the others once it is empty.
constexpr int kBands = 8;

// Fetch the next pixel: own band first, then steal from the others.
__device__ __forceinline__ int32_t fetch_pixel(unsigned int* queue, int band0, int64_t n_pix) {
  for (int i = 0; i < kBands; ++i) {
    const int b = (band0 + i) % kBands;
    const int64_t lo = n_pix * b / kBands, hi = n_pix * (b + 1) / kBands;
    if (__hip_atomic_load(queue + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= (unsigned)(hi - lo)) continue;
    const unsigned q = atomicAdd(queue + b, 1u);
    if ((int64_t)q < hi - lo) return (int32_t)(lo + q);
  }
  return -1;
}

// Wave-level pixel pool: the frame is cut into 8x8-pixel tiles taken one at
// a time by a wave from the banded queue above (one atomic per 64 pixels),
// so the rays a wave works on at any time are neighbours and their samples
// share cache lines.  The pool is wave-uniform state kept in registers.
struct PixelPool {
  int64_t tile;  // current tile, -1 before the first
  int pos;       // next pixel of the tile (64: used up)
  bool done;     // the queue is empty
};

__device__ __forceinline__ PixelPool pool_init() { return PixelPool{-1, 64, false}; }

// Gives every lane with `want` set a pixel of the wave's tiles, in lane
// order (-1 once the frame has no pixels left).  Called by the whole wave.
__device__ inline int32_t pool_take(PixelPool& pool, bool want, unsigned int* queue, int band0, int W, int H) {
  const int lane = threadIdx.x & 63;
  const int tiles_x = (W + 7) >> 3, tiles_y = (H + 7) >> 3;
  const int64_t n_tiles = (int64_t)tiles_x * tiles_y;
  int32_t got = -1;
  unsigned long long m = __ballot(want);
  while (m && !pool.done) {
    if (pool.pos >= 64) {
      int32_t t = -1;
      if (lane == 0) t = fetch_pixel(queue, band0, n_tiles);
      t = __builtin_amdgcn_readfirstlane(t);
      if (t < 0) {
        pool.done = true;
        break;
      }
      pool.tile = t;
      pool.pos = 0;
    }
    const int w = pool.pos++;
    const int px = (int)(pool.tile % tiles_x) * 8 + (w & 7), py = (int)(pool.tile / tiles_x) * 8 + (w >> 3);
    if (px >= W || py >= H) continue;  // outside the frame (edge tile)
    const int leader = __ffsll(m) - 1;
    if (lane == leader) got = py * W + px;
    m &= m - 1;
  }
  return got;
}

}  // namespace ngvol
