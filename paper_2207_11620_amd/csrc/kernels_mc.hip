// Macro-cells (Section 5.3): value ranges built from samples, and the
// maximum opacity of each cell under a transfer function, which the ray
// marcher uses to skip empty space.
#include "device_common.hpp"
#include "kernels.hpp"
#include "render.hpp"

namespace ngvol {

namespace {

__global__ void __launch_bounds__(256) k_mc_reset(uint32_t* __restrict__ range, int64_t n_cells) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells; c += stride) {
    range[2 * c] = 0xFFFFFFFFu;
    range[2 * c + 1] = 0u;
  }
}

__global__ void __launch_bounds__(256) k_mc_update(McGeom g, const float* __restrict__ xyz,
                                                   const float* __restrict__ values, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t c = mc_index(g, clamp01(xyz[3 * i]), clamp01(xyz[3 * i + 1]), clamp01(xyz[3 * i + 2]));
    mc_extend(g.range, c, values[i]);
  }
}

__device__ __forceinline__ float key_value(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// alpha of the shading's transfer function at v (u and its fraction in
// binary32, as the renderer forms them)
__device__ __forceinline__ float tf_alpha(const float* lut, float v) {
  const float c = fminf(fmaxf(v, 0.0f), 1.0f);
  const float u = 255.0f * c;
  const float fi = fminf(floorf(u), 254.0f);
  const int i0 = (int)fi;
  const float fr = u - fi;
  return __builtin_fmaf(fr, lut[4 * (i0 + 1) + 3] - lut[4 * i0 + 3], lut[4 * i0 + 3]);
}

__global__ void __launch_bounds__(256) k_mc_opacity(const uint32_t* __restrict__ range, float* __restrict__ mu,
                                                    int64_t n_cells, const float* __restrict__ lut) {
  __shared__ float la[256];
  __shared__ float lut4[1024];
  for (int t = threadIdx.x; t < 1024; t += blockDim.x) lut4[t] = lut[t];
  __syncthreads();
  for (int t = threadIdx.x; t < 256; t += blockDim.x) la[t] = lut4[4 * t + 3];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells; c += stride) {
    const uint32_t klo = range[2 * c], khi = range[2 * c + 1];
    if (klo > khi) {  // no sample has reached the cell
      mu[c] = 0.0f;
      continue;
    }
    const float lo = key_value(klo), hi = key_value(khi);
    float m = fmaxf(tf_alpha(lut4, lo), tf_alpha(lut4, hi));
    const float ul = 255.0f * fminf(fmaxf(lo, 0.0f), 1.0f);
    const float uh = 255.0f * fminf(fmaxf(hi, 0.0f), 1.0f);
    // nodes strictly inside (ul, uh)
    const int i0 = (int)floorf(ul) + 1;
    const int i1 = (int)ceilf(uh) - 1;
    for (int i = i0 < 0 ? 0 : i0; i <= (i1 > 255 ? 255 : i1); ++i) m = fmaxf(m, la[i]);
    mu[c] = m;
  }
}

int64_t mc_cells(const McGeom& g) { return (int64_t)g.m[0] * g.m[1] * g.m[2]; }

unsigned grid_of(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

hipError_t launch_mc_reset(const McGeom& g, hipStream_t st) {
  const int64_t n = mc_cells(g);
  hipLaunchKernelGGL(k_mc_reset, dim3(grid_of(n)), dim3(256), 0, st, g.range, n);
  return hipGetLastError();
}

hipError_t launch_mc_update(const McGeom& g, const float* xyz, const float* values, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mc_update, dim3(grid_of(n)), dim3(256), 0, st, g, xyz, values, n);
  return hipGetLastError();
}

hipError_t launch_mc_opacity(const McGeom& g, const float* lut, hipStream_t st) {
  const int64_t n = mc_cells(g);
  hipLaunchKernelGGL(k_mc_opacity, dim3(grid_of(n)), dim3(256), 0, st, g.range, const_cast<float*>(g.mu), n, lut);
  return hipGetLastError();
}

}  // namespace ngvol
