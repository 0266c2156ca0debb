// Spatial binning of sample coordinates.
//
// Random query or training coordinates make every table gather (and every
// gradient scatter) touch an unrelated cache line.  Reordering the samples
// so that consecutive 16-sample tiles lie in the same small cell of space
// lets neighbouring samples share the coarse and middle levels' lines in L2.
// The order of samples does not change any result of the method (queries
// are written back to their own slots; the training loss is a sum).
//
// The reorder is a counting sort by the Morton code of the sample's cell in
// a 2^k x 2^k x 2^k grid (k = 4 or 5): per-block LDS histograms, a per-bin
// prefix over blocks, one scan of the bin totals, and a scatter with LDS
// cursors; then each cell's records are regrouped by 512 sub-cells in LDS,
// so the order follows the Morton curve down to 1/256 of the domain.
#include "kernels.hpp"
#include "device_common.hpp"

namespace ngvol {

namespace {

constexpr int kSortThreads = 1024;

__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ __forceinline__ uint32_t cell_key(float x, float y, float z, int k) {
  const float s = (float)(1 << k);
  const uint32_t m = (1u << k) - 1u;
  const uint32_t qx = min((uint32_t)(clamp01(x) * s), m);
  const uint32_t qy = min((uint32_t)(clamp01(y) * s), m);
  const uint32_t qz = min((uint32_t)(clamp01(z) * s), m);
  return spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2);
}

// Coordinates of sample i: explicit array, or the training-batch generator.
struct Src {
  const float* xyz;
  uint64_t seed;
  int64_t step, B;
  __device__ __forceinline__ void get(int64_t i, float& x, float& y, float& z) const {
    if (xyz) {
      x = xyz[3 * i];
      y = xyz[3 * i + 1];
      z = xyz[3 * i + 2];
    } else {
      x = batch_coord(seed, step, B, i, 0);
      y = batch_coord(seed, step, B, i, 1);
      z = batch_coord(seed, step, B, i, 2);
    }
  }
};

__global__ void __launch_bounds__(kSortThreads) k_bin_hist(Src src, int64_t n, int k, int64_t chunk,
                                                           uint32_t* __restrict__ counts) {
  extern __shared__ uint32_t hist[];
  const int nb = 1 << (3 * k);
  for (int b = threadIdx.x; b < nb; b += blockDim.x) hist[b] = 0u;
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  // 4 samples per thread per round, their coordinates loaded together
  for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += 4 * (int64_t)blockDim.x) {
    uint32_t key[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = i0 + (int64_t)u * blockDim.x;
      float x = 0.0f, y = 0.0f, z = 0.0f;
      if (i < hi) src.get(i, x, y, z);
      key[u] = cell_key(x, y, z, k);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + (int64_t)u * blockDim.x < hi) atomicAdd(hist + key[u], 1u);
  }
  __syncthreads();
  uint32_t* dst = counts + (size_t)blockIdx.x * nb;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) dst[b] = hist[b];
}

// counts[blk][bin] <- exclusive prefix over blocks; totals[bin] <- sum.
// The counts of a bin are read kPrefixBatch at a time, so their loads are
// in flight together rather than one after another.
constexpr int kPrefixBatch = 16;

__global__ void __launch_bounds__(256) k_bin_prefix(uint32_t* __restrict__ counts, int blocks, int nb,
                                                    uint32_t* __restrict__ totals) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  uint32_t run = 0;
  for (int k0 = 0; k0 < blocks; k0 += kPrefixBatch) {
    uint32_t v[kPrefixBatch];
#pragma unroll
    for (int u = 0; u < kPrefixBatch; ++u) v[u] = k0 + u < blocks ? counts[(size_t)(k0 + u) * nb + b] : 0u;
#pragma unroll
    for (int u = 0; u < kPrefixBatch; ++u) {
      if (k0 + u < blocks) counts[(size_t)(k0 + u) * nb + b] = run;
      run += v[u];
    }
  }
  totals[b] = run;
}

// Exclusive scan of the bin totals, one block; each thread owns a run of
// consecutive bins, read in batches.
__global__ void __launch_bounds__(kSortThreads) k_bin_scan(const uint32_t* __restrict__ totals, int nb,
                                                           uint32_t* __restrict__ offsets) {
  __shared__ uint32_t part[kSortThreads];
  const int per = (nb + kSortThreads - 1) / kSortThreads;
  const int lo = threadIdx.x * per;
  uint32_t s = 0;
  for (int i0 = 0; i0 < per; i0 += kPrefixBatch) {
    uint32_t v[kPrefixBatch];
#pragma unroll
    for (int u = 0; u < kPrefixBatch; ++u) v[u] = (i0 + u < per && lo + i0 + u < nb) ? totals[lo + i0 + u] : 0u;
#pragma unroll
    for (int u = 0; u < kPrefixBatch; ++u) s += v[u];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int d = 1; d < kSortThreads; d <<= 1) {
    const uint32_t v = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - s;  // exclusive
  for (int i0 = 0; i0 < per; i0 += kPrefixBatch) {
    uint32_t v[kPrefixBatch];
#pragma unroll
    for (int u = 0; u < kPrefixBatch; ++u) v[u] = (i0 + u < per && lo + i0 + u < nb) ? totals[lo + i0 + u] : 0u;
#pragma unroll
    for (int u = 0; u < kPrefixBatch; ++u) {
      if (i0 + u < per && lo + i0 + u < nb) offsets[lo + i0 + u] = run;
      run += v[u];
    }
  }
}

// Scatter one 16-byte record per sample: (x, y, z, aux), where aux is the
// original index (queries, as integer bits) or the target value (training:
// explicit or sampled from the volume).
template <typename VT>
__global__ void __launch_bounds__(kSortThreads) k_bin_scatter(Src src, int64_t n, int k, int64_t chunk,
                                                              const uint32_t* __restrict__ counts,
                                                              const uint32_t* __restrict__ offsets,
                                                              float4* __restrict__ out, bool with_target,
                                                              const float* __restrict__ target_in,
                                                              const VT* __restrict__ vol, int dx, int dy, int dz) {
  extern __shared__ uint32_t cur[];
  const int nb = 1 << (3 * k);
  const uint32_t* mine = counts + (size_t)blockIdx.x * nb;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) cur[b] = offsets[b] + mine[b];
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  if (!with_target) {
    // queries: 4 per thread per round, so that their loads and their cursor
    // increments are in flight together
    for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += 4 * (int64_t)blockDim.x) {
      float4 r[4];
      uint32_t key[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = i0 + (int64_t)u * blockDim.x;
        float x = 0.0f, y = 0.0f, z = 0.0f;
        if (i < hi) src.get(i, x, y, z);
        r[u] = make_float4(x, y, z, __uint_as_float((uint32_t)i));
        key[u] = cell_key(x, y, z, k);
      }
      uint32_t pos[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i0 + (int64_t)u * blockDim.x < hi) pos[u] = atomicAdd(cur + key[u], 1u);
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i0 + (int64_t)u * blockDim.x < hi) out[pos[u]] = r[u];
    }
    return;
  }
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    float x, y, z;
    src.get(i, x, y, z);
    const uint32_t pos = atomicAdd(cur + cell_key(x, y, z, k), 1u);
    const float aux = target_in ? target_in[i] : volume_sample<VT>(vol, dx, dy, dz, x, y, z);
    out[pos] = make_float4(x, y, z, aux);
  }
}

// Within-cell refinement: the records of one cell are regrouped by the next
// SB bits per axis of their position (2^(3 SB) sub-cells, Morton order) with
// an LDS counting sort, so the final order follows the Morton curve down to
// cells of 2^-(k+SB) per axis; the order inside a sub-cell is arbitrary.
// Cells with more records than fit are left as they are (still grouped).
template <int SB>
struct Refine {
  static constexpr int bins = 1 << (3 * SB);
  static constexpr int threads = SB == 3 ? 512 : 1024;
  static constexpr int cap = SB == 3 ? 2048 : 6144;  // records of one cell held in LDS
  static constexpr int per = bins / threads;          // bins per thread in the scan
};

template <int SB>
__global__ void __launch_bounds__(Refine<SB>::threads) k_bin_refine(float4* __restrict__ rec,
                                                                    const uint32_t* __restrict__ totals,
                                                                    const uint32_t* __restrict__ offsets, int k,
                                                                    int n_cells) {
  typedef Refine<SB> R;
  __shared__ float4 buf[R::cap];
  __shared__ uint16_t key[R::cap];
  __shared__ uint16_t rank[R::cap];
  __shared__ uint32_t hist[R::bins];
  __shared__ uint32_t wsum[R::threads / 64];
  const float scale = (float)(1 << (k + SB));  // cells hold 2^-k per axis; SB more bits each
  const uint32_t top = (1u << (k + SB)) - 1u;
  const uint32_t low = (1u << SB) - 1u;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // each workgroup walks several cells
  for (int cell = blockIdx.x; cell < n_cells; cell += gridDim.x) {
    const uint32_t cnt = totals[cell];
    if (cnt < 2 || cnt > (uint32_t)R::cap) continue;  // uniform over the workgroup
    const uint32_t base = offsets[cell];
    for (int b = threadIdx.x; b < R::bins; b += R::threads) hist[b] = 0u;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < cnt; i += R::threads) {
      const float4 r = rec[base + i];
      buf[i] = r;
      const uint32_t qx = min((uint32_t)(clamp01(r.x) * scale), top) & low;
      const uint32_t qy = min((uint32_t)(clamp01(r.y) * scale), top) & low;
      const uint32_t qz = min((uint32_t)(clamp01(r.z) * scale), top) & low;
      const uint32_t kk = spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2);
      key[i] = (uint16_t)kk;
      rank[i] = (uint16_t)atomicAdd(hist + kk, 1u);
    }
    __syncthreads();
    // exclusive scan of the sub-cell counts: each thread owns `per`
    // consecutive bins; their sums are scanned within waves by shuffles,
    // then across the wave totals
    uint32_t v[R::per];
    uint32_t own = 0;
#pragma unroll
    for (int j = 0; j < R::per; ++j) {
      v[j] = hist[threadIdx.x * R::per + j];
      own += v[j];
    }
    uint32_t inc = own;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t t = __shfl_up(inc, d, 64);
      if (lane >= d) inc += t;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t run = inc - own;
#pragma unroll
    for (int w = 0; w < R::threads / 64; ++w) run += w < wave ? wsum[w] : 0u;
#pragma unroll
    for (int j = 0; j < R::per; ++j) {
      hist[threadIdx.x * R::per + j] = run;
      run += v[j];
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < cnt; i += R::threads) rec[base + hist[key[i]] + rank[i]] = buf[i];
    __syncthreads();  // buf, key and hist are reused by the next cell
  }
}

}  // namespace

hipError_t launch_count_offsets(uint32_t* counts, int blocks, int nb, uint32_t* totals, uint32_t* offsets,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_bin_prefix, dim3((nb + 255) / 256), dim3(256), 0, st, counts, blocks, nb, totals);
  hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(kSortThreads), 0, st, totals, nb, offsets);
  return hipGetLastError();
}

BinPlan bin_plan(const ngvol_plan* plan, int64_t n) {
  BinPlan bp{};
  if (n < ((int64_t)1 << 15)) return bp;  // too small to pay off
  // 4096 cells, refined by 3 bits per axis (by 4 from 2^22 queries: cells
  // of about 4096 records, written in runs of ~16 by each block)
  bp.k = 4;
  bp.sb = n >= ((int64_t)1 << 22) ? 4 : 3;
  bp.n_bins = 1 << (3 * bp.k);
  int64_t g = (n + 4095) / 4096;
  if (g > plan->cus) g = plan->cus;
  if (g < 1) g = 1;
  bp.blocks = (int)g;
  bp.chunk = (n + g - 1) / g;
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  bp.rec_off = 0;  // float4 records (x, y, z, aux)
  bp.counts_off = up((size_t)n * 16);
  bp.totals_off = bp.counts_off + up((size_t)bp.blocks * bp.n_bins * 4);
  bp.offsets_off = bp.totals_off + up((size_t)bp.n_bins * 4);
  bp.bytes = bp.offsets_off + up((size_t)bp.n_bins * 4);
  bp.split = use_split(plan, n);
  if (bp.split) {
    bp.planes_off = bp.bytes;
    bp.idx_off = bp.planes_off + up(split_planes_bytes(plan, n));
    bp.bytes = bp.idx_off + up((size_t)split_slab(plan, n) * 4);
  }
  return bp;
}

hipError_t launch_bin(const ngvol_plan* plan, const BinPlan& bp, const float* xyz, const BatchArgs* ba, int64_t n,
                      void* ws, hipStream_t st) {
  char* base = reinterpret_cast<char*>(ws);
  float4* rec = reinterpret_cast<float4*>(base + bp.rec_off);
  uint32_t* counts = reinterpret_cast<uint32_t*>(base + bp.counts_off);
  uint32_t* totals = reinterpret_cast<uint32_t*>(base + bp.totals_off);
  uint32_t* offsets = reinterpret_cast<uint32_t*>(base + bp.offsets_off);
  Src src{xyz, 0, 0, n};
  if (ba) {
    src.xyz = ba->xyz;
    src.seed = ba->seed;
    src.step = ba->step;  // training batches are not regrouped (see the training workspace)
    src.B = ba->B;
  }
  const size_t lds = (size_t)bp.n_bins * 4;
  hipLaunchKernelGGL(k_bin_hist, dim3(bp.blocks), dim3(kSortThreads), lds, st, src, n, bp.k, bp.chunk, counts);
  launch_count_offsets(counts, bp.blocks, bp.n_bins, totals, offsets, st);
  if (!ba) {
    hipLaunchKernelGGL(k_bin_scatter<float>, dim3(bp.blocks), dim3(kSortThreads), lds, st, src, n, bp.k, bp.chunk,
                       counts, offsets, rec, false, nullptr, nullptr, 1, 1, 1);
    if (bp.sb == 3) {
      int rgrid = plan->cus * 4;  // workgroups walking cells
      if (rgrid > bp.n_bins) rgrid = bp.n_bins;
      hipLaunchKernelGGL(k_bin_refine<3>, dim3(rgrid), dim3(Refine<3>::threads), 0, st, rec, totals, offsets, bp.k,
                         bp.n_bins);
    } else {
      int rgrid = plan->cus;
      if (rgrid > bp.n_bins) rgrid = bp.n_bins;
      hipLaunchKernelGGL(k_bin_refine<4>, dim3(rgrid), dim3(Refine<4>::threads), 0, st, rec, totals, offsets, bp.k,
                         bp.n_bins);
    }
  } else if (ba->xyz || ba->vdtype != NGVOL_DT_F16) {
    hipLaunchKernelGGL(k_bin_scatter<float>, dim3(bp.blocks), dim3(kSortThreads), lds, st, src, n, bp.k, bp.chunk,
                       counts, offsets, rec, true, ba->target, reinterpret_cast<const float*>(ba->volume), ba->dims[0],
                       ba->dims[1], ba->dims[2]);
  } else {
    hipLaunchKernelGGL(k_bin_scatter<__half>, dim3(bp.blocks), dim3(kSortThreads), lds, st, src, n, bp.k, bp.chunk,
                       counts, offsets, rec, true, nullptr, reinterpret_cast<const __half*>(ba->volume), ba->dims[0],
                       ba->dims[1], ba->dims[2]);
  }
  return hipGetLastError();
}

}  // namespace ngvol
