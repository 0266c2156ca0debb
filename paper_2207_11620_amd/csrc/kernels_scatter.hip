// Encoding backward as a bucketed scatter (Section 3.1 encoding, reversed):
// grad_table[slot][f] += w_corner * dL/dfeature[l*F + f] for every sample,
// level and corner.
//
// FP32 atomic adds to device memory run at a fixed rate on this GPU
// whatever the footprint, so the scatter avoids them.  Table entries
// (all levels, concatenated) are cut into buckets of 2^bshift entries whose
// F features fill 32 KB of LDS:
//   1. count: per-block LDS histograms of the bucket of every contribution;
//   2. block prefix and scan of the counts (shared with the spatial sort);
//   3. fill: each contribution is written as a packed record
//      (entry, w*d[0..F-1]) at its bucket's next position (LDS cursors);
//   4. reduce: one workgroup per (bucket, chunk of records) - a work list
//      built on the device from the bucket sizes, so no workgroup is empty -
//      accumulates the records in LDS (compare-and-swap adds) and adds the
//      bucket's entries into the gradient, with plain stores when the bucket
//      fits one chunk (it owns those entries), with atomics only when a
//      heavily hit bucket is split.
#include "kernels.hpp"
#include "device_common.hpp"
#include "lds_add.hpp"

namespace ngvol {

namespace {

constexpr int kScThreads = 256;
constexpr int kReduceThreads = 1024;
constexpr int64_t kChunkAdds = 1 << 17;  // LDS feature adds per reduce work item
constexpr int kUnroll = 8;  // records per thread per round in the reduce

struct Coords {
  const float* xyz;
  uint64_t seed;
  int64_t step, B;
  const int64_t* step_ptr;
  __device__ __forceinline__ void resolve() {
    if (step_ptr) step = *step_ptr;
  }
  __device__ __forceinline__ void get(int64_t i, float& x, float& y, float& z) const {
    if (xyz) {
      x = clamp01(xyz[3 * i]);
      y = clamp01(xyz[3 * i + 1]);
      z = clamp01(xyz[3 * i + 2]);
    } else {
      x = batch_coord(seed, step, B, i, 0);
      y = batch_coord(seed, step, B, i, 1);
      z = batch_coord(seed, step, B, i, 2);
    }
  }
};

__global__ void __launch_bounds__(kScThreads) k_sc_count(ModelDesc md, Coords src, int64_t B, int64_t chunk,
                                                         int bshift, int nb, uint32_t* __restrict__ counts) {
  extern __shared__ uint32_t hist[];
  src.resolve();
  for (int b = threadIdx.x; b < nb; b += blockDim.x) hist[b] = 0u;
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < B ? lo + chunk : B;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    float x, y, z;
    src.get(i, x, y, z);
    for (int l = 0; l < md.L; ++l) {
      Corners cr;
      level_corners(md.lv[l], x, y, z, cr);
#pragma unroll
      for (int k = 0; k < 8; ++k) atomicAdd(hist + (cr.slot[k] >> bshift), 1u);
    }
  }
  __syncthreads();
  uint32_t* dst = counts + (size_t)blockIdx.x * nb;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) dst[b] = hist[b];
}

// Record of one contribution: dword 0 = entry index, dwords 1..F = values,
// packed (12 bytes for F = 2).
template <int F>
struct Rec {
  static constexpr int dwords = 1 + F;
};

struct alignas(4) Dw3 {
  uint32_t x, y, z;
};

template <int N>
__device__ __forceinline__ void store_dwords(uint32_t* __restrict__ dst, const uint32_t* w) {
  if constexpr (N == 3) {
    *reinterpret_cast<Dw3*>(dst) = Dw3{w[0], w[1], w[2]};
  } else {
#pragma unroll
    for (int q = 0; q < N; ++q) dst[q] = w[q];
  }
}

template <int N>
__device__ __forceinline__ void load_dwords(const uint32_t* __restrict__ src, uint32_t* w) {
  if constexpr (N == 3) {
    const Dw3 t = *reinterpret_cast<const Dw3*>(src);
    w[0] = t.x;
    w[1] = t.y;
    w[2] = t.z;
  } else {
#pragma unroll
    for (int q = 0; q < N; ++q) w[q] = src[q];
  }
}

template <int F>
__global__ void __launch_bounds__(kScThreads) k_sc_fill(ModelDesc md, Coords src, int64_t B, int64_t chunk, int bshift,
                                                        int nb, const uint32_t* __restrict__ counts,
                                                        const uint32_t* __restrict__ offsets,
                                                        const float* __restrict__ dfeat, uint32_t* __restrict__ rec) {
  extern __shared__ uint32_t cur[];
  src.resolve();
  const uint32_t* mine = counts + (size_t)blockIdx.x * nb;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) cur[b] = offsets[b] + mine[b];
  __syncthreads();
  constexpr int RD = Rec<F>::dwords;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < B ? lo + chunk : B;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    float x, y, z;
    src.get(i, x, y, z);
    const float* d = dfeat + i * md.n_in;
    for (int l = 0; l < md.L; ++l) {
      float dv[F];
#pragma unroll
      for (int f = 0; f < F; ++f) dv[f] = d[l * F + f];
      Corners cr;
      level_corners(md.lv[l], x, y, z, cr);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t pos = atomicAdd(cur + (cr.slot[k] >> bshift), 1u);
        uint32_t w[RD];
        w[0] = cr.slot[k];
#pragma unroll
        for (int f = 0; f < F; ++f) w[1 + f] = __float_as_uint(cr.w[k] * dv[f]);
        store_dwords<RD>(rec + (size_t)pos * RD, w);
      }
    }
  }
}

// Work list of the reduce: one item per (bucket, chunk of records) that has
// records, built by one workgroup from the bucket sizes.  items[0] holds the
// count; item i is (bucket, chunk) = (items[2 + 2i], items[3 + 2i]).
__global__ void __launch_bounds__(1024) k_sc_worklist(const uint32_t* __restrict__ totals, int nb,
                                                      int64_t chunk_records, uint32_t* __restrict__ items) {
  __shared__ uint32_t part[1024];
  const int per = (nb + 1023) / 1024;
  const int lo = threadIdx.x * per;
  uint32_t c = 0;
  for (int i = 0; i < per; ++i)
    if (lo + i < nb) c += (uint32_t)((totals[lo + i] + chunk_records - 1) / chunk_records);
  part[threadIdx.x] = c;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const uint32_t v = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t pos = part[threadIdx.x] - c;
  for (int i = 0; i < per; ++i) {
    if (lo + i >= nb) break;
    const uint32_t nch = (uint32_t)((totals[lo + i] + chunk_records - 1) / chunk_records);
    for (uint32_t ch = 0; ch < nch; ++ch, ++pos) {
      items[2 + 2 * (size_t)pos] = (uint32_t)(lo + i);
      items[3 + 2 * (size_t)pos] = ch;
    }
  }
  if (threadIdx.x == 1023) items[0] = part[1023];
}

template <int F>
__global__ void __launch_bounds__(kReduceThreads) k_sc_reduce(const uint32_t* __restrict__ rec,
                                                              const uint32_t* __restrict__ totals,
                                                              const uint32_t* __restrict__ offsets,
                                                              const uint32_t* __restrict__ items, int bshift,
                                                              int64_t chunk_records, int64_t n_entries,
                                                              float* __restrict__ grad,
                                                              int32_t* __restrict__ nonfinite) {
  extern __shared__ float acc[];
  if (blockIdx.x >= items[0]) return;
  const int bucket = (int)items[2 + 2 * (size_t)blockIdx.x];
  const int64_t cnt = totals[bucket];
  const int64_t lo = (int64_t)items[3 + 2 * (size_t)blockIdx.x] * chunk_records;
  const int64_t hi = lo + chunk_records < cnt ? lo + chunk_records : cnt;
  // feature-major accumulator acc[f][entry] with a pitch of E + 1: the F
  // adds of a record, and lanes adding the same feature of different
  // entries, fall in different banks
  const int E = 1 << bshift;
  const int pitch = E + 1;
  const int span = E * F;
  for (int t = threadIdx.x; t < pitch * F; t += blockDim.x) acc[t] = 0.0f;
  __syncthreads();
  constexpr int RD = Rec<F>::dwords;
  const uint32_t base_entry = (uint32_t)bucket << bshift;
  const uint32_t* r0 = rec + (size_t)offsets[bucket] * RD;
  // kUnroll records per thread per round: their loads are all in flight
  // before the first LDS add
  for (int64_t rb = lo + threadIdx.x; rb < hi; rb += (int64_t)blockDim.x * kUnroll) {
    uint32_t w[kUnroll][RD];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t r = rb + (int64_t)u * blockDim.x;
      if (r < hi) {
        load_dwords<RD>(r0 + (size_t)r * RD, w[u]);
      } else {
        w[u][0] = base_entry;
#pragma unroll
        for (int q = 1; q < RD; ++q) w[u][q] = 0u;
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int local = (int)(w[u][0] - base_entry);
#pragma unroll
      for (int f = 0; f < F; ++f) {
        const float v = __uint_as_float(w[u][1 + f]);
        if (v != 0.0f) lds_add_f32(acc + f * pitch + local, v);
      }
    }
  }
  __syncthreads();
  const bool owner = cnt <= chunk_records;  // the bucket fits one chunk: this workgroup owns its entries
  const int64_t first = (int64_t)base_entry * F;
  const int64_t last = n_entries * F;
  constexpr int U = 8;  // entries per thread per round; the owner's gradient loads are issued together
  bool bad = false;
  for (int t0 = threadIdx.x; t0 < span; t0 += blockDim.x * U) {
    float a[U], old[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * (int)blockDim.x;  // gradient order: entry t / F, feature t % F
      const bool in = t < span && first + t < last;
      a[u] = in ? acc[(t % F) * pitch + t / F] : 0.0f;
      old[u] = (owner && in) ? grad[first + t] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * (int)blockDim.x;
      if (a[u] == 0.0f) continue;  // also every entry outside the table
      // a sum that leaves the finite range marks the step as skipped (the
      // last atomic on an entry sees its final value)
      float v;
      if (owner) {
        v = old[u] + a[u];
        grad[first + t] = v;
      } else {
        v = atomicAdd(grad + first + t, a[u]) + a[u];
      }
      if (!__builtin_isfinite(v)) bad = true;
    }
  }
  if (bad) *nonfinite = 1;
}

}  // namespace

ScatterPlan scatter_plan(const ngvol_plan* plan, int64_t B) {
  ScatterPlan sp{};
  const ModelDesc& md = plan->md;
  const int F = md.F;
  sp.bshift = F <= 2 ? 12 : (F == 4 ? 11 : 10);  // 2^bshift * F * 4 bytes = 32 KB of LDS
  const int64_t entries = md.n_table / F;
  sp.n_buckets = (int)((entries + (1 << sp.bshift) - 1) >> sp.bshift);
  int64_t g = (B + 1023) / 1024;
  if (g > plan->cus) g = plan->cus;
  if (g < 1) g = 1;
  sp.blocks = (int)g;
  sp.chunk = (B + g - 1) / g;
  sp.rec_words = 1 + F;  // dwords per record
  sp.n_records = B * 8 * md.L;
  // a chunk is one workgroup's serial share of a bucket's LDS adds: bound it
  // to kChunkAdds feature adds so the hot coarse buckets spread over as many
  // workgroups as their records need (F = 8: 16384 records a chunk)
  sp.chunk_records = kChunkAdds / F;
  // upper bound of the work items: one partial chunk per bucket plus full chunks
  sp.max_items = sp.n_buckets + (int)((sp.n_records + sp.chunk_records - 1) / sp.chunk_records);
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  sp.rec_off = 0;
  sp.counts_off = up((size_t)sp.n_records * 4 * sp.rec_words);
  sp.totals_off = sp.counts_off + up((size_t)sp.blocks * sp.n_buckets * 4);
  sp.offsets_off = sp.totals_off + up((size_t)sp.n_buckets * 4);
  sp.items_off = sp.offsets_off + up((size_t)sp.n_buckets * 4);
  sp.bytes = sp.items_off + up((size_t)(sp.max_items + 1) * 8);
  return sp;
}

hipError_t launch_scatter(const ngvol_plan* plan, const ScatterPlan& sp, const BatchArgs& ba, const float* dfeat,
                          float* grad, void* ws, int32_t* nonfinite, hipStream_t st) {
  const ModelDesc& md = plan->md;
  char* base = reinterpret_cast<char*>(ws);
  uint32_t* rec = reinterpret_cast<uint32_t*>(base + sp.rec_off);
  uint32_t* counts = reinterpret_cast<uint32_t*>(base + sp.counts_off);
  uint32_t* totals = reinterpret_cast<uint32_t*>(base + sp.totals_off);
  uint32_t* offsets = reinterpret_cast<uint32_t*>(base + sp.offsets_off);
  const Coords src{ba.xyz, ba.seed, ba.step, ba.B, ba.step_ptr};
  const size_t hist_lds = (size_t)sp.n_buckets * 4;
  hipLaunchKernelGGL(k_sc_count, dim3(sp.blocks), dim3(kScThreads), hist_lds, st, md, src, ba.B, sp.chunk, sp.bshift,
                     sp.n_buckets, counts);
  launch_count_offsets(counts, sp.blocks, sp.n_buckets, totals, offsets, st);
  uint32_t* items = reinterpret_cast<uint32_t*>(base + sp.items_off);
  hipLaunchKernelGGL(k_sc_worklist, dim3(1), dim3(1024), 0, st, totals, sp.n_buckets, sp.chunk_records, items);
  const size_t acc_lds = (((size_t)1 << sp.bshift) + 1) * md.F * 4;
  const dim3 rgrid(sp.max_items);
  const int64_t n_entries = md.n_table / md.F;
#define NGV_SC(FV)                                                                                                 \
  hipLaunchKernelGGL(k_sc_fill<FV>, dim3(sp.blocks), dim3(kScThreads), hist_lds, st, md, src, ba.B, sp.chunk,      \
                     sp.bshift, sp.n_buckets, counts, offsets, dfeat, rec);                                        \
  hipLaunchKernelGGL(k_sc_reduce<FV>, rgrid, dim3(kReduceThreads), acc_lds, st, rec, totals, offsets, items,      \
                     sp.bshift, sp.chunk_records, n_entries, grad, nonfinite)
  switch (md.F) {
    case 2: NGV_SC(2); break;
    case 4: NGV_SC(4); break;
    case 8: NGV_SC(8); break;
    default: return hipErrorInvalidValue;
  }
#undef NGV_SC
  return hipGetLastError();
}

}  // namespace ngvol
