// Ray-marched emission-absorption rendering through the network with sample
// streaming (Section 5.2.1), as one persistent launch.
//
// The paper's host loop {compaction; coordinates; batch inference; shading}
// becomes a loop inside each wave: the wave keeps 8 rays in flight; each
// round it streams K = 8 sample coordinates per ray (a 64-sample batch,
// four 16-sample MFMA tiles), evaluates the network on them, and composites
// them front to back.  A ray that has terminated or run out of samples is
// written out and its slot refilled from a device work queue, which plays
// the role of stream compaction: no wave ever works on a dead ray, and no
// control returns to the host until the frame is done.
//
// Work distribution is XCD-aware: the frame is cut into 8 bands of rows,
// workgroups fetch rays from the band of their XCD (workgroup id mod 8),
// so neighbouring rays (coherent hash-table footprints) share an L2, and
// steal from the other bands once their own is empty.
// build: one object per MLP precision and width (NGV_PSEL, NGV_WSEL)
#include "kernels.hpp"
#include "dispatch.hpp"
#include "mlp_tile.hpp"

namespace ngvol {

namespace {
constexpr int kSlots = 8;  // rays per wave
constexpr int kK = 8;      // samples per ray per round
constexpr int kBands = 8;  // one work band per XCD
}  // namespace

struct RayGeom {
  float o[3], d[3], t0, j;
  uint32_t n;
};

// Ray of pixel (px, py): binary32, one rounding per operation, no FMA.
__device__ __forceinline__ RayGeom make_ray(const float* cam, int W, int px, int py, uint32_t seed, float dt) {
  RayGeom r;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  float dir[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float t1 = __fmul_rn(fx, cam[3 + a]);
    const float t2 = __fadd_rn(cam[9 + a], t1);
    const float t3 = __fmul_rn(fy, cam[6 + a]);
    dir[a] = __fadd_rn(t2, t3);
  }
  const float n2 = __fadd_rn(__fadd_rn(__fmul_rn(dir[0], dir[0]), __fmul_rn(dir[1], dir[1])), __fmul_rn(dir[2], dir[2]));
  const float nrm = __fsqrt_rn(n2);
  float tmin = -INFINITY, tmax = INFINITY;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r.o[a] = cam[a];
    r.d[a] = __fdiv_rn(dir[a], nrm);
    const float inv = __fdiv_rn(1.0f, r.d[a]);
    const float ta = __fmul_rn(__fsub_rn(0.0f, r.o[a]), inv);
    const float tb = __fmul_rn(__fsub_rn(1.0f, r.o[a]), inv);
    tmin = fmaxf(tmin, fminf(ta, tb));
    tmax = fminf(tmax, fmaxf(ta, tb));
  }
  const float tn = fmaxf(tmin, 0.0f);
  r.t0 = tn;
  r.j = rng_u01((uint64_t)seed, 5u, (uint64_t)py * (uint64_t)W + (uint64_t)px);
  r.n = 0;
  if (tn < tmax) {
    const float q = __fdiv_rn(__fsub_rn(tmax, tn), dt);
    // a unit-cube chord is at most sqrt(3) long; more than 2^24 steps (or a
    // NaN span) means a degenerate ray, which gets no samples
    if (q <= 16777216.0f) {
      const float c = ceilf(__fsub_rn(q, r.j));
      if (c > 0.0f) r.n = (uint32_t)c;
    }
  }
  return r;
}

__device__ __forceinline__ void ray_point(const RayGeom& r, uint32_t k, float dt, float& x, float& y, float& z) {
  const float kj = __fadd_rn((float)k, r.j);
  const float t = __fadd_rn(r.t0, __fmul_rn(kj, dt));
  x = __fadd_rn(r.o[0], __fmul_rn(t, r.d[0]));
  y = __fadd_rn(r.o[1], __fmul_rn(t, r.d[1]));
  z = __fadd_rn(r.o[2], __fmul_rn(t, r.d[2]));
}

struct SlotState {
  RayGeom g;
  int32_t pix;  // -1: empty
  uint32_t k;   // next sample index
  uint32_t used;
  float C[3], A;
};

// Empty-space skipping, per slot: this round's samples (those in a non-empty
// macro-cell), their count, and the first sample index after the round.
constexpr int kList = kK + 2;
constexpr int kCnt = kK, kNext = kK + 1;

#if NGV_PRIMARY
__global__ void k_render_init(unsigned int* queue, unsigned long long* counters) {
  const int t = threadIdx.x;
  if (t < kBands) queue[t] = 0u;
  if (t < 4 && counters) counters[t] = 0ull;
}
#else
__global__ void k_render_init(unsigned int* queue, unsigned long long* counters);
#endif

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

// LDS layout of k_render: staged weights, the W_out region, the LUT
// [256][4], the slots and per-sample outputs of every wave, then the
// encoding stages.
__host__ __device__ inline size_t render_stage_offset(size_t weight_bytes, size_t wout_bytes, int waves) {
  const size_t end = weight_bytes + wout_bytes + 1024 * 4 + (size_t)waves * kSlots * sizeof(SlotState) +
                     (size_t)waves * kSlots * kK * 4 + (size_t)waves * kSlots * kList * 4;
  return (end + 15) & ~(size_t)15;
}

template <int P, int F, int KIN, int W, typename TT, bool SKIP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P != 0 && KIN == 32 ? 4 : 1)))
k_render(ModelDesc md, TablePtrs tp, const float* __restrict__ mlp, RenderArgs ra) {
  typedef typename Prec<P>::Frag Frag;
  typedef WeightLayout<P, KIN, W> WL;
  extern __shared__ __align__(16) unsigned char smem[];
  Frag* lds_frag = reinterpret_cast<Frag*>(smem);
  const size_t wbytes = (size_t)WL::frags(md.n_hidden, false) * 64 * sizeof(Frag);
  float* lds_wout = reinterpret_cast<float*>(smem + wbytes);
  float* lds_lut = reinterpret_cast<float*>(smem + wbytes + wout_region_bytes<P, W>());  // [256][4]
  const int wave = threadIdx.x >> 6;
  SlotState* slots = reinterpret_cast<SlotState*>(lds_lut + 1024) + wave * kSlots;
  float* yv = reinterpret_cast<float*>(reinterpret_cast<SlotState*>(lds_lut + 1024) + (blockDim.x >> 6) * kSlots) +
              wave * kSlots * kK;
  uint32_t* lst = reinterpret_cast<uint32_t*>(yv - wave * kSlots * kK + (blockDim.x >> 6) * kSlots * kK) +
                  wave * kSlots * kList;
  typedef typename Prec<P>::T T;
  T* stage = reinterpret_cast<T*>(smem + render_stage_offset(wbytes, wout_region_bytes<P, W>(), blockDim.x >> 6) +
                                  wave * Stage<P, KIN>::wave_bytes);
  T* row = stage + (threadIdx.x & 63) * Stage<P, KIN>::pitch;

  stage_weights<P, KIN, W>(md, mlp, lds_frag, lds_wout, false);
  for (int t = threadIdx.x; t < 1024; t += blockDim.x) lds_lut[t] = ra.lut[t];
  __syncthreads();

  const TT* table = table_ptr<TT>(tp);
  const int lane = threadIdx.x & 63, nl = lane & 15, g = lane >> 4;
  const int band0 = blockIdx.x % kBands;
  const int64_t n_pix = (int64_t)ra.width * ra.height;
  unsigned long long n_eval = 0, n_used_tot = 0, n_rays = 0;

  // Owner lanes (lane < kSlots) keep their slot in LDS.
  auto refill = [&](SlotState& sl) {
    for (;;) {
      const int32_t p = fetch_pixel(ra.queue, band0, n_pix);
      sl.pix = p;
      if (p < 0) return;
      const int px = p % ra.width, py = p / ra.width;
      sl.g = make_ray(ra.cam, ra.width, px, py, ra.seed, ra.dt);
      sl.k = 0;
      sl.used = 0;
      sl.C[0] = sl.C[1] = sl.C[2] = 0.0f;
      sl.A = 0.0f;
      if (sl.g.n > 0) {
        ++n_rays;
        return;
      }
      // empty ray: write it out and take another
      float4* o4 = reinterpret_cast<float4*>(ra.rgba) + p;
      *o4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (ra.n_geo) ra.n_geo[p] = 0u;
      if (ra.n_used) ra.n_used[p] = 0u;
    }
  };

  if (lane < kSlots) {
    SlotState sl;
    refill(sl);
    slots[lane] = sl;
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");

  constexpr bool skip_empty = SKIP;  // ra.mc.mu is set
  for (;;) {
    // any live slot in this wave?
    const bool live = lane < kSlots && slots[lane].pix >= 0;
    if (!__any(live)) break;
    if constexpr (skip_empty) {
      // each slot's next 64 samples are checked against the macro-cells, one
      // per lane; the first kK in a non-empty cell are this round's samples
      for (int s = 0; s < kSlots; ++s) {
        const SlotState& so = slots[s];
        const uint32_t k0 = so.k, n = so.g.n;
        const uint32_t c = k0 + (uint32_t)lane;
        bool in = false;
        if (so.pix >= 0 && c < n) {
          float x, y, z;
          ray_point(so.g, c, ra.dt, x, y, z);
          in = ra.mc.mu[mc_index(ra.mc, clamp01(x), clamp01(y), clamp01(z))] > 0.0f;
        }
        const unsigned long long mask = __ballot(in);
        const uint32_t below = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
        const uint32_t total = (uint32_t)__popcll(mask);
        uint32_t next = k0 + 64u;
        if (total >= (uint32_t)kK) {
          const unsigned long long last = __ballot(in && below == (uint32_t)kK - 1u);
          next = k0 + (uint32_t)(__ffsll((unsigned long long)last) - 1) + 1u;
        }
        __builtin_amdgcn_wave_barrier();
        if (in && below < (uint32_t)kK) lst[s * kList + below] = c;
        if (lane == 0) {
          lst[s * kList + kCnt] = total < (uint32_t)kK ? total : (uint32_t)kK;
          lst[s * kList + kNext] = next < n ? next : n;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      }
    }
    // lane j evaluates sample k = slot.k + j%8 of slot j/8 (with skipping:
    // the slot's (j%8)-th listed sample)
    {
      const int si = lane >> 3, q = lane & 7;
      const SlotState& sl = slots[si];
      uint32_t k;
      bool valid;
      if (skip_empty) {
        valid = sl.pix >= 0 && (uint32_t)q < lst[si * kList + kCnt];
        k = valid ? lst[si * kList + q] : 0u;
      } else {
        k = sl.k + (uint32_t)q;
        valid = sl.pix >= 0 && k < sl.g.n;
      }
      // a round in which no ray of the wave has a sample outside empty
      // cells only advances the rays
      if (!skip_empty || __any(valid)) {
        float x = 0.5f, y = 0.5f, z = 0.5f;
        if (valid) {
          ray_point(sl.g, k, ra.dt, x, y, z);
          x = clamp01(x);
          y = clamp01(y);
          z = clamp01(z);
        }
        encode_row<P, F, KIN>(md, table, x, y, z, row, [](int, const Oct<P>&) {});
        wave_sync();
        yv[lane] = mlp_wave64<P, KIN, W>(md.n_hidden, md.out_relu != 0, lds_frag, lds_wout, stage);
        if (valid) ++n_eval;
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (lane < kSlots) {
      SlotState sl = slots[lane];
      if (sl.pix >= 0) {
        bool done = false;
        const uint32_t kend =
            skip_empty ? lst[lane * kList + kCnt] : (sl.g.n - sl.k < (uint32_t)kK ? sl.g.n - sl.k : (uint32_t)kK);
        for (uint32_t q = 0; q < kend; ++q) {
          const float val = fminf(fmaxf(yv[lane * kK + q], 0.0f), 1.0f);
          const float u = 255.0f * val;
          const float fi = fminf(floorf(u), 254.0f);
          const int i0 = (int)fi;
          const float fr = u - fi;
          float c4[4];
#pragma unroll
          for (int ch = 0; ch < 4; ++ch) c4[ch] = __builtin_fmaf(fr, lds_lut[4 * (i0 + 1) + ch] - lds_lut[4 * i0 + ch],
                                                                   lds_lut[4 * i0 + ch]);
          const float w = (1.0f - sl.A) * c4[3];
          sl.C[0] = __builtin_fmaf(w, c4[0], sl.C[0]);
          sl.C[1] = __builtin_fmaf(w, c4[1], sl.C[1]);
          sl.C[2] = __builtin_fmaf(w, c4[2], sl.C[2]);
          sl.A += w;
          sl.used += 1;
          if (sl.A >= 0.99f) {
            done = true;
            break;
          }
        }
        sl.k = skip_empty ? lst[lane * kList + kNext] : sl.k + kend;
        if (done || sl.k >= sl.g.n) {
          const int32_t p = sl.pix;
          float4* o4 = reinterpret_cast<float4*>(ra.rgba) + p;
          *o4 = make_float4(sl.C[0], sl.C[1], sl.C[2], sl.A);
          if (ra.n_geo) ra.n_geo[p] = sl.g.n;
          if (ra.n_used) ra.n_used[p] = sl.used;
          n_used_tot += sl.used;
          refill(sl);
        }
        slots[lane] = sl;
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
  if (ra.counters) {
    const unsigned long long e = (unsigned long long)wave_sum((double)n_eval);
    const unsigned long long u = (unsigned long long)wave_sum((double)n_used_tot);
    const unsigned long long r = (unsigned long long)wave_sum((double)n_rays);
    if (lane == 0) {
      atomicAdd(ra.counters + 0, e);
      atomicAdd(ra.counters + 1, u);
      atomicAdd(ra.counters + 2, r);
    }
  }
}

#if NGV_PRIMARY
size_t render_lds_bytes(const ngvol_plan* plan, int waves) {
  const size_t esz = plan->layout.precision ? 2 : 4;
  const size_t stage = (size_t)64 * (plan->kin + 16 / esz) * esz;
  return render_stage_offset(mlp_weight_bytes(plan), wout_bytes(plan), waves) +
         (size_t)waves * stage;
}
#endif

template <int P, int W>
hipError_t launch_render_p(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const RenderArgs& ra,
                           hipStream_t st) {
  const ModelDesc& md = plan->md;
  const size_t lds = render_lds_bytes(plan, 4);
  const int64_t n_pix = (int64_t)ra.width * ra.height;
  int64_t grid = (n_pix + 4 * kSlots - 1) / (4 * kSlots);
  const int64_t cap = (int64_t)plan->cus * 8;
  if (grid > cap) grid = cap;
  if (grid < 1) grid = 1;
  const bool skip = ra.mc.mu != nullptr;
  NGV_DISPATCH_F_KIN(md.F, plan->kin, {
    if (tp.f16) {
      if (skip)
        hipLaunchKernelGGL((k_render<P, F, KIN, W, __half, true>), dim3((unsigned)grid), dim3(256), lds, st, md, tp, mlp, ra);
      else
        hipLaunchKernelGGL((k_render<P, F, KIN, W, __half, false>), dim3((unsigned)grid), dim3(256), lds, st, md, tp, mlp, ra);
    } else {
      if (skip)
        hipLaunchKernelGGL((k_render<P, F, KIN, W, float, true>), dim3((unsigned)grid), dim3(256), lds, st, md, tp, mlp, ra);
      else
        hipLaunchKernelGGL((k_render<P, F, KIN, W, float, false>), dim3((unsigned)grid), dim3(256), lds, st, md, tp, mlp, ra);
    }
  });
  return hipGetLastError();
}

template hipError_t launch_render_p<NGV_PSEL, NGV_WSEL>(const ngvol_plan*, TablePtrs, const float*, const RenderArgs&,
                                              hipStream_t);

#if NGV_PRIMARY
hipError_t launch_render(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const RenderArgs& ra,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_render_init, dim3(1), dim3(64), 0, st, ra.queue, ra.counters);
  NGV_DISPATCH_P(plan->layout.precision, NGV_DISPATCH_W(plan->md.width, return launch_render_p<P, W>(plan, tp, mlp, ra, st)));
  return hipErrorInvalidValue;
}
#endif

}  // namespace ngvol
