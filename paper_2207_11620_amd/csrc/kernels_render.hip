// Ray-marched emission-absorption rendering through the network with sample
// streaming (Section 5.2.1), as one persistent launch.
//
// The paper's host loop {compaction; coordinates; batch inference; shading}
// becomes a loop inside each wave: the wave keeps 8 rays in flight; each
// round it streams K = 8 sample coordinates per ray (a 64-sample batch,
// four 16-sample MFMA tiles), evaluates the network on them, and composites
// them front to back.  A ray that has terminated or run out of samples is
// written out and its slot refilled at the next round from the wave's
// 8x8-pixel tiles, taken from a device work queue: this plays the role of
// stream compaction (no wave works on a dead ray, and no control returns to
// the host until the frame is done), and the 8 rays of a wave stay
// neighbours, so their samples share cache lines.
//
// Work distribution is XCD-aware: the tiles are cut into 8 bands of rows,
// workgroups take tiles from the band of their XCD (workgroup id mod 8),
// so neighbouring rays (coherent hash-table footprints) share an L2, and
// steal from the other bands once their own is empty.
// build: one object per MLP precision and width (NGV_PSEL, NGV_WSEL)
#include "kernels.hpp"
#include "render.hpp"
#include "ray_geom.hpp"
#include "dispatch.hpp"
#include "mlp_tile.hpp"

namespace ngvol {

namespace {
constexpr int kSlots = 8;  // rays per wave
constexpr int kK = 8;      // samples per ray per round
}  // namespace

// First sample index after k outside the macro-cell of sample k: the ray's
// exit from the cell's box (a DDA step), the grid index just past it, then
// an exact correction on the samples' own cells (their cell indices change
// monotonically along the ray, so the result is the first such sample).
__device__ uint32_t cell_exit(const RayGeom& r, uint32_t k, float dt, const McGeom& g) {
  float p[3];
  ray_point(r, k, dt, p[0], p[1], p[2]);
  const uint32_t c = mc_index(g, clamp01(p[0]), clamp01(p[1]), clamp01(p[2]));
  float t_exit = INFINITY;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (r.d[a] == 0.0f) continue;
    const int M = g.m[a];
    const float q = clamp01(p[a]);
    int ca = (int)floorf(__fmul_rn(q, (float)g.dims[a])) / g.cell;
    ca = ca < M - 1 ? ca : M - 1;
    float bound;
    if (r.d[a] > 0.0f) {
      if (ca == M - 1) continue;  // the last cell reaches the cube's face
      bound = __fdiv_rn((float)((ca + 1) * g.cell), (float)g.dims[a]);
    } else {
      if (ca == 0) continue;
      bound = __fdiv_rn((float)(ca * g.cell), (float)g.dims[a]);
    }
    const float ta = __fdiv_rn(__fsub_rn(bound, r.o[a]), r.d[a]);
    t_exit = fminf(t_exit, ta);
  }
  uint32_t q;
  if (!(t_exit < INFINITY)) {
    q = r.n;
  } else {
    const float gq = ceilf(__fsub_rn(__fdiv_rn(__fsub_rn(t_exit, r.t0), dt), r.j));
    q = gq <= (float)(k + 1) ? k + 1 : (gq >= (float)r.n ? r.n : (uint32_t)gq);
  }
  while (q < r.n && sample_cell(r, q, dt, g) == c) ++q;
  while (q > k + 1 && sample_cell(r, q - 1, dt, g) != c) --q;
  return q;
}

struct SlotState {
  RayGeom g;
  int32_t pix;  // -1: empty
  uint32_t k;   // next sample index
  uint32_t used;
  float C[3], A;
  // single-shot shadow: the largest contribution so far and its sample
  // index (first pass), the primary ray's sample count, and the shadow
  // ray's transmittance (second pass)
  uint32_t kmax, n0;
  float wmax, T;
  // macro-cell walk: exit index and mu of the cell of the current sample
  uint32_t kexit;
  float mu_cur;
};

// Macro-cell modes, per slot: this round's samples (the walk through the
// cells: empty-space skipping lists the samples of non-empty cells,
// adaptive marching one sample per adaptive step), the grid steps each
// stands for (adaptive), their count, and the first sample index after the
// round.
constexpr int kSpan = kK;
constexpr int kCnt = 2 * kK, kNext = 2 * kK + 1;
constexpr int kList = 2 * kK + 2;

// Macro-cell modes of the marcher.
constexpr int kMcNone = 0, kMcSkip = 1, kMcAdaptive = 2;

// Grid steps a sample in a cell of maximum opacity mu stands for (Section
// 5.3): sbar = max(1 + (s2 - 1) |min(mu,1) - 1|^p, 1), floored; binary32,
// one rounding per operation.
__device__ __forceinline__ uint32_t adaptive_steps(float mu, float s2, int p) {
  const float m = fminf(mu, 1.0f);
  const float d = fabsf(__fsub_rn(m, 1.0f));
  float pw = 1.0f;
  for (int i = 0; i < p; ++i) pw = __fmul_rn(pw, d);
  const float t = __fmul_rn(__fsub_rn(s2, 1.0f), pw);
  const float sb = fmaxf(__fadd_rn(1.0f, t), 1.0f);
  return (uint32_t)floorf(sb);
}

#if NGV_PRIMARY
__global__ void k_render_init(unsigned int* queue, unsigned long long* counters) {
  const int t = threadIdx.x;
  if (t < kBands) queue[t] = 0u;
  if (t < 4 && counters) counters[t] = 0ull;
}
#else
__global__ void k_render_init(unsigned int* queue, unsigned long long* counters);
#endif

// LDS layout of k_render: staged weights, the W_out region, the LUT
// [256][4], the slots and per-sample outputs of every wave, then the
// encoding stages.
__host__ __device__ inline size_t render_stage_offset(size_t weight_bytes, size_t wout_bytes, int waves) {
  const size_t end = weight_bytes + wout_bytes + 1024 * 4 + (size_t)waves * kSlots * sizeof(SlotState) +
                     (size_t)waves * kSlots * kK * 4 + (size_t)waves * kSlots * kList * 4;
  return (end + 15) & ~(size_t)15;
}

// SHM: 0 plain; 1 the camera-ray pass of single-shot shadows, which also
// records each pixel's shading point; 2 the shadow-ray pass, which marches
// from the recorded points towards the light and scales the pixels.
template <int P, int F, int KIN, int W, typename TT, int MC, int SHM>
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

  // Owner lanes (lane < kSlots) keep their slot in LDS.  A slot's pixel is
  // >= 0 while its ray is marched, -2 while it waits for a new pixel and -1
  // once the frame has none left.
  constexpr bool rec = SHM == 1, shadow = SHM == 2;
  float lhat[3] = {0.0f, 0.0f, 1.0f};
  if constexpr (shadow) unit3(ra.light, lhat);
  auto start = [&](SlotState& sl, int32_t p) -> bool {
    const int px = p % ra.width, py = p / ra.width;
    sl.pix = p;
    sl.g = make_ray(ra.cam, ra.width, px, py, ra.seed, ra.dt);
    sl.k = 0;
    sl.kexit = 0;
    sl.mu_cur = 0.0f;
    sl.T = 1.0f;
    if constexpr (shadow) {
      // the shadow ray from the pixel's shading point, from its sample 1 on;
      // a pixel without one, or a ray with no sample beyond it, keeps T = 1
      const uint32_t ks = ra.aux[p];
      if (ks != 0xFFFFFFFFu) {
        float ps[3];
        ray_point(sl.g, ks, ra.dt, ps[0], ps[1], ps[2]);
        sl.g = ray_from(ps, lhat, sl.g.j, ra.dt);
        sl.k = 1;
        if (sl.g.n > 1u) return true;
      }
      sl.pix = -2;
      return false;
    }
    sl.used = 0;
    sl.C[0] = sl.C[1] = sl.C[2] = 0.0f;
    sl.A = 0.0f;
    sl.kmax = 0xFFFFFFFFu;
    sl.n0 = sl.g.n;
    sl.wmax = 0.0f;
    if (sl.g.n > 0) {
      ++n_rays;
      return true;
    }
    // empty ray: write it out
    float4* o4 = reinterpret_cast<float4*>(ra.rgba) + p;
    *o4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (ra.n_geo) ra.n_geo[p] = 0u;
    if (ra.n_used) ra.n_used[p] = 0u;
    if (rec) ra.aux[p] = 0xFFFFFFFFu;
    sl.pix = -2;
    return false;
  };
  // waiting slots take pixels of the wave's tiles (whole wave)
  PixelPool pool = pool_init();
  auto fill = [&]() {
    for (;;) {
      const bool want = lane < kSlots && slots[lane].pix == -2;
      if (!__any(want)) return;
      const int32_t p = pool_take(pool, want, ra.queue, band0, ra.width, ra.height);
      if (want) {
        SlotState sl = slots[lane];
        if (p < 0) sl.pix = -1;
        else start(sl, p);
        slots[lane] = sl;
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
  };
  if (lane < kSlots) slots[lane].pix = -2;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");

  constexpr bool skip_empty = MC == kMcSkip;     // ra.mc.mu is set
  constexpr bool adaptive = MC == kMcAdaptive;   // ra.mc.mu is set
  for (;;) {
    fill();
    // any live slot in this wave?
    const bool live = lane < kSlots && slots[lane].pix >= 0;
    if (!__any(live)) break;
    if constexpr (skip_empty || adaptive) {
      // each slot's owner lane walks its ray: a transparent cell is passed
      // whole (a DDA jump to its exit); in an opaque cell every sample is
      // listed (skipping), or one sample stands for adaptive_steps of the
      // cell's mu grid steps, cut at the cell's exit (adaptive marching)
      if (lane < kSlots) {
        SlotState& so = slots[lane];
        uint32_t k = so.k, cnt = 0;
        const uint32_t n = so.g.n;
        if (so.pix >= 0) {
          // the slot remembers the cell it is in (its exit index and mu), so
          // a cell is looked up once, not once per sample
          uint32_t kexit = so.kexit;
          float mu = so.mu_cur;
          while (cnt < (uint32_t)kK && k < n) {
            if (k >= kexit) {
              mu = ra.mc.mu[sample_cell(so.g, k, ra.dt, ra.mc)];
              kexit = cell_exit(so.g, k, ra.dt, ra.mc);
            }
            if (!(mu > 0.0f)) {
              k = kexit;
              continue;
            }
            uint32_t kn = k + 1;
            if constexpr (adaptive) {
              const uint32_t steps = adaptive_steps(mu, ra.step_max, ra.step_exp);
              kn = k + steps < kexit ? k + steps : kexit;
            }
            kn = kn < n ? kn : n;
            lst[lane * kList + cnt] = k;
            lst[lane * kList + kSpan + cnt] = kn - k;
            ++cnt;
            k = kn;
          }
          so.kexit = kexit;
          so.mu_cur = mu;
        }
        lst[lane * kList + kCnt] = cnt;
        lst[lane * kList + kNext] = k;
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    // lane j evaluates sample k = slot.k + j%8 of slot j/8 (with skipping or
    // adaptive marching: the slot's (j%8)-th listed sample)
    {
      const int si = lane >> 3, q = lane & 7;
      const SlotState& sl = slots[si];
      uint32_t k;
      bool valid;
      if (skip_empty || adaptive) {
        valid = sl.pix >= 0 && (uint32_t)q < lst[si * kList + kCnt];
        k = valid ? lst[si * kList + q] : 0u;
      } else {
        k = sl.k + (uint32_t)q;
        valid = sl.pix >= 0 && k < sl.g.n;
      }
      // a round in which no ray of the wave has a sample outside empty
      // cells only advances the rays
      if (!(skip_empty || adaptive) || __any(valid)) {
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
        const uint32_t kend = (skip_empty || adaptive) ? lst[lane * kList + kCnt]
                                                       : (sl.g.n - sl.k < (uint32_t)kK ? sl.g.n - sl.k : (uint32_t)kK);
        for (uint32_t q = 0; q < kend; ++q) {
          float c4[4];
          tf_lookup(lds_lut, yv[lane * kK + q], c4);
          float a = c4[3];
          if constexpr (adaptive) {
            // opacity of a sample standing for `span` grid steps
            const uint32_t span = lst[lane * kList + kSpan + q];
            if (span > 1u) a = __fsub_rn(1.0f, powf(__fsub_rn(1.0f, a), (float)span));
          }
          if constexpr (shadow) {
            // shadow ray: transmittance towards the light
            sl.T = sl.T * (1.0f - a);
            if (sl.T <= 0.01f) {
              done = true;
              break;
            }
            continue;
          }
          const float w = (1.0f - sl.A) * a;
          if (rec && w > sl.wmax) {
            sl.wmax = w;
            sl.kmax = (skip_empty || adaptive) ? lst[lane * kList + q] : sl.k + q;
          }
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
        sl.k = (skip_empty || adaptive) ? lst[lane * kList + kNext] : sl.k + kend;
        if (done || sl.k >= sl.g.n) {
          const int32_t p = sl.pix;
          float4* o4 = reinterpret_cast<float4*>(ra.rgba) + p;
          if constexpr (shadow) {
            // T attenuates the whole colour of the camera-ray pass
            const float4 c = *o4;
            *o4 = make_float4(sl.T * c.x, sl.T * c.y, sl.T * c.z, c.w);
          } else {
            *o4 = make_float4(sl.C[0], sl.C[1], sl.C[2], sl.A);
            if (ra.n_geo) ra.n_geo[p] = sl.n0;
            if (ra.n_used) ra.n_used[p] = sl.used;
            if (rec) ra.aux[p] = sl.kmax;
            n_used_tot += sl.used;
          }
          sl.pix = -2;
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
#define NGV_RENDER_GO(TT, MCM)                                                                                    \
  do {                                                                                                            \
    if constexpr (MCM != kMcAdaptive) {                                                                          \
      if (ra.mode == NGVOL_RENDER_RM_SHADOW) {                                                                    \
        /* camera rays (recording the shading points), then the shadow rays */                                  \
        hipLaunchKernelGGL((k_render<P, F, KIN, W, TT, MCM, 1>), dim3((unsigned)grid), dim3(256), lds, st, md, tp,  \
                           mlp, ra);                                                                              \
        hipLaunchKernelGGL(k_render_init, dim3(1), dim3(64), 0, st, ra.queue, nullptr);                          \
        hipLaunchKernelGGL((k_render<P, F, KIN, W, TT, MCM, 2>), dim3((unsigned)grid), dim3(256), lds, st, md, tp,  \
                           mlp, ra);                                                                              \
        break;                                                                                                    \
      }                                                                                                           \
    }                                                                                                             \
    hipLaunchKernelGGL((k_render<P, F, KIN, W, TT, MCM, 0>), dim3((unsigned)grid), dim3(256), lds, st, md, tp,      \
                       mlp, ra);                                                                                  \
  } while (0)
  NGV_DISPATCH_F_KIN(md.F, plan->kin, {
    const int mcm = ra.mc.mu == nullptr ? kMcNone : (ra.adaptive ? kMcAdaptive : kMcSkip);
    if (tp.f16) {
      if (mcm == kMcNone) NGV_RENDER_GO(__half, kMcNone);
      else if (mcm == kMcSkip) NGV_RENDER_GO(__half, kMcSkip);
      else NGV_RENDER_GO(__half, kMcAdaptive);
    } else {
      if (mcm == kMcNone) NGV_RENDER_GO(float, kMcNone);
      else if (mcm == kMcSkip) NGV_RENDER_GO(float, kMcSkip);
      else NGV_RENDER_GO(float, kMcAdaptive);
    }
  });
#undef NGV_RENDER_GO
  return hipGetLastError();
}

template hipError_t launch_render_p<NGV_PSEL, NGV_WSEL>(const ngvol_plan*, TablePtrs, const float*, const RenderArgs&,
                                              hipStream_t);

#if NGV_PRIMARY
hipError_t launch_render(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const RenderArgs& ra,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_render_init, dim3(1), dim3(64), 0, st, ra.queue, ra.counters);
  if (ra.mode == NGVOL_RENDER_PT)
    NGV_DISPATCH_P(plan->layout.precision,
                   NGV_DISPATCH_W(plan->md.width, return launch_render_pt_p<P, W>(plan, tp, mlp, ra, st)));
  NGV_DISPATCH_P(plan->layout.precision, NGV_DISPATCH_W(plan->md.width, return launch_render_p<P, W>(plan, tp, mlp, ra, st)));
  return hipErrorInvalidValue;
}
#endif

}  // namespace ngvol
