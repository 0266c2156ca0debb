// Volumetric path tracing through the network (Section 5.2.2): Woodcock
// tracking with null collisions (Algorithm 1), next-event estimation by
// shadow rays towards a directional light, isotropic scattering with the
// transfer function's colour as albedo, Russian roulette, and optional
// macro-cell majorants walked by optical thickness (Section 5.3, Eqs. 1-2).
//
// The paper's streaming loop {sample; batch inference; shade} runs inside
// each wave of one persistent launch: every lane owns one path and advances
// it to its next tentative collision (the sample step: tracking, escapes,
// light and background terms, new directions, finished paths and pixels);
// the wave then evaluates its 64 collision points through the network on the
// matrix cores in one batch, and every lane decides real or null collision
// and moves its path on (the shade step).  A lane whose pixel is done takes
// the next pixel of its wave's 8x8-pixel tiles, fetched from the device work
// queue, which stands in for the paper's stream compaction: no lane idles
// while pixels remain, and a wave's camera rays stay neighbours.
//
// Path geometry is binary32 with one rounding per operation (positions,
// distances, optical-thickness sums); -ln(1 - zeta) and the new directions'
// cos, sin and sqrt are evaluated in FP64 and rounded to binary32, so that
// paths are reproducible across implementations.  Throughput and radiance
// are FP32.
// build: one object per MLP precision and width (NGV_PSEL, NGV_WSEL)
#include "kernels.hpp"
#include "render.hpp"
#include "ray_geom.hpp"
#include "dispatch.hpp"
#include "mlp_tile.hpp"

namespace ngvol {

namespace {

constexpr uint32_t kPtMaxSamples = 65536u;         // tentative collisions per path
constexpr float kInv4Pi = 0.0795774715459476679f;  // isotropic phase value 1/(4 pi)
constexpr double kTwoPi = 6.283185307179586477;

// One tracking step from distance t of the ray o + t d (span [t, tf)) for
// the target optical thickness tau: the next tentative collision tc and the
// majorant there, or false when the ray leaves the span first.  Without
// macro-cells the majorant is density * amax over the whole cube; with them,
// density * mu(c) per cell, the cells visited by a 3-D DDA from the cell of
// the point at t, the thickness accumulated cell by cell, and the collision
// placed inside the first cell where it would exceed tau (Hofmann et al.).
template <bool MC>
__device__ bool pt_track(const float o[3], const float d[3], float t, float tf, float tau, float density, float amax,
                         const McGeom& g, float& tc, float& maj) {
  if constexpr (!MC) {
    const float m = __fmul_rn(density, amax);
    if (!(m > 0.0f)) return false;
    const float tt = __fadd_rn(t, __fdiv_rn(tau, m));
    if (!(tt < tf)) return false;
    tc = tt;
    maj = m;
    return true;
  } else {
    int ca[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float pa = clamp01(__fadd_rn(o[a], __fmul_rn(t, d[a])));
      const int c = (int)floorf(__fmul_rn(pa, (float)g.dims[a])) / g.cell;
      ca[a] = c < g.m[a] - 1 ? c : g.m[a] - 1;
    }
    float acc = 0.0f;
    const int iters = g.m[0] + g.m[1] + g.m[2] + 3;
    for (int it = 0; it < iters; ++it) {
      float ta[3], tb = tf;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        ta[a] = INFINITY;
        if (d[a] > 0.0f) {
          int b = (ca[a] + 1) * g.cell;
          b = b < g.dims[a] ? b : g.dims[a];
          ta[a] = __fdiv_rn(__fsub_rn(__fdiv_rn((float)b, (float)g.dims[a]), o[a]), d[a]);
        } else if (d[a] < 0.0f) {
          ta[a] = __fdiv_rn(__fsub_rn(__fdiv_rn((float)(ca[a] * g.cell), (float)g.dims[a]), o[a]), d[a]);
        }
        tb = fminf(tb, ta[a]);
      }
      float seg = __fsub_rn(tb, t);
      if (seg < 0.0f) seg = 0.0f;
      const float m = __fmul_rn(density, g.mu[(ca[2] * g.m[1] + ca[1]) * g.m[0] + ca[0]]);
      const float dtau = __fmul_rn(m, seg);
      if (m > 0.0f && __fadd_rn(acc, dtau) > tau) {
        tc = __fadd_rn(t, __fdiv_rn(__fsub_rn(tau, acc), m));
        maj = m;
        return true;
      }
      acc = __fadd_rn(acc, dtau);
      if (!(tb < tf)) return false;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        if (d[a] != 0.0f && ta[a] == tb) {
          ca[a] += d[a] > 0.0f ? 1 : -1;
          if (ca[a] < 0 || ca[a] >= g.m[a]) return false;
        }
      t = tb;
    }
    return false;
  }
}

}  // namespace

template <int P, int F, int KIN, int W, typename TT, bool MC>
__global__ void __launch_bounds__(256) k_render_pt(ModelDesc md, TablePtrs tp, const float* __restrict__ mlp,
                                                   RenderArgs ra) {
  typedef typename Prec<P>::Frag Frag;
  typedef typename Prec<P>::T T;
  typedef WeightLayout<P, KIN, W> WL;
  extern __shared__ __align__(16) unsigned char smem[];
  Frag* lds_frag = reinterpret_cast<Frag*>(smem);
  const size_t wbytes = (size_t)WL::frags(md.n_hidden, false) * 64 * sizeof(Frag);
  float* lds_wout = reinterpret_cast<float*>(smem + wbytes);
  float* lds_lut = reinterpret_cast<float*>(smem + wbytes + wout_region_bytes<P, W>());  // [256][4]
  const size_t stage_off = (wbytes + wout_region_bytes<P, W>() + 4096 + 15) & ~(size_t)15;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  T* stage = reinterpret_cast<T*>(smem + stage_off + wave * Stage<P, KIN>::wave_bytes);
  T* row = stage + lane * Stage<P, KIN>::pitch;

  stage_weights<P, KIN, W>(md, mlp, lds_frag, lds_wout, false);
  for (int i = threadIdx.x; i < 1024; i += blockDim.x) lds_lut[i] = ra.lut[i];
  __syncthreads();

  const TT* table = table_ptr<TT>(tp);
  float amax = 0.0f;
  for (int i = 0; i < 256; ++i) amax = fmaxf(amax, lds_lut[4 * i + 3]);
  float lhat[3];
  unit3(ra.light, lhat);
  const float density = ra.density;
  float E4[3], B[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    E4[c] = ra.radiance[c] * kInv4Pi;
    B[c] = ra.background[c];
  }
  const int band0 = blockIdx.x % kBands;
  const int64_t n_pix = (int64_t)ra.width * ra.height;
  const uint64_t seed = (uint64_t)ra.seed;
  const int spp = ra.spp;

  // the lane's pixel (-2 while it waits for one, -1 once the frame has none
  // left) and path
  PixelPool pool = pool_init();
  int32_t pix = -2;
  int s = 0;
  bool fresh = true;
  uint64_t key = 0;
  uint32_t di = 0, psamp = 0;
  int shadow = 0, depth = 0;
  float o[3] = {0.0f, 0.0f, 0.0f}, d[3] = {0.0f, 0.0f, 1.0f}, xs[3] = {0.0f, 0.0f, 0.0f}, t = 0.0f, tf = 0.0f;
  float beta[3] = {1.0f, 1.0f, 1.0f}, L[3] = {0.0f, 0.0f, 0.0f};
  uint32_t hits = 0, nreal = 0, nsamp = 0;
  unsigned long long n_eval = 0, n_real_tot = 0, n_paths = 0;

  auto draw = [&]() -> float { return rng_u01(seed, 8u, key + (uint64_t)di++); };
  auto end_path = [&]() {
    ++n_paths;
    fresh = true;
    if (++s < spp) return;
    float4* o4 = reinterpret_cast<float4*>(ra.rgba) + pix;
    const float fs = (float)spp;
    *o4 = make_float4(L[0] / fs, L[1] / fs, L[2] / fs, (float)hits / fs);
    if (ra.n_geo) ra.n_geo[pix] = nreal;
    if (ra.n_used) ra.n_used[pix] = nsamp;
    n_real_tot += nreal;
    s = 0;
    L[0] = L[1] = L[2] = 0.0f;
    hits = nreal = nsamp = 0;
    pix = -2;  // a new pixel comes from the wave's tiles next round
  };
  auto add = [&](const float* r) {
#pragma unroll
    for (int c = 0; c < 3; ++c) L[c] = __builtin_fmaf(beta[c], r[c], L[c]);
  };
  // the path continues as a scattering ray from xs in a new direction drawn
  // from the isotropic phase function
  auto new_direction = [&]() {
    shadow = 0;
    if (depth >= ra.max_depth) {
      end_path();
      return;
    }
    const float u1 = draw(), u2 = draw();
    const float z = __fsub_rn(1.0f, __fmul_rn(2.0f, u1));
    const double rr = sqrt(fmax(0.0, 1.0 - (double)z * (double)z));
    const double ph = kTwoPi * (double)u2;
    o[0] = xs[0];
    o[1] = xs[1];
    o[2] = xs[2];
    d[0] = (float)(rr * cos(ph));
    d[1] = (float)(rr * sin(ph));
    d[2] = z;
    slab(o, d, t, tf);
    if (!(t < tf)) {
      add(B);
      end_path();
    }
  };

  for (;;) {
    // lanes whose pixel is done take the next pixels of the wave's tiles
    {
      const bool want = pix == -2;
      const int32_t p = pool_take(pool, want, ra.queue, band0, ra.width, ra.height);
      if (want) {
        pix = p >= 0 ? p : -1;
        s = 0;
        fresh = true;
      }
    }
    // sample: advance the path to its next tentative collision
    bool cand = false;
    float x[3] = {0.5f, 0.5f, 0.5f}, tc = 0.0f, maj = 0.0f;
    while (pix >= 0) {
      if (fresh) {
        fresh = false;
        key = ((uint64_t)pix * (uint64_t)spp + (uint64_t)s) << 24;
        di = psamp = 0;
        shadow = depth = 0;
        beta[0] = beta[1] = beta[2] = 1.0f;
        camera_dir(ra.cam, pix % ra.width, pix / ra.width, d);
        o[0] = ra.cam[0];
        o[1] = ra.cam[1];
        o[2] = ra.cam[2];
        slab(o, d, t, tf);
        if (!(t < tf)) {
          add(B);
          end_path();
          continue;
        }
      }
      if (psamp >= kPtMaxSamples) {
        end_path();
        continue;
      }
      const float zeta = draw();
      const float tau = (float)(-log(1.0 - (double)zeta));
      if (pt_track<MC>(o, d, t, tf, tau, density, amax, ra.mc, tc, maj)) {
#pragma unroll
        for (int a = 0; a < 3; ++a) x[a] = __fadd_rn(o[a], __fmul_rn(tc, d[a]));
        cand = true;
        break;
      }
      if (!shadow) {  // the scattering ray leaves the cube
        add(B);
        end_path();
        continue;
      }
      add(E4);  // the shadow ray reaches the light
      new_direction();
    }
    if (!__any(cand)) {
      if (__any(pix == -2)) continue;  // pixels finished without a collision this round
      break;
    }

    // batch inference: the wave's 64 collision points through the network
    encode_row<P, F, KIN>(md, table, clamp01(x[0]), clamp01(x[1]), clamp01(x[2]), row, [](int, const Oct<P>&) {});
    wave_sync();
    const float y = mlp_wave64<P, KIN, W>(md.n_hidden, md.out_relu != 0, lds_frag, lds_wout, stage);
    wave_sync();

    // shade: real or null collision, and the path's next state
    if (cand) {
      ++n_eval;
      ++nsamp;
      ++psamp;
      float c4[4];
      tf_lookup(lds_lut, y, c4);
      const float xi = draw();
      if (!(__fmul_rn(xi, maj) < __fmul_rn(density, c4[3]))) {
        t = tc;  // null collision: the ray goes on
      } else {
        ++nreal;
        if (shadow) {
          new_direction();  // the light is blocked
        } else {
          if (depth == 0) ++hits;
          ++depth;
          bool alive = true;
          if (depth > ra.rr_depth) {
            const float q = fminf(1.0f, fmaxf(beta[0], fmaxf(beta[1], beta[2])));
            if (draw() >= q) {
              end_path();
              alive = false;
            } else {
#pragma unroll
              for (int c = 0; c < 3; ++c) beta[c] = beta[c] / q;
            }
          }
          if (alive) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              beta[a] = beta[a] * c4[a];
              xs[a] = x[a];
              o[a] = x[a];
              d[a] = lhat[a];
            }
            shadow = 1;
            slab(o, d, t, tf);
            if (!(t < tf)) {
              add(E4);
              new_direction();
            }
          }
        }
      }
    }
  }
  if (ra.counters) {
    const unsigned long long e = (unsigned long long)wave_sum((double)n_eval);
    const unsigned long long r = (unsigned long long)wave_sum((double)n_real_tot);
    const unsigned long long q = (unsigned long long)wave_sum((double)n_paths);
    if (lane == 0) {
      atomicAdd(ra.counters + 0, e);
      atomicAdd(ra.counters + 1, r);
      atomicAdd(ra.counters + 2, q);
    }
  }
}

#if NGV_PRIMARY
size_t render_pt_lds_bytes(const ngvol_plan* plan, int waves) {
  const size_t esz = plan->layout.precision ? 2 : 4;
  const size_t stage = (size_t)64 * (plan->kin + 16 / esz) * esz;
  const size_t off = (mlp_weight_bytes(plan) + wout_bytes(plan) + 4096 + 15) & ~(size_t)15;
  return off + (size_t)waves * stage;
}
#endif

template <int P, int W>
hipError_t launch_render_pt_p(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const RenderArgs& ra,
                              hipStream_t st) {
  const ModelDesc& md = plan->md;
  const size_t lds = render_pt_lds_bytes(plan, 4);
  const int64_t n_pix = (int64_t)ra.width * ra.height;
  int64_t grid = (n_pix + 255) / 256;
  const int64_t cap = (int64_t)plan->cus * 8;
  if (grid > cap) grid = cap;
  if (grid < 1) grid = 1;
#define NGV_PT_GO(TT, MCB)                                                                                       \
  hipLaunchKernelGGL((k_render_pt<P, F, KIN, W, TT, MCB>), dim3((unsigned)grid), dim3(256), lds, st, md, tp, mlp, ra)
  NGV_DISPATCH_F_KIN(md.F, plan->kin, {
    const bool mc = ra.mc.mu != nullptr;
    if (tp.f16) {
      if (mc) NGV_PT_GO(__half, true);
      else NGV_PT_GO(__half, false);
    } else {
      if (mc) NGV_PT_GO(float, true);
      else NGV_PT_GO(float, false);
    }
  });
#undef NGV_PT_GO
  return hipGetLastError();
}

template hipError_t launch_render_pt_p<NGV_PSEL, NGV_WSEL>(const ngvol_plan*, TablePtrs, const float*,
                                                           const RenderArgs&, hipStream_t);

}  // namespace ngvol
