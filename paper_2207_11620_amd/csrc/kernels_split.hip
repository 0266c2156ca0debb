// Level groups, one per XCD: the encoding of Section 3.1 and the network of
// Section 3.2 evaluated in two passes for large query sets.
//
// At the paper's sizes the FP16 tables (16 levels of up to 2^19 entries,
// 24 MB) exceed the L2 of one XCD (4 MB), and the entries a hashed level
// needs for any region of space are spread over its whole table, so when
// every XCD evaluates all levels for its share of the queries most gathers
// miss its L2.  Here XCD x evaluates only its own group of levels
// {x, x+8, ...} for all queries, so its gathers stay in its own L2; the
// round-robin groups pair a coarse level (many queries share its corner
// lines) with a fine one, which balances the XCDs.
//   1. k_level_feat: the workgroups placed on XCD x (blockIdx % 8 == x, the
//      hardware's round-robin placement of workgroups) interpolate their
//      levels and write them, in the MLP's operand type, into their group's
//      own plane [query][group levels][F] - one store per query, and no
//      cache line shared with another XCD's writes;
//   2. k_mlp_planes: the network on the planes, with the next tiles' features
//      loaded while the current ones are evaluated; each result goes to the
//      query's original slot.  Its first-layer operands take the features in
//      plane order (the columns of W0 are permuted to match when staged), so
//      a lane reads its 8 features as whole group entries.
// Features are converted to the operand type exactly as in the fused
// kernel; the products of the first layer are summed in another order, so
// outputs agree with the fused kernel to FP32 rounding, not bitwise.
// build: one object per MLP precision and width (NGV_PSEL, NGV_WSEL)
#include <type_traits>

#include "kernels.hpp"
#include "dispatch.hpp"
#include "mlp_tile.hpp"

namespace ngvol {

namespace {

template <int BYTES>
struct alignas(BYTES < 16 ? BYTES : 16) Bytes {
  uint32_t w[BYTES / 4];
};

template <int F, typename OT, int NL>
struct alignas(NL * F * sizeof(OT) <= 16 ? NL * F * sizeof(OT) : 16) LevelPack {
  OT v[NL * F];
};

// Plane element of (query q, level l, feature 0): group l % 8 (level l
// itself when L < 8) holds its levels l, l+8, ... side by side, gw per query.
__device__ __forceinline__ int64_t plane_elem(int64_t q, int l, int F, int gw, int64_t m) {
  const int x = l & 7, i = l >> 3;
  return ((int64_t)x * m * gw + q * gw + i) * F;
}

template <int F, typename TT, typename OT>
__global__ void __launch_bounds__(256) k_level_feat(ModelDesc md, const TT* __restrict__ table,
                                                    const float4* __restrict__ rec, int64_t m,
                                                    OT* __restrict__ planes, uint32_t* __restrict__ idx,
                                                    SplitArgs sa) {
  const int x = blockIdx.x & 7;
  const int r = blockIdx.x >> 3;
  const int nbx = (int)((gridDim.x - x + 7) >> 3);  // workgroups on this XCD
  const int wpb = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l0 = sa.first[x], nl = sa.count[x], gw = sa.width;
  if (nl == 0) return;
  const uint32_t n_ent = (uint32_t)(md.n_table / F);
  const int64_t chunks = (m + 63) >> 6;
  const int64_t c_lo = chunks * sa.part[x] / sa.parts[x];
  const int64_t c_hi = chunks * (sa.part[x] + 1) / sa.parts[x];
  // the XCDs holding level 0 also write the queries' slots
  const bool write_idx = l0 == 0;
  for (int64_t c = c_lo + (int64_t)r * wpb + wave; c < c_hi; c += (int64_t)nbx * wpb) {
    const int64_t q = c * 64 + lane;
    const bool valid = q < m;
    const float4 rr = rec[valid ? q : m - 1];
    const float px = clamp01(rr.x), py = clamp01(rr.y), pz = clamp01(rr.z);
    if (write_idx && valid) idx[q] = __float_as_uint(rr.w);
    OT* dst = planes + plane_elem(q, l0, F, gw, m);
    if (nl == 2 && gw == 2) {
      LevelPack<F, OT, 2> pk;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        Corners cr;
        level_corners(md.lv[l0 + 8 * i], px, py, pz, cr);
        float acc[F];
        gather_level<F>(cr, table, n_ent, acc);
#pragma unroll
        for (int f = 0; f < F; ++f) pk.v[i * F + f] = (OT)acc[f];
      }
      if (valid) *reinterpret_cast<LevelPack<F, OT, 2>*>(dst) = pk;
    } else {
      for (int i = 0; i < gw; ++i) {
        LevelPack<F, OT, 1> pk;
        if (i < nl) {
          Corners cr;
          level_corners(md.lv[l0 + 8 * i], px, py, pz, cr);
          float acc[F];
          gather_level<F>(cr, table, n_ent, acc);
#pragma unroll
          for (int f = 0; f < F; ++f) pk.v[f] = (OT)acc[f];
        } else {
#pragma unroll
          for (int f = 0; f < F; ++f) pk.v[f] = (OT)0.0f;  // padding slot of a short group
        }
        if (valid) *reinterpret_cast<LevelPack<F, OT, 1>*>(dst + i * F) = pk;
      }
    }
  }
}

// Plane order of the features: entry e = gw*F features of plane group x
// (levels x, x+8, ... for L >= 8; level x for L < 8), feature p = x*E + i*F + f.
struct PlaneOrder {
  int8_t col[64];  // input feature of plane-order position p (-1: none)
};

// EC: entry class of the planes, 0 for entries of 8 or more features, else
// the entry size (4 or 2 features); FULL: the planes hold all KIN features
// (no zero padding to supply).
template <int P, int F, int KIN, int W, typename OT, int EC, bool FULL, int NHC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(mlp_waves_per_eu(P, KIN, NHC))))
k_mlp_planes(ModelDesc md, const float* __restrict__ mlp, const OT* __restrict__ planes,
             const uint32_t* __restrict__ idx, int64_t m, float* __restrict__ out, PlaneOrder po, int E,
             int n_plane_feat) {
  constexpr int NB = 2;
  constexpr int CH0 = InChunks<P, KIN>::n;
  constexpr int DW = 8 * (int)sizeof(OT) / 4;  // dwords of one 8-feature block
  typedef typename Prec<P>::Frag Frag;
  typedef WeightLayout<P, KIN, W> WL;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int8_t colmap[64];
  if (threadIdx.x < 64) colmap[threadIdx.x] = po.col[threadIdx.x];
  __syncthreads();
  Frag* lds_frag = reinterpret_cast<Frag*>(smem);
  float* lds_wout = reinterpret_cast<float*>(smem + (size_t)WL::frags(md.n_hidden, false) * 64 * sizeof(Frag));
  stage_weights<P, KIN, W>(md, mlp, lds_frag, lds_wout, false, colmap);
  __syncthreads();
  const int lane = threadIdx.x & 63, nl = lane & 15, g = lane >> 4;
  const int64_t n_groups = (m + 16 * NB - 1) / (16 * NB);
  TileIter it(n_groups);
  struct Raw {
    uint32_t d[NB][KIN / 32][DW];
    uint32_t slot[NB];
  };
  // DWS-dword load (1, 2 or 4) at element offset o of the planes
  auto load1 = [&](int64_t o, uint32_t* w) { w[0] = *reinterpret_cast<const uint32_t*>(planes + o); };
  auto load2 = [&](int64_t o, uint32_t* w) {
    const uint2 t = *reinterpret_cast<const uint2*>(planes + o);
    w[0] = t.x;
    w[1] = t.y;
  };
  auto load4 = [&](int64_t o, uint32_t* w) {
    const uint4 t = *reinterpret_cast<const uint4*>(planes + o);
    w[0] = t.x;
    w[1] = t.y;
    w[2] = t.z;
    w[3] = t.w;
  };
  constexpr int EPD = 4 / (int)sizeof(OT);  // elements per dword
  mlp_stream<P, KIN, W, NB, Raw, NHC>(
      md.n_hidden, md.out_relu != 0, lds_frag, lds_wout, it.next, it.step, it.end,
      [&](int64_t grp, Raw& r) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          int64_t s = (grp * NB + nb) * 16 + nl;
          s = s < m ? s : m - 1;
          r.slot[nb] = idx[s];
#pragma unroll
          for (int b = 0; b < KIN / 32; ++b) {
            uint32_t* d = r.d[nb][b];
            const int p0 = 32 * b + 8 * g;  // this lane's plane-order features p0 .. p0+7
            if constexpr (!FULL) {
#pragma unroll
              for (int k = 0; k < DW; ++k) d[k] = 0u;
            }
            if constexpr (EC == 0) {
              // the block lies inside entry p0 / E
              if (FULL || p0 < n_plane_feat) {
                const int64_t o = ((int64_t)(p0 / E) * m + s) * E + p0 % E;
#pragma unroll
                for (int k = 0; k < DW; k += 4) load4(o + k * EPD, d + k);
              }
            } else if constexpr (EC == 4) {
              // two entries of 4 features
#pragma unroll
              for (int j = 0; j < 2; ++j) {
                const int p = p0 + 4 * j;
                if (FULL || p < n_plane_feat) {
                  const int64_t o = ((int64_t)(p / 4) * m + s) * 4;
                  if constexpr (EPD == 2) load2(o, d + 2 * j);
                  else load4(o, d + 4 * j);
                }
              }
            } else {
              // four entries of 2 features (EC == 2)
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                const int p = p0 + 2 * j;
                if (FULL || p < n_plane_feat) {
                  const int64_t o = ((int64_t)(p / 2) * m + s) * 2;
                  if constexpr (EPD == 2) load1(o, d + j);
                  else load2(o, d + 2 * j);
                }
              }
            }
          }
        }
      },
      [&](const Raw& r, Frag (*in)[CH0]) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int b = 0; b < KIN / 32; ++b) {
            if constexpr (P) {
              Bytes<16> t;
#pragma unroll
              for (int k = 0; k < 4; ++k) t.w[k] = r.d[nb][b][k];
              in[nb][b] = __builtin_bit_cast(Frag, t);
            } else {
#pragma unroll
              for (int jj = 0; jj < 8; ++jj) in[nb][8 * b + jj] = __uint_as_float(r.d[nb][b][jj]);
            }
          }
      },
      [&](int64_t grp, int nb, float y, const Raw& r) {
        const int64_t s = (grp * NB + nb) * 16 + nl;
        if (s < m && g == 0) out[r.slot[nb]] = y;
      });
}

}  // namespace

#if NGV_PRIMARY
bool use_split(const ngvol_plan* plan, int64_t n) {
  // worth it when the queries are many and the FP16 tables exceed one XCD's L2
  return n >= ((int64_t)1 << 20) && plan->md.L >= 2 && (int64_t)plan->md.n_table * 2 > ((int64_t)4 << 20);
}
#endif

static SplitArgs split_args(const ngvol_plan* plan) {
  SplitArgs sa{};
  const int L = plan->md.L;
  sa.width = L >= 8 ? (L + 7) / 8 : 1;
  for (int x = 0; x < 8; ++x) {
    if (L >= 8) {
      // levels x, x+8, ... (the plane group x of plane_elem)
      sa.first[x] = x;
      sa.count[x] = (L - x + 7) / 8;
      sa.part[x] = 0;
      sa.parts[x] = 1;
    } else {
      // fewer levels than XCDs: a level's queries are shared by the XCDs holding it
      const int l = x % L;
      sa.first[x] = l;
      sa.count[x] = 1;
      sa.part[x] = x / L;
      sa.parts[x] = (8 - l + L - 1) / L;
    }
  }
  return sa;
}

static int split_operand_bytes(const ngvol_plan* plan) { return plan->layout.precision ? 2 : 4; }

static int64_t plane_levels(const ngvol_plan* plan) {
  // levels of plane storage per query: 8 groups of equal width (or L < 8 single levels)
  const int L = plan->md.L;
  return L >= 8 ? 8 * ((L + 7) / 8) : L;
}

#if NGV_PRIMARY
int64_t split_slab(const ngvol_plan* plan, int64_t n) {
  // planes of at most 1 GiB (or 2^20 queries) per pass, in whole 64-query chunks
  const int64_t per_query = plane_levels(plan) * plan->md.F * split_operand_bytes(plan);
  int64_t slab = ((int64_t)1 << 30) / per_query;
  if (slab < ((int64_t)1 << 20)) slab = (int64_t)1 << 20;
  slab &= ~(int64_t)63;
  return slab < n ? slab : n;
}

size_t split_planes_bytes(const ngvol_plan* plan, int64_t n) {
  return (size_t)split_slab(plan, n) * plane_levels(plan) * plan->md.F * split_operand_bytes(plan);
}
#endif

template <int P, int W>
hipError_t launch_infer_split_p(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const float4* rec, int64_t n,
                                float* out, void* planes, uint32_t* idx, hipStream_t st) {
  const ModelDesc& md = plan->md;
  const SplitArgs sa = split_args(plan);
  const int64_t slab = split_slab(plan, n);
  const size_t lds = fwd_lds_bytes(plan);
  // plane order of the MLP's input columns
  const int L = md.L, F_ = md.F;
  const int E = sa.width * F_;
  const int n_plane_feat = (L >= 8 ? 8 : L) * E;
  PlaneOrder po;
  for (int p = 0; p < 64; ++p) {
    int col = -1;
    if (p < n_plane_feat) {
      const int x = p / E, i = (p % E) / F_, f = p % F_;
      const int l = L >= 8 ? x + 8 * i : x;
      if (l < L) col = l * F_ + f;
    }
    po.col[p] = (int8_t)col;
  }
#define NGV_MP(EC, FULL)                                                                                        \
  do {                                                                                                          \
    if (md.n_hidden == 2)                                                                                       \
      hipLaunchKernelGGL((k_mlp_planes<P, F, KIN, W, OT, EC, FULL, 2>), dim3((unsigned)mgrid), dim3(256), lds, st, \
                         md, mlp, pl, idx, m, out, po, E, n_plane_feat);                                        \
    else                                                                                                        \
      hipLaunchKernelGGL((k_mlp_planes<P, F, KIN, W, OT, EC, FULL, 0>), dim3((unsigned)mgrid), dim3(256), lds, st, \
                         md, mlp, pl, idx, m, out, po, E, n_plane_feat);                                        \
  } while (0)
  for (int64_t s0 = 0; s0 < n; s0 += slab) {
    const int64_t m = n - s0 < slab ? n - s0 : slab;
    const int64_t chunks = (m + 63) / 64;
    int64_t per_xcd = (chunks + 3) / 4;
    if (per_xcd > plan->cus) per_xcd = plan->cus;
    if (per_xcd < 1) per_xcd = 1;
    const dim3 lgrid((unsigned)(8 * per_xcd));
    int64_t mgrid = (m + 511) / 512;  // about 4 groups of 32 queries per wave
    if (mgrid > (int64_t)plan->cus * 8) mgrid = (int64_t)plan->cus * 8;
    if (mgrid < 1) mgrid = 1;
    const float4* r = rec + s0;
    NGV_DISPATCH_F_KIN(md.F, plan->kin, {
      typedef typename std::conditional<P == 0, float, typename Prec<P>::T>::type OT;
      OT* pl = reinterpret_cast<OT*>(planes);
      if (tp.f16)
        hipLaunchKernelGGL((k_level_feat<F, __half, OT>), lgrid, dim3(256), 0, st, md, tp.f16, r, m, pl, idx, sa);
      else
        hipLaunchKernelGGL((k_level_feat<F, float, OT>), lgrid, dim3(256), 0, st, md, tp.f32, r, m, pl, idx, sa);
      const bool full = n_plane_feat >= KIN;
      if (E >= 8) {
        if (full) NGV_MP(0, true);
        else NGV_MP(0, false);
      } else if (E == 4) {
        if (full) NGV_MP(4, true);
        else NGV_MP(4, false);
      } else {
        if (full) NGV_MP(2, true);
        else NGV_MP(2, false);
      }
    });
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
#undef NGV_MP
  return hipSuccess;
}

template hipError_t launch_infer_split_p<NGV_PSEL, NGV_WSEL>(const ngvol_plan*, TablePtrs, const float*, const float4*, int64_t,
                                                   float*, void*, uint32_t*, hipStream_t);

#if NGV_PRIMARY
hipError_t launch_infer_split(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const float4* rec, int64_t n,
                              float* out, void* planes, uint32_t* idx, hipStream_t st) {
  NGV_DISPATCH_P(plan->layout.precision,
                 NGV_DISPATCH_W(plan->md.width, return launch_infer_split_p<P, W>(plan, tp, mlp, rec, n, out, planes, idx, st)));
  return hipErrorInvalidValue;
}
#endif

}  // namespace ngvol
