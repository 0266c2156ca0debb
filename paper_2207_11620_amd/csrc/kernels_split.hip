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
//      cache line shared with another XCD's writes.  For plans of 9..16
//      levels k_level_brick (below) takes its place: it works on level pairs
//      over spatial bricks, staging the levels that fit in LDS, and spreads
//      the fully staged pairs over all XCDs;
//   2. k_mlp_planes: the network on the planes, with the next tiles' features
//      loaded while the current ones are evaluated; each result goes to the
//      query's original slot.  Its first-layer operands take the features in
//      plane order (the columns of W0 are permuted to match when staged), so
//      a lane reads its 8 features as whole group entries.
// Features are converted to the operand type exactly as in the fused
// kernel; the products of the first layer are summed in another order, so
// outputs agree with the fused kernel to FP32 rounding, not bitwise.
// build: one object per MLP precision and width (NGV_PSEL, NGV_WSEL)
#include <cmath>
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

// ---------------------------------------------------------------------------
// Brick-staged level groups.  The grouped records come in Morton order of
// 2^k cells per axis (bins), so the records of one cell of space (a brick of
// 1/2^k per axis) are one contiguous range.  For a level whose vertices over
// a brick fit in LDS, the workgroup first copies that box of vertices from
// the table into LDS - rows of consecutive vertices, whose slots (dense, or
// hashed with an x prime of 1) lie in a few aligned blocks, so a wave's loads
// touch a few cache lines - and then reads every query's 8 corners from LDS.
// Corner values, weights and the order of the interpolation are those of
// gather_level, so the features are bitwise the same; levels whose box does
// not fit are gathered from the table as before.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int compact3(uint32_t v) {
  v &= 0x09249249u;
  v = (v ^ (v >> 2)) & 0x030C30C3u;
  v = (v ^ (v >> 4)) & 0x0300F00Fu;
  v = (v ^ (v >> 8)) & 0x030000FFu;
  v = (v ^ (v >> 16)) & 0x000003FFu;
  return (int)v;
}

// Vertex range of level resolution N over brick coordinate q (of 2^k): the
// cells of the points with floor(x 2^k) = q are min(floor(x (N-1)), N-2) in
// [lo, hi], so the corners lie in [lo, hi + 1].
__host__ __device__ __forceinline__ void brick_range(int N, int q, int k, int& lo, int& n) {
  lo = (q * (N - 1)) >> k;
  int hi = ((q + 1) * (N - 1)) >> k;
  hi = hi < N - 2 ? hi : N - 2;
  n = hi - lo + 2;
}

struct BrickBox {
  int lo[3], n[3];
};

// e / d for 0 <= e < 2^22 and d >= 1, from a float reciprocal: the
// product is within one of the quotient, which one step corrects.
__device__ __forceinline__ int small_div(int e, int d, float inv) {
  int q = (int)((float)e * inv);
  const int r = e - q * d;
  q += r >= d ? 1 : (r < 0 ? -1 : 0);
  return q;
}

// Copy the vertices of level lv over brick (bq) into LDS dst[z][y][x][ED].
template <int ED, typename TT>
__device__ __forceinline__ void stage_box(const LevelDesc& lv, const TT* __restrict__ table, const BrickBox& bb,
                                          uint32_t* __restrict__ dst) {
  constexpr int U = 8;  // entries per thread per round: their loads are in flight together
  const int nx = bb.n[0], nxy = bb.n[0] * bb.n[1], total = nxy * bb.n[2];
  const float inx = 1.0f / (float)nx, inxy = 1.0f / (float)nxy;
  const void* base = table;
  for (int e0 = threadIdx.x; e0 < total; e0 += (int)blockDim.x * U) {
    uint32_t d[U][ED];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * (int)blockDim.x;
      const int ee = e < total ? e : 0;
      const int iz = small_div(ee, nxy, inxy), rem = ee - iz * nxy, iy = small_div(rem, nx, inx), ix = rem - iy * nx;
      const uint32_t slot = lv.offset + level_slot(lv, (uint32_t)(bb.lo[0] + ix), (uint32_t)(bb.lo[1] + iy),
                                                   (uint32_t)(bb.lo[2] + iz));
      load_entry<ED>(base, slot, d[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * (int)blockDim.x;
      if (e < total) {
#pragma unroll
        for (int q = 0; q < ED; ++q) dst[e * ED + q] = d[u][q];
      }
    }
  }
}

// F features of one level for a point, from the level's box in LDS.
template <int F, typename TT>
__device__ __forceinline__ void lookup_box(const LevelDesc& lv, const BrickBox& bb, const uint32_t* __restrict__ box,
                                           float x, float y, float z, float acc[F]) {
  constexpr int ED = Entry<F, TT>::ED;
  Cell cl;
  level_cell(lv, x, y, z, cl);
  const int nx = bb.n[0], nxy = bb.n[0] * bb.n[1];
  const int li = (cl.c[0] - bb.lo[0]) + nx * ((cl.c[1] - bb.lo[1]) + bb.n[1] * (cl.c[2] - bb.lo[2]));
  float v[8][F];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int e = li + (k & 1) + ((k >> 1) & 1) * nx + ((k >> 2) & 1) * nxy;
    uint32_t d[ED];
#pragma unroll
    for (int q = 0; q < ED; ++q) d[q] = box[e * ED + q];
    entry_values<F, TT>(d, v[k]);
  }
#pragma unroll
  for (int f = 0; f < F; ++f) acc[f] = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int f = 0; f < F; ++f) acc[f] = __builtin_fmaf(cl.w[k], v[k][f], acc[f]);
}

template <int F, typename TT, typename OT>
__global__ void __launch_bounds__(256) k_level_brick(ModelDesc md, const TT* __restrict__ table,
                                                     const float4* __restrict__ rec, int64_t s0, int64_t m,
                                                     OT* __restrict__ planes, uint32_t* __restrict__ idx,
                                                     BrickArgs ba) {
  constexpr int ED = Entry<F, TT>::ED;
  extern __shared__ __align__(16) uint32_t lds[];
  const int x = blockIdx.x & 7;
  const int r = blockIdx.x >> 3;
  const int nbx = (int)((gridDim.x - x + 7) >> 3);  // workgroups on this XCD
  const uint32_t n_ent = (uint32_t)(md.n_table / F);
  const int gw = ba.gw;
  // the XCD's items: an eighth of the bricks of each of the first n_shared
  // pairs of the list, spread evenly among its segment of the (pair, brick)
  // items of the others, pair-major
  const int slice = ba.n_bins >> 3;
  const int n_sh = ba.n_shared * slice;
  const int o_lo = ba.item_lo[x], n_all = n_sh + (ba.item_lo[x + 1] - o_lo);
  for (int v = r; v < n_all; v += nbx) {
    const int js = (int)((int64_t)v * n_sh / n_all), js1 = (int)((int64_t)(v + 1) * n_sh / n_all);
    const int it = js1 > js ? (js / slice) * ba.n_bins + x * slice + js % slice : o_lo + (v - js);
    const int p = it / ba.n_bins, b = it - p * ba.n_bins;
    const int la = ba.lev[p][0], lb = ba.lev[p][1];
    const int64_t g0 = (int64_t)ba.bin_off[b], g1 = g0 + (int64_t)ba.bin_cnt[b];
    const int64_t q0 = g0 - s0 > 0 ? g0 - s0 : 0, q1 = g1 - s0 < m ? g1 - s0 : m;
    if (q0 >= q1) continue;  // uniform over the workgroup
    const LevelDesc lva = md.lv[la], lvb = md.lv[lb >= 0 ? lb : la];  // held in registers over the item
    const bool sa = ba.lds_off[p][0] >= 0, sb = lb >= 0 && ba.lds_off[p][1] >= 0;
    const bool write_idx = la == 0;  // the pair holding level 0 also writes the queries' slots
    const int bq[3] = {compact3((uint32_t)b), compact3((uint32_t)b >> 1), compact3((uint32_t)b >> 2)};
    BrickBox bba, bbb;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      brick_range(lva.N, bq[a], ba.k, bba.lo[a], bba.n[a]);
      brick_range(lvb.N, bq[a], ba.k, bbb.lo[a], bbb.n[a]);
    }
    const uint32_t* box_a = lds + (sa ? ba.lds_off[p][0] / 4 : 0);
    const uint32_t* box_b = lds + (sb ? ba.lds_off[p][1] / 4 : 0);
    __syncthreads();  // the previous item's boxes are no longer read
    if (sa) stage_box<ED>(lva, table, bba, lds + ba.lds_off[p][0] / 4);
    if (sb) stage_box<ED>(lvb, table, bbb, lds + ba.lds_off[p][1] / 4);
    __syncthreads();
    for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
      const float4 rr = rec[s0 + q];
      const float px = clamp01(rr.x), py = clamp01(rr.y), pz = clamp01(rr.z);
      if (write_idx) idx[q] = __float_as_uint(rr.w);
      LevelPack<F, OT, 2> pk;
      float acc[F];
      if (sa) {
        lookup_box<F, TT>(lva, bba, box_a, px, py, pz, acc);
      } else {
        Corners cr;
        level_corners(lva, px, py, pz, cr);
        gather_level<F>(cr, table, n_ent, acc);
      }
#pragma unroll
      for (int f = 0; f < F; ++f) pk.v[f] = (OT)acc[f];
      if (lb >= 0) {
        if (sb) {
          lookup_box<F, TT>(lvb, bbb, box_b, px, py, pz, acc);
        } else {
          Corners cr;
          level_corners(lvb, px, py, pz, cr);
          gather_level<F>(cr, table, n_ent, acc);
        }
#pragma unroll
        for (int f = 0; f < F; ++f) pk.v[F + f] = (OT)acc[f];
      } else {
#pragma unroll
        for (int f = 0; f < F; ++f) pk.v[F + f] = (OT)0.0f;  // padding slot of a short group
      }
      *reinterpret_cast<LevelPack<F, OT, 2>*>(planes + plane_elem(q, la, F, gw, m)) = pk;
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

// LDS a brick-staged workgroup may give to its levels' vertex boxes (four
// workgroups per compute unit).
constexpr size_t kBrickLds = 40 * 1024;

// Brick-staged levels for plans of 9..16 levels (two levels of plane storage
// per group; 8 or fewer levels have one, and take k_level_feat) whose table
// entries are at most 8 bytes.  Pair p holds levels p
// and p + 8; a level is staged when its largest box over a brick fits in what
// the pair leaves of kBrickLds.  The (pair, brick) items, pair-major, are cut
// into 8 contiguous segments of equal estimated cost, one per XCD, so that
// the XCDs whose pairs are staged share the others' gathers.  Returns false
// when the plan or the workspace does not qualify; lds = bytes the launch
// needs.
//
// Estimated cost of one level over all queries, in units of a staged level
// (whose per-query arithmetic bounds it).  A gathered level costs more the
// fewer corner lines neighbouring queries share: with rho = cells of the
// level per mean query spacing, (N - 1) / n^(1/3), the cost measured on
// MI355X (2^24 grouped queries, levels of 406 to 2047 cells, FP16 tables)
// follows 4.2 - 3.92 exp(-rho / 2) within 2 %; it is kept above the cost of
// a staged level.
static double level_cost(int N, int64_t n, bool staged) {
  if (staged) return 1.0;
  const double rho = (double)(N - 1) / std::cbrt((double)(n > 1 ? n : 1));
  const double c = 4.2 - 3.92 * std::exp(-rho / 2.0);
  return c > 1.2 ? c : 1.2;
}

static bool brick_args(const ngvol_plan* plan, BinRanges bins, int64_t n, int entry_bytes, BrickArgs& ba,
                       size_t& lds) {
  const ModelDesc& md = plan->md;
  if (!bins.off || !bins.cnt || md.L <= 8 || md.L > 16 || entry_bytes > 8) return false;
  ba = BrickArgs{};
  ba.bin_off = bins.off;
  ba.bin_cnt = bins.cnt;
  ba.k = bins.k;
  ba.n_bins = 1 << (3 * bins.k);
  ba.gw = 2;
  lds = 0;
  double cost[8];
  for (int p = 0; p < 8; ++p) {
    size_t used = 0;
    cost[p] = 0.0;
    for (int i = 0; i < 2; ++i) {
      const int l = p + 8 * i;
      ba.lev[p][i] = l < md.L ? l : -1;
      ba.lds_off[p][i] = -1;
      if (l >= md.L) continue;
      int most = 0;
      for (int q = 0; q < (1 << bins.k); ++q) {
        int lo, cnt;
        brick_range(md.lv[l].N, q, bins.k, lo, cnt);
        most = cnt > most ? cnt : most;
      }
      const size_t bytes = ((size_t)most * most * most * entry_bytes + 15) & ~(size_t)15;
      const bool staged = used + bytes <= kBrickLds;
      if (staged) {
        ba.lds_off[p][i] = (int)used;
        used += bytes;
      }
      cost[p] += level_cost(md.lv[l].N, n, staged);
    }
    lds = used > lds ? used : lds;
  }
  // Pairs whose levels are all staged are bound by their arithmetic, the
  // others by their gathers: the former go first in the list and every XCD
  // takes an eighth of their bricks, interleaved with its segment of the
  // latter, so that each compute unit has both kinds of work in flight.
  int order[8], n_sh = 0;
  for (int p = 0; p < 8; ++p) {
    const bool shared = ba.lds_off[p][0] >= 0 && (ba.lev[p][1] < 0 || ba.lds_off[p][1] >= 0);
    if (shared) order[n_sh++] = p;
  }
  int n_list = n_sh;
  for (int p = 0; p < 8; ++p) {
    const bool shared = ba.lds_off[p][0] >= 0 && (ba.lev[p][1] < 0 || ba.lds_off[p][1] >= 0);
    if (!shared) order[n_list++] = p;
  }
  BrickArgs src = ba;
  double c2[8];
  for (int i = 0; i < 8; ++i) {
    for (int j = 0; j < 2; ++j) {
      ba.lev[i][j] = src.lev[order[i]][j];
      ba.lds_off[i][j] = src.lds_off[order[i]][j];
    }
    c2[i] = cost[order[i]];
  }
  ba.n_shared = n_sh;
  // equal-cost segments of the other pairs' items (list positions from
  // n_sh * n_bins on)
  double total = 0.0;
  for (int i = n_sh; i < 8; ++i) total += c2[i];
  const int base = n_sh * ba.n_bins;
  if (n_sh == 8) {  // every pair is shared: no segments
    for (int x = 0; x <= 8; ++x) ba.item_lo[x] = base;
    return true;
  }
  ba.item_lo[0] = base;
  int i = n_sh;
  double before = 0.0;  // cost of the list pairs before i
  for (int x = 1; x < 8; ++x) {
    const double target = total * x / 8.0;
    while (i < 7 && before + c2[i] <= target) before += c2[i++];
    const double frac = c2[i] > 0.0 ? (target - before) / c2[i] : 0.0;
    int cut = i * ba.n_bins + (int)(frac * ba.n_bins + 0.5);
    cut = cut < ba.item_lo[x - 1] ? ba.item_lo[x - 1] : cut;
    cut = cut > 8 * ba.n_bins ? 8 * ba.n_bins : cut;
    ba.item_lo[x] = cut;
  }
  ba.item_lo[8] = 8 * ba.n_bins;
  return true;
}

template <int P, int W>
hipError_t launch_infer_split_p(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const float4* rec, int64_t n,
                                float* out, void* planes, uint32_t* idx, BinRanges bins, hipStream_t st) {
  const ModelDesc& md = plan->md;
  const SplitArgs sa = split_args(plan);
  BrickArgs bk;
  size_t brick_lds = 0;
  const bool brick = brick_args(plan, bins, n, md.F * (tp.f16 ? 2 : 4), bk, brick_lds);
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
      if (brick) {
        // four workgroups per compute unit on each XCD
        int64_t per = (int64_t)bk.n_bins;
        const int64_t cap = (int64_t)plan->cus / 8 * 4;
        if (per > cap) per = cap;
        if (per < 1) per = 1;
        const dim3 bgrid((unsigned)(8 * per));
        if constexpr (F * 2 <= 8) {
          if (tp.f16)
            hipLaunchKernelGGL((k_level_brick<F, __half, OT>), bgrid, dim3(256), brick_lds, st, md, tp.f16, rec, s0,
                               m, pl, idx, bk);
        }
        if constexpr (F * 4 <= 8) {
          if (!tp.f16)
            hipLaunchKernelGGL((k_level_brick<F, float, OT>), bgrid, dim3(256), brick_lds, st, md, tp.f32, rec, s0,
                               m, pl, idx, bk);
        }
      } else if (tp.f16) {
        hipLaunchKernelGGL((k_level_feat<F, __half, OT>), lgrid, dim3(256), 0, st, md, tp.f16, r, m, pl, idx, sa);
      } else {
        hipLaunchKernelGGL((k_level_feat<F, float, OT>), lgrid, dim3(256), 0, st, md, tp.f32, r, m, pl, idx, sa);
      }
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

template hipError_t launch_infer_split_p<NGV_PSEL, NGV_WSEL>(const ngvol_plan*, TablePtrs, const float*,
                                                             const float4*, int64_t, float*, void*, uint32_t*,
                                                             BinRanges, hipStream_t);

#if NGV_PRIMARY
hipError_t launch_infer_split(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const float4* rec, int64_t n,
                              float* out, void* planes, uint32_t* idx, BinRanges bins, hipStream_t st) {
  NGV_DISPATCH_P(plan->layout.precision,
                 NGV_DISPATCH_W(plan->md.width,
                                return launch_infer_split_p<P, W>(plan, tp, mlp, rec, n, out, planes, idx, bins, st)));
  return hipErrorInvalidValue;
}
#endif

}  // namespace ngvol
