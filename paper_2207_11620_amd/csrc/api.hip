// C-ABI of libngvol: argument validation, plan construction and workspace
// carve-up.  Every step of the computation runs in the kernels; this file
// only checks arguments and enqueues launches.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <cmath>
#include <cstdlib>

#include <new>
#include <string>

#include "kernels.hpp"
#include "render.hpp"

using namespace ngvol;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

// Debug mode (NGVOL_DEBUG=1 in the environment, or ngvol_set_debug): every
// call waits for the device after its launches and reports a failure of
// theirs as its own.
std::atomic<int> g_debug{-1};

bool debug_on() {
  int d = g_debug.load(std::memory_order_relaxed);
  if (d < 0) {
    const char* e = getenv("NGVOL_DEBUG");
    d = (e && e[0] && e[0] != '0') ? 1 : 0;
    g_debug.store(d, std::memory_order_relaxed);
  }
  return d != 0;
}

// In debug mode a call on a stream that is being captured into a graph
// cannot wait for the device; it then only checks the launches' status.
int hip_check(hipError_t e, const char* what, hipStream_t st) {
  if (e == hipSuccess && debug_on()) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
      e = hipGetLastError();
    } else {
      e = hipDeviceSynchronize();
      if (e == hipSuccess) e = hipGetLastError();
    }
  }
  if (e == hipSuccess) return NGVOL_OK;
  return fail(NGVOL_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
bool aligned4(const void* p) { return ((uintptr_t)p & 3u) == 0; }

constexpr size_t kLdsBytes = kLdsLimit;  // LDS per workgroup on gfx950

#define NGV_REQUIRE(cond, ...) \
  do {                         \
    if (!(cond)) return fail(NGVOL_EINVAL, __VA_ARGS__); \
  } while (0)

int check_plan(const ngvol_plan* p) {
  if (!p) return fail(NGVOL_EINVAL, "plan is NULL");
  return NGVOL_OK;
}

// Vertices per axis: N_l = base * b^l, kept when integral (1e-9 relative),
// else rounded up; b from max_resolution when given.
int resolve_resolutions(const ngvol_config* c, int32_t* out) {
  if (c->resolutions) {
    for (int l = 0; l < c->n_levels; ++l) out[l] = c->resolutions[l];
    return NGVOL_OK;
  }
  double b = c->per_level_scale;
  if (c->max_resolution > 0)
    b = c->n_levels > 1 ? exp((log((double)c->max_resolution) - log((double)c->base_resolution)) / (c->n_levels - 1))
                        : 1.0;
  if (!(b >= 1.0) || !std::isfinite(b)) return fail(NGVOL_EINVAL, "per-level scale must be >= 1 (got %g)", b);
  for (int l = 0; l < c->n_levels; ++l) {
    const double r = (double)c->base_resolution * pow(b, (double)l);
    const double rr = floor(r + 0.5);
    const double v = fabs(r - rr) < 1e-9 * r ? rr : ceil(r);
    if (v > 65536.0) return fail(NGVOL_EINVAL, "level %d resolution %g exceeds 65536", l, v);
    out[l] = (int32_t)v;
  }
  return NGVOL_OK;
}

TablePtrs tables_of(const ngvol_plan* p, const ngvol_weights* w) {
  TablePtrs t;
  t.f32 = w->params;
  t.f16 = reinterpret_cast<const __half*>(w->table_f16);
  (void)p;
  return t;
}

// The backward keeps W, W^T, dW and per-wave activations in LDS.
int check_bwd_lds(const ngvol_plan* p) {
  const size_t b = bwd_lds_bytes(p, 1, true);
  if (b > kLdsBytes)
    return fail(NGVOL_EUNSUPPORTED, "network too large for the LDS-resident backward (%zu > %zu bytes)", b, kLdsBytes);
  return NGVOL_OK;
}

int check_weights(const ngvol_weights* w) {
  NGV_REQUIRE(w && w->params, "weights or weights->params is NULL");
  NGV_REQUIRE(aligned16(w->params) && aligned16(w->table_f16), "weights must be 16-byte aligned");
  return NGVOL_OK;
}

}  // namespace

namespace ngvol {

// Error reporting for the entry points defined in other sources.
int api_fail(int code, const char* msg) { return fail(code, "%s", msg); }
int api_hip_check(hipError_t e, const char* what, hipStream_t st) { return hip_check(e, what, st); }

TrainWorkspace train_workspace(const ngvol_plan* plan, int64_t B) {
  TrainWorkspace ws;
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  const size_t esz = plan->layout.precision ? 2 : 4;
  ws.bwd_grid = bwd_grid(plan, B);
  ws.e_off = 0;
  ws.g_off = up((size_t)B * plan->kin * esz);
  ws.de_off = ws.g_off + up((size_t)B * 4);
  ws.partial_off = ws.de_off + up((size_t)B * plan->md.n_in * 4);
  ws.misc_off = ws.partial_off + up((size_t)ws.bwd_grid * plan->md.n_mlp * 4);
  ws.sc = scatter_plan(plan, B);
  ws.scatter_off = ws.misc_off + 256;
  ws.total = ws.scatter_off + ws.sc.bytes;
  return ws;
}

}  // namespace ngvol

extern "C" {

const char* ngvol_last_error(void) { return g_err.c_str(); }
const char* ngvol_version(void) { return "ngvol 0.1 (gfx950)"; }

int ngvol_set_debug(int32_t on) {
  g_debug.store(on ? 1 : 0, std::memory_order_relaxed);
  return NGVOL_OK;
}

int ngvol_plan_create(const ngvol_config* c, ngvol_plan** out) {
  NGV_REQUIRE(c && out, "config and out must be non-NULL");
  *out = nullptr;
  NGV_REQUIRE(c->n_levels >= 1 && c->n_levels <= NGVOL_MAX_LEVELS, "n_levels must be in [1,%d]", NGVOL_MAX_LEVELS);
  NGV_REQUIRE(c->n_features >= 1 && c->n_features <= 8, "n_features must be in [1,8]");
  NGV_REQUIRE(c->log2_hashmap_size >= 1 && c->log2_hashmap_size <= 28, "log2_hashmap_size must be in [1,28]");
  NGV_REQUIRE(c->resolutions || c->base_resolution >= 2, "base_resolution must be >= 2");
  NGV_REQUIRE(c->n_hidden_layers >= 1 && c->n_hidden_layers <= NGVOL_MAX_LAYERS - 1, "n_hidden_layers must be in [1,%d]",
              NGVOL_MAX_LAYERS - 1);
  NGV_REQUIRE(c->n_neurons >= 1, "n_neurons must be positive");
  NGV_REQUIRE(c->precision == NGVOL_FP32 || c->precision == NGVOL_BF16 || c->precision == NGVOL_FP16,
              "precision must be NGVOL_FP32, NGVOL_BF16 or NGVOL_FP16");
  NGV_REQUIRE(c->loss == NGVOL_LOSS_L2 || c->loss == NGVOL_LOSS_L1, "loss must be NGVOL_LOSS_L2 or NGVOL_LOSS_L1");
  NGV_REQUIRE(c->output_activation == NGVOL_ACT_NONE || c->output_activation == NGVOL_ACT_RELU,
              "output_activation must be NGVOL_ACT_NONE or NGVOL_ACT_RELU");
  if (c->n_features != 2 && c->n_features != 4 && c->n_features != 8)
    return fail(NGVOL_EUNSUPPORTED, "n_features %d unsupported (2, 4 or 8)", c->n_features);
  if (c->n_neurons != 32 && c->n_neurons != 64)
    return fail(NGVOL_EUNSUPPORTED, "n_neurons %d unsupported (32 or 64)", c->n_neurons);
  const int n_in = c->n_levels * c->n_features;
  if (n_in > 64) return fail(NGVOL_EUNSUPPORTED, "n_levels * n_features = %d exceeds 64", n_in);

  int32_t res[NGVOL_MAX_LEVELS];
  int rc = resolve_resolutions(c, res);
  if (rc) return rc;
  for (int l = 0; l < c->n_levels; ++l)
    NGV_REQUIRE(res[l] >= 2 && res[l] <= 65536, "resolution of level %d (%d) must be in [2,65536]", l, res[l]);

  ngvol_plan* p = new (std::nothrow) ngvol_plan;
  if (!p) return fail(NGVOL_ENOMEM, "out of host memory");
  memset(p, 0, sizeof *p);
  ngvol_layout& L = p->layout;
  ModelDesc& md = p->md;
  const int64_t T = (int64_t)1 << c->log2_hashmap_size;
  L.n_levels = md.L = c->n_levels;
  L.n_features = md.F = c->n_features;
  L.n_input = md.n_in = n_in;
  L.n_neurons = md.width = c->n_neurons;
  L.n_hidden_layers = md.n_hidden = c->n_hidden_layers;
  L.precision = c->precision;
  md.n_layers = md.n_hidden + 1;
  md.out_relu = c->output_activation == NGVOL_ACT_RELU;
  int64_t off = 0;
  for (int l = 0; l < md.L; ++l) {
    const int64_t N = res[l];
    const int64_t cube = N * N * N;
    const bool dense = cube <= T;
    const int64_t entries = dense ? cube : T;
    L.resolution[l] = (int32_t)N;
    L.dense[l] = dense;
    L.level_entries[l] = entries;
    L.level_offset[l] = off;
    md.lv[l].N = (int32_t)N;
    md.lv[l].dense = dense;
    md.lv[l].offset = (uint32_t)off;
    md.lv[l].mask = (uint32_t)(T - 1);
    off += entries;
  }
  L.level_offset[md.L] = off;
  if (off * md.F > ((int64_t)1 << 30) - 4) {  // table byte offsets stay 32-bit
    delete p;
    return fail(NGVOL_EUNSUPPORTED, "tables of %lld entries exceed 2^30 - 4 floats (4 GiB)", (long long)off);
  }
  md.n_table = L.n_table_params = off * md.F;
  int64_t pos = 0;
  for (int i = 0; i < md.n_layers; ++i) {
    const int in = i == 0 ? n_in : md.width;
    const int outd = i == md.n_layers - 1 ? 1 : md.width;
    md.w_off[i] = (int32_t)pos;
    L.layer_offset[i] = md.n_table + pos;
    pos += (int64_t)in * outd;
  }
  md.n_mlp = (int32_t)pos;
  L.n_mlp_params = pos;
  md.n_params = L.n_params = md.n_table + pos;
  p->kin = n_in <= 32 ? 32 : 64;
  p->loss = c->loss;

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  p->cus = cus;
  p->device = dev;
  if (enc_lds_bytes(p, 1) > kLdsBytes || fwd_lds_bytes(p) + 8192 > kLdsBytes) {
    const size_t b = enc_lds_bytes(p, 1);
    delete p;
    return fail(NGVOL_EUNSUPPORTED, "network too large for LDS-resident weights (%zu bytes)", b);
  }
  *out = p;
  return NGVOL_OK;
}

int ngvol_plan_destroy(ngvol_plan* plan) {
  delete plan;
  return NGVOL_OK;
}

int ngvol_get_layout(const ngvol_plan* plan, ngvol_layout* out) {
  if (int rc = check_plan(plan)) return rc;
  NGV_REQUIRE(out, "out is NULL");
  *out = plan->layout;
  return NGVOL_OK;
}

int ngvol_encode(const ngvol_plan* plan, const ngvol_weights* w, const float* xyz, int64_t n, float* feat,
                 hipStream_t st) {
  if (int rc = check_plan(plan)) return rc;
  if (int rc = check_weights(w)) return rc;
  NGV_REQUIRE(n >= 0, "n must be >= 0");
  if (n == 0) return NGVOL_OK;
  NGV_REQUIRE(xyz && feat && aligned4(xyz) && aligned4(feat), "xyz and feat must be non-NULL and 4-byte aligned");
  return hip_check(launch_encode(plan, tables_of(plan, w), xyz, n, feat, st), "encode launch", st);
}

int ngvol_encode_debug(const ngvol_plan* plan, const float* xyz, int64_t n, uint32_t* idx, float* w, hipStream_t st) {
  if (int rc = check_plan(plan)) return rc;
  NGV_REQUIRE(n >= 0, "n must be >= 0");
  if (n == 0) return NGVOL_OK;
  NGV_REQUIRE(xyz && aligned4(xyz) && aligned4(idx) && aligned4(w), "xyz must be non-NULL; buffers 4-byte aligned");
  NGV_REQUIRE(n * plan->md.L < ((int64_t)1 << 31) * 256, "n too large");
  return hip_check(launch_encode_debug(plan, xyz, n, idx, w, st), "encode_debug launch", st);
}

int ngvol_mlp_fwd(const ngvol_plan* plan, const float* params, const void* feat, int32_t dtype, int64_t n, float* out,
                  hipStream_t st) {
  if (int rc = check_plan(plan)) return rc;
  NGV_REQUIRE(n >= 0, "n must be >= 0");
  if (n == 0) return NGVOL_OK;
  NGV_REQUIRE(params && feat && out && aligned16(params) && aligned16(feat) && aligned4(out),
              "params and feat must be non-NULL and 16-byte aligned, out 4-byte aligned");
  NGV_REQUIRE(dtype == NGVOL_DT_F32 || dtype == NGVOL_DT_BF16 || dtype == NGVOL_DT_F16,
              "feat dtype must be NGVOL_DT_F32, NGVOL_DT_BF16 or NGVOL_DT_F16");
  return hip_check(launch_mlp_fwd(plan, params + plan->md.n_table, feat, dtype, n, out, st), "mlp_fwd launch", st);
}

// Query on grouped records: level-split passes for large sets, else the
// fused kernel.
static hipError_t launch_grouped(const ngvol_plan* plan, const BinPlan& bp, const ngvol_weights* w, void* ws,
                                 int64_t n, float* out, hipStream_t st) {
  char* base = reinterpret_cast<char*>(ws);
  const float4* rec = reinterpret_cast<const float4*>(base + bp.rec_off);
  const float* mlp = w->params + plan->md.n_table;
  if (bp.split && w->table_f16) {  // FP32 tables (4 MB per level) would not fit an L2 per level pair
    const BinRanges bins{reinterpret_cast<const uint32_t*>(base + bp.offsets_off),
                         reinterpret_cast<const uint32_t*>(base + bp.totals_off), bp.k};
    return launch_infer_split(plan, tables_of(plan, w), mlp, rec, n, out, base + bp.planes_off,
                              reinterpret_cast<uint32_t*>(base + bp.idx_off), bins, st);
  }
  return launch_infer(plan, tables_of(plan, w), mlp, nullptr, rec, n, out, st);
}

int ngvol_infer_workspace_bytes(const ngvol_plan* plan, int64_t n, size_t* bytes) {
  if (int rc = check_plan(plan)) return rc;
  NGV_REQUIRE(bytes && n >= 0 && n < ((int64_t)1 << 31), "bytes must be non-NULL and 0 <= n < 2^31");
  const BinPlan bp = bin_plan(plan, n);
  *bytes = bp.k ? bp.bytes : 0;
  return NGVOL_OK;
}

int ngvol_infer(const ngvol_plan* plan, const ngvol_weights* w, const float* xyz, int64_t n, float* out, void* ws,
                size_t ws_bytes, hipStream_t st) {
  if (int rc = check_plan(plan)) return rc;
  if (int rc = check_weights(w)) return rc;
  NGV_REQUIRE(n >= 0 && n < ((int64_t)1 << 31), "n must be in [0, 2^31)");
  if (n == 0) return NGVOL_OK;
  NGV_REQUIRE(xyz && out && aligned4(xyz) && aligned4(out), "xyz and out must be non-NULL and 4-byte aligned");
  NGV_REQUIRE(aligned16(ws), "workspace must be 16-byte aligned");
  const float* mlp = w->params + plan->md.n_table;
  const BinPlan bp = bin_plan(plan, n);
  if (ws && bp.k) {
    if (ws_bytes < bp.bytes) return fail(NGVOL_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, bp.bytes);
    hipError_t e = launch_bin(plan, bp, xyz, nullptr, n, ws, st);
    if (e != hipSuccess) return hip_check(e, "infer binning launch", st);
    return hip_check(launch_grouped(plan, bp, w, ws, n, out, st), "infer launch", st);
  }
  return hip_check(launch_infer(plan, tables_of(plan, w), mlp, xyz, nullptr, n, out, st), "infer launch", st);
}

int ngvol_sort_queries(const ngvol_plan* plan, const float* xyz, int64_t n, void* ws, size_t ws_bytes,
                       hipStream_t st) {
  if (int rc = check_plan(plan)) return rc;
  NGV_REQUIRE(n > 0 && n < ((int64_t)1 << 31), "n must be in [1, 2^31)");
  NGV_REQUIRE(xyz && ws && aligned4(xyz) && aligned16(ws), "xyz and workspace must be non-NULL and aligned");
  const BinPlan bp = bin_plan(plan, n);
  NGV_REQUIRE(bp.k, "%lld queries are too few to group (ngvol_infer_workspace_bytes is 0)", (long long)n);
  if (ws_bytes < bp.bytes) return fail(NGVOL_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, bp.bytes);
  return hip_check(launch_bin(plan, bp, xyz, nullptr, n, ws, st), "sort_queries launch", st);
}

int ngvol_infer_sorted(const ngvol_plan* plan, const ngvol_weights* w, void* ws, int64_t n, float* out,
                       hipStream_t st) {
  if (int rc = check_plan(plan)) return rc;
  if (int rc = check_weights(w)) return rc;
  NGV_REQUIRE(n > 0 && n < ((int64_t)1 << 31), "n must be in [1, 2^31)");
  NGV_REQUIRE(ws && out && aligned16(ws) && aligned4(out), "workspace and out must be non-NULL and aligned");
  const BinPlan bp = bin_plan(plan, n);
  NGV_REQUIRE(bp.k, "%lld queries are too few to group (ngvol_infer_workspace_bytes is 0)", (long long)n);
  return hip_check(launch_grouped(plan, bp, w, ws, n, out, st), "infer_sorted launch", st);
}

}  // extern "C"

namespace {
// MLP backward on caller features (MODE 1 of k_bwd), dW partial sums in
// `partial` ([grid][n_mlp]), then their fixed-order reduction into grad.
hipError_t launch_mlp_bwd_pass(const ngvol_plan* plan, const float* params, const float* feat, int64_t n,
                               const float* dout, float* dfeat, float* grad, float* partial, int grid, int32_t* flag,
                               hipStream_t st) {
  BatchArgs ba{};
  ba.B = n;
  hipError_t e = launch_bwd(plan, 1, params + plan->md.n_table, feat, dout, ba, grad, dfeat, partial, grid, flag, 1.0f,
                            st);
  if (e == hipSuccess) e = launch_reduce_partials(plan, partial, grid, grad, flag, st);
  return e;
}
}  // namespace

extern "C" {

int ngvol_mlp_bwd_workspace_bytes(const ngvol_plan* plan, int64_t n, size_t* bytes) {
  if (int rc = check_plan(plan)) return rc;
  NGV_REQUIRE(bytes && n >= 0, "bytes must be non-NULL and n >= 0");
  *bytes = ((size_t)bwd_grid(plan, n) * plan->md.n_mlp * 4 + 255) / 256 * 256 + 256;
  return NGVOL_OK;
}

int ngvol_mlp_bwd(const ngvol_plan* plan, const float* params, const float* feat, int64_t n, const float* dout,
                  float* dfeat, float* grad, void* ws, size_t ws_bytes, hipStream_t st) {
  if (int rc = check_plan(plan)) return rc;
  NGV_REQUIRE(n >= 0, "n must be >= 0");
  if (n == 0) return NGVOL_OK;
  NGV_REQUIRE(params && feat && dout && grad && ws, "params, feat, dout, grad and workspace must be non-NULL");
  NGV_REQUIRE(aligned16(params) && aligned4(feat) && aligned4(dout) && aligned4(grad) && aligned4(dfeat) &&
                  aligned16(ws),
              "params and workspace must be 16-byte aligned, other buffers 4-byte aligned");
  if (int rc = check_bwd_lds(plan)) return rc;
  size_t need = 0;
  ngvol_mlp_bwd_workspace_bytes(plan, n, &need);
  if (ws_bytes < need) return fail(NGVOL_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, need);
  const int grid = bwd_grid(plan, n);
  float* partial = reinterpret_cast<float*>(ws);
  int32_t* flag = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(ws) + need - 256);
  return hip_check(launch_mlp_bwd_pass(plan, params, feat, n, dout, dfeat, grad, partial, grid, flag, st),
                   "mlp_bwd launch", st);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free MLP backward.  Its partial sums live in `scratch`, a
// file-scope device array: every GPU the library runs on holds its own copy
// at its own address until the process ends.  Host code never uses the
// array's name as an address; the address is resolved once per device, with
// that device current, on the entry point's first call there.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = (size_t)8 << 20;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch array (NULL + error on failure).
int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(NGVOL_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(NGVOL_EUNSUPPORTED, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(NGVOL_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return NGVOL_OK;
}

}  // namespace

extern "C" {

size_t ngvol_mlp_bwd_noalloc_scratch_bytes(void) { return kScratchBytes; }

int ngvol_mlp_bwd_noalloc(const ngvol_plan* plan, const float* params, const float* feat, int64_t n, const float* dout,
                          float* dfeat, float* grad, hipStream_t st) {
  if (int rc = check_plan(plan)) return rc;
  NGV_REQUIRE(n >= 0, "n must be >= 0");
  if (n == 0) return NGVOL_OK;
  NGV_REQUIRE(params && feat && dout && grad, "params, feat, dout and grad must be non-NULL");
  NGV_REQUIRE(aligned16(params) && aligned4(feat) && aligned4(dout) && aligned4(grad) && aligned4(dfeat),
              "params must be 16-byte aligned, other buffers 4-byte aligned");
  if (int rc = check_bwd_lds(plan)) return rc;
  // one partial-sum row of n_mlp floats per workgroup, then the 256-byte flag block
  const size_t row = (size_t)plan->md.n_mlp * 4;
  if (row + 256 > kScratchBytes)
    return fail(NGVOL_EINVAL, "one partial-sum row of %zu bytes exceeds the %zu-byte scratch", row, kScratchBytes);
  const int64_t rows = (int64_t)((kScratchBytes - 256) / row);
  int grid = bwd_grid(plan, n);
  if (grid > rows) grid = (int)rows;  // fewer workgroups, each taking more tiles
  void* base = nullptr;
  if (int rc = scratch_address(&base)) return rc;
  float* partial = reinterpret_cast<float*>(base);
  int32_t* flag = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(base) + kScratchBytes - 256);
  return hip_check(launch_mlp_bwd_pass(plan, params, feat, n, dout, dfeat, grad, partial, grid, flag, st),
                   "mlp_bwd_noalloc launch", st);
}

int ngvol_encode_bwd(const ngvol_plan* plan, const float* xyz, int64_t n, const float* dfeat, float* grad,
                     hipStream_t st) {
  if (int rc = check_plan(plan)) return rc;
  NGV_REQUIRE(n >= 0, "n must be >= 0");
  if (n == 0) return NGVOL_OK;
  NGV_REQUIRE(xyz && dfeat && grad && aligned4(xyz) && aligned4(dfeat) && aligned4(grad),
              "xyz, dfeat and grad must be non-NULL and 4-byte aligned");
  return hip_check(launch_encode_bwd(plan, xyz, n, dfeat, grad, st), "encode_bwd launch", st);
}

static int resolve_mc(const ngvol_macrocells* mc, McGeom& g, bool need_range, bool need_mu) {
  NGV_REQUIRE(mc, "macrocells is NULL");
  NGV_REQUIRE(mc->cell >= 1, "macro-cell size must be >= 1");
  int64_t total = 1;
  for (int a = 0; a < 3; ++a) {
    NGV_REQUIRE(mc->dims[a] >= 1 && mc->dims[a] <= (1 << 20), "macro-cell volume dims must be in [1, 2^20]");
    g.dims[a] = mc->dims[a];
    g.m[a] = (mc->dims[a] + mc->cell - 1) / mc->cell;
    total *= g.m[a];
  }
  NGV_REQUIRE(total <= ((int64_t)1 << 24), "more than 2^24 macro-cells");
  g.cell = mc->cell;
  NGV_REQUIRE(!need_range || (mc->range && aligned4(mc->range)), "macro-cell range must be non-NULL, 4-byte aligned");
  NGV_REQUIRE(!need_mu || (mc->mu && aligned4(mc->mu)), "macro-cell mu must be non-NULL, 4-byte aligned");
  g.range = need_range ? mc->range : nullptr;
  g.mu = need_mu ? mc->mu : nullptr;
  return NGVOL_OK;
}

static int resolve_batch(const ngvol_plan* plan, const ngvol_batch* b, BatchArgs& ba) {
  (void)plan;
  NGV_REQUIRE(b, "batch is NULL");
  NGV_REQUIRE(b->batch_size > 0 && b->batch_size < ((int64_t)1 << 31), "batch_size must be in [1, 2^31)");
  ba.B = b->batch_size;
  ba.xyz = b->xyz;
  ba.target = b->target;
  ba.volume = b->volume;
  ba.dims[0] = b->dims[0];
  ba.dims[1] = b->dims[1];
  ba.dims[2] = b->dims[2];
  ba.vdtype = b->volume_dtype;
  ba.seed = b->seed;
  ba.step = b->step_index;
  ba.step_ptr = nullptr;
  if (b->xyz) {
    NGV_REQUIRE(b->target && aligned4(b->xyz) && aligned4(b->target),
                "explicit batch needs 4-byte aligned xyz and target");
  } else {
    NGV_REQUIRE(b->volume && aligned16(b->volume), "generated batch needs a 16-byte aligned volume");
    NGV_REQUIRE(b->dims[0] >= 2 && b->dims[1] >= 2 && b->dims[2] >= 2, "volume dims must be >= 2");
    NGV_REQUIRE(b->volume_dtype == NGVOL_DT_F32 || b->volume_dtype == NGVOL_DT_F16, "volume dtype must be F32 or F16");
    NGV_REQUIRE(b->seed < (1ull << 56), "seed must be < 2^56");
    NGV_REQUIRE(b->step_index >= -1, "step_index must be >= 0, or -1 for the state's step counter");
  }
  ba.mc = McGeom{};
  if (b->macrocells)
    if (int rc = resolve_mc(b->macrocells, ba.mc, true, false)) return rc;
  return NGVOL_OK;
}

int ngvol_mc_reset(const ngvol_macrocells* mc, hipStream_t st) {
  McGeom g{};
  if (int rc = resolve_mc(mc, g, true, false)) return rc;
  return hip_check(launch_mc_reset(g, st), "mc_reset launch", st);
}

int ngvol_mc_update(const ngvol_macrocells* mc, const float* xyz, const float* values, int64_t n, hipStream_t st) {
  McGeom g{};
  if (int rc = resolve_mc(mc, g, true, false)) return rc;
  NGV_REQUIRE(n >= 0 && n < ((int64_t)1 << 40), "n out of range");
  NGV_REQUIRE(n == 0 || (xyz && values && aligned4(xyz) && aligned4(values)),
              "xyz and values must be non-NULL and 4-byte aligned");
  return hip_check(launch_mc_update(g, xyz, values, n, st), "mc_update launch", st);
}

int ngvol_mc_opacity(const ngvol_macrocells* mc, const float* lut, hipStream_t st) {
  McGeom g{};
  if (int rc = resolve_mc(mc, g, true, true)) return rc;
  NGV_REQUIRE(lut && aligned4(lut), "lut must be non-NULL and 4-byte aligned");
  return hip_check(launch_mc_opacity(g, lut, st), "mc_opacity launch", st);
}

int ngvol_sample_batch(const ngvol_plan* plan, const ngvol_batch* b, float* xyz, float* y, hipStream_t st) {
  if (int rc = check_plan(plan)) return rc;
  BatchArgs ba{};
  if (int rc = resolve_batch(plan, b, ba)) return rc;
  NGV_REQUIRE(!b->xyz, "ngvol_sample_batch needs a generated batch (xyz == NULL)");
  NGV_REQUIRE(b->step_index >= 0, "ngvol_sample_batch needs an explicit step_index");
  NGV_REQUIRE(xyz && y && aligned4(xyz) && aligned4(y), "outputs must be non-NULL and 4-byte aligned");
  return hip_check(launch_sample_batch(ba, xyz, y, st), "sample_batch launch", st);
}

// Limits of the bucketed table-gradient scatter: record positions and bucket
// offsets are 32-bit (B * 8 * L < 2^32 records), and one workgroup counts
// every bucket of the tables in an LDS histogram (4 bytes per 2^bshift
// entries).
static int check_train_limits(const ngvol_plan* plan, int64_t B) {
  const ScatterPlan sp = scatter_plan(plan, B);
  if (sp.n_records >= ((int64_t)1 << 32))
    return fail(NGVOL_EINVAL, "batch of %lld samples gives %lld table-gradient records (B*8*L must be < 2^32)",
                (long long)B, (long long)sp.n_records);
  if ((size_t)sp.n_buckets * 4 > kLdsBytes)
    return fail(NGVOL_EUNSUPPORTED, "tables of %lld entries need a %zu-byte gradient bucket histogram (> %zu of LDS)",
                (long long)(plan->md.n_table / plan->md.F), (size_t)sp.n_buckets * 4, kLdsBytes);
  return NGVOL_OK;
}

int ngvol_train_workspace_bytes(const ngvol_plan* plan, int64_t B, size_t* bytes) {
  if (int rc = check_plan(plan)) return rc;
  NGV_REQUIRE(bytes && B > 0 && B < ((int64_t)1 << 31), "bytes must be non-NULL and 0 < B < 2^31");
  if (int rc = check_train_limits(plan, B)) return rc;
  *bytes = train_workspace(plan, B).total;
  return NGVOL_OK;
}

static int check_state(const ngvol_plan* plan, const ngvol_train_state* s) {
  (void)plan;
  NGV_REQUIRE(s, "state is NULL");
  NGV_REQUIRE(s->params && s->grad && s->adam_m && s->adam_v && s->step && s->workspace,
              "state needs params, grad, adam_m, adam_v, step and workspace");
  NGV_REQUIRE(aligned16(s->params) && aligned16(s->grad) && aligned16(s->adam_m) && aligned16(s->adam_v) &&
                  aligned16(s->table_f16) && aligned16(s->workspace) && ((uintptr_t)s->draws & 7u) == 0,
              "state buffers must be 16-byte aligned (draws 8-byte aligned)");
  return NGVOL_OK;
}

static int check_adam(const ngvol_adam* a, float loss_scale) {
  NGV_REQUIRE(a, "adam is NULL");
  NGV_REQUIRE(a->learning_rate >= 0 && a->beta1 >= 0 && a->beta1 < 1 && a->beta2 >= 0 && a->beta2 < 1 &&
                  a->epsilon >= 0,
              "Adam hyper-parameters out of range");
  NGV_REQUIRE(a->l2_reg >= 0 && std::isfinite(a->l2_reg), "l2_reg must be finite and >= 0");
  NGV_REQUIRE(a->decay_start >= 0 && a->decay_interval >= 0, "decay_start and decay_interval must be >= 0");
  NGV_REQUIRE(a->decay_interval == 0 || (a->decay_base > 0 && a->decay_base <= 1), "decay_base must be in (0,1]");
  NGV_REQUIRE(loss_scale > 0.0f && std::isfinite(loss_scale), "loss_scale must be positive and finite");
  return NGVOL_OK;
}

static AdamArgs adam_args(const ngvol_adam* a, float loss_scale) {
  AdamArgs aa{};
  aa.lr = a->learning_rate;
  aa.b1 = a->beta1;
  aa.b2 = a->beta2;
  aa.eps = a->epsilon;
  aa.l2_reg = a->l2_reg;
  aa.decay_start = a->decay_start;
  aa.decay_interval = a->decay_interval;
  aa.decay_base = a->decay_interval > 0 ? a->decay_base : 1.0;
  aa.inv_scale = 1.0f / loss_scale;
  return aa;
}

}  // extern "C"

namespace {

// A training step's host-side checks, done before anything is launched.
int train_prepare(const ngvol_plan* plan, const ngvol_train_state* s, const ngvol_batch* b, const ngvol_adam* a,
                  float loss_scale, BatchArgs& ba, TrainWorkspace& ws) {
  if (int rc = check_plan(plan)) return rc;
  if (int rc = check_state(plan, s)) return rc;
  if (int rc = check_adam(a, loss_scale)) return rc;
  if (int rc = check_bwd_lds(plan)) return rc;
  NGV_REQUIRE(b, "batch is NULL");
  ba = BatchArgs{};
  if (int rc = resolve_batch(plan, b, ba)) return rc;
  if (!b->xyz && b->step_index < 0) ba.step_ptr = s->draws ? s->draws : s->step;  // graph-replayable batch index
  if (int rc = check_train_limits(plan, ba.B)) return rc;
  ws = train_workspace(plan, ba.B);
  if (s->workspace_bytes < ws.total)
    return fail(NGVOL_ENOMEM, "workspace of %zu bytes < %zu needed", s->workspace_bytes, ws.total);
  return NGVOL_OK;
}

// The step's launches: sampling and forward, backward, scatter, Adam.
hipError_t train_enqueue(const ngvol_plan* plan, const ngvol_train_state* s, const BatchArgs& ba,
                         const TrainWorkspace& ws, const ngvol_adam* a, float loss_scale, hipStream_t st) {
  char* base = reinterpret_cast<char*>(s->workspace);
  void* e_buf = base + ws.e_off;
  float* g_buf = reinterpret_cast<float*>(base + ws.g_off);
  float* partial = reinterpret_cast<float*>(base + ws.partial_off);
  double* loss_acc = reinterpret_cast<double*>(base + ws.misc_off);
  int32_t* flag = reinterpret_cast<int32_t*>(base + ws.misc_off + 8);
  TablePtrs tp;
  tp.f32 = s->params;
  tp.f16 = reinterpret_cast<const __half*>(s->table_f16);
  const float* mlp = s->params + plan->md.n_table;
  // g = S * dL/dy: S * 2 (y - t) / B for L2, S * sign(y - t) / B for L1
  const float gscale = (float)((double)loss_scale * (plan->loss == NGVOL_LOSS_L1 ? 1.0 : 2.0) / (double)ba.B);
  hipError_t e = launch_step_begin(loss_acc, flag, st);
  if (e == hipSuccess) e = launch_train_fwd(plan, tp, mlp, ba, e_buf, g_buf, loss_acc, gscale, plan->loss, st);
  // 16-bit backward operands carry dz times a power of two that brings the
  // per-sample gradient scale S*2/B back to about one
  float bscale = 1.0f;
  if (plan->layout.precision != NGVOL_FP32) {
    int ex = (int)lrint(-log2((double)gscale));
    ex = ex < -24 ? -24 : (ex > 24 ? 24 : ex);
    bscale = ldexpf(1.0f, ex);
  }
  float* de = reinterpret_cast<float*>(base + ws.de_off);
  if (e == hipSuccess)
    e = launch_bwd(plan, 0, mlp, e_buf, g_buf, ba, s->grad, de, partial, ws.bwd_grid, flag, bscale, st);
  if (e == hipSuccess) e = launch_reduce_partials(plan, partial, ws.bwd_grid, s->grad, flag, st);
  if (e == hipSuccess) e = launch_scatter(plan, ws.sc, ba, de, s->grad, base + ws.scatter_off, flag, st);
  const AdamArgs aa = adam_args(a, loss_scale);
  if (e == hipSuccess)
    e = launch_adam(plan, s->params, reinterpret_cast<__half*>(s->table_f16), s->grad, s->adam_m, s->adam_v, s->step,
                    flag, aa, st);
  if (e == hipSuccess)
    e = launch_step_end(loss_acc, flag, s->step, s->draws, s->skipped, s->loss, 1.0 / (double)ba.B, st);
  return e;
}

}  // namespace

extern "C" {

int ngvol_train_step(const ngvol_plan* plan, const ngvol_train_state* s, const ngvol_batch* b, const ngvol_adam* a,
                     float loss_scale, hipStream_t st) {
  BatchArgs ba;
  TrainWorkspace ws;
  if (int rc = train_prepare(plan, s, b, a, loss_scale, ba, ws)) return rc;
  return hip_check(train_enqueue(plan, s, ba, ws, a, loss_scale, st), "train_step launch", st);
}

int ngvol_adam_step(const ngvol_plan* plan, const ngvol_train_state* s, const ngvol_adam* a, float loss_scale,
                    hipStream_t st) {
  if (int rc = check_plan(plan)) return rc;
  if (int rc = check_state(plan, s)) return rc;
  if (int rc = check_adam(a, loss_scale)) return rc;
  NGV_REQUIRE(s->workspace_bytes >= 256, "workspace must hold at least 256 bytes");
  char* base = reinterpret_cast<char*>(s->workspace);
  double* loss_acc = reinterpret_cast<double*>(base);
  int32_t* flag = reinterpret_cast<int32_t*>(base + 8);
  const AdamArgs aa = adam_args(a, loss_scale);
  hipError_t e = launch_step_begin(loss_acc, flag, st);
  if (e == hipSuccess)
    e = launch_adam(plan, s->params, reinterpret_cast<__half*>(s->table_f16), s->grad, s->adam_m, s->adam_v, s->step,
                    flag, aa, st);
  if (e == hipSuccess) e = launch_step_end(loss_acc, flag, s->step, s->draws, s->skipped, nullptr, 1.0, st);
  return hip_check(e, "adam launch", st);
}

int ngvol_make_f16_tables(const ngvol_plan* plan, const float* params, uint16_t* out, hipStream_t st) {
  if (int rc = check_plan(plan)) return rc;
  NGV_REQUIRE(params && out && aligned16(params) && aligned16(out), "params and out must be non-NULL, 16-byte aligned");
  return hip_check(launch_make_f16(params, reinterpret_cast<__half*>(out), plan->md.n_table, st), "make_f16 launch", st);
}

int ngvol_sq_error_grid(const ngvol_plan* plan, const ngvol_weights* w, const void* vol, const int32_t dims[3],
                        int32_t dtype, double* sq, hipStream_t st) {
  if (int rc = check_plan(plan)) return rc;
  if (int rc = check_weights(w)) return rc;
  NGV_REQUIRE(vol && sq && dims && aligned16(vol), "volume, dims and output must be non-NULL");
  NGV_REQUIRE(dims[0] >= 1 && dims[1] >= 1 && dims[2] >= 1, "dims must be positive");
  NGV_REQUIRE(dtype == NGVOL_DT_F32 || dtype == NGVOL_DT_F16, "volume dtype must be F32 or F16");
  return hip_check(launch_sq_error_grid(plan, tables_of(plan, w), w->params + plan->md.n_table, vol, dtype, dims, sq, st),
                   "sq_error_grid launch", st);
}

int ngvol_psnr(const ngvol_plan* plan, const ngvol_weights* w, const void* vol, const int32_t dims[3], int32_t dtype,
               double* mse, double* psnr, hipStream_t st) {
  if (int rc = check_plan(plan)) return rc;
  if (int rc = check_weights(w)) return rc;
  NGV_REQUIRE(vol && mse && dims && aligned16(vol) && ((uintptr_t)mse & 7u) == 0 && ((uintptr_t)psnr & 7u) == 0,
              "volume, dims and d_mse must be non-NULL; the volume 16-byte, the outputs 8-byte aligned");
  NGV_REQUIRE(dims[0] >= 1 && dims[1] >= 1 && dims[2] >= 1, "dims must be positive");
  NGV_REQUIRE(dtype == NGVOL_DT_F32 || dtype == NGVOL_DT_F16, "volume dtype must be F32 or F16");
  const double n = (double)dims[0] * (double)dims[1] * (double)dims[2];
  hipError_t e = launch_zero_f64(mse, st);
  if (e == hipSuccess)
    e = launch_sq_error_grid(plan, tables_of(plan, w), w->params + plan->md.n_table, vol, dtype, dims, mse, st);
  if (e == hipSuccess) e = launch_psnr_finish(mse, 1.0 / n, psnr, st);
  return hip_check(e, "psnr launch", st);
}

size_t ngvol_render_workspace_bytes(void) { return 256; }

int ngvol_render_ex(const ngvol_plan* plan, const ngvol_weights* w, const ngvol_camera* cam, const float* lut,
                    int32_t W, int32_t H, float dt, uint32_t seed, const ngvol_macrocells* mc,
                    const ngvol_render_opts* opts, float* rgba, uint32_t* n_geo, uint32_t* n_used,
                    ngvol_render_counters* counters, void* ws, size_t ws_bytes, hipStream_t st) {
  if (int rc = check_plan(plan)) return rc;
  if (int rc = check_weights(w)) return rc;
  NGV_REQUIRE(cam && lut && rgba && ws, "camera, lut, rgba and workspace must be non-NULL");
  NGV_REQUIRE(aligned16(lut) && aligned16(rgba) && aligned16(ws) && aligned4(n_geo) && aligned4(n_used) &&
                  aligned16(counters),
              "lut, rgba, counters and workspace must be 16-byte aligned, counts 4-byte aligned");
  NGV_REQUIRE(W >= 1 && H >= 1 && (int64_t)W * H < ((int64_t)1 << 31), "image size out of range");
  NGV_REQUIRE(dt >= 0x1p-20f && dt <= 1.0f, "dt must be in [2^-20, 1]");
  NGV_REQUIRE(ws_bytes >= ngvol_render_workspace_bytes(), "render workspace too small");
  RenderArgs ra{};
  ra.mode = NGVOL_RENDER_RM;
  if (opts) {
    const int mode = opts->mode;
    NGV_REQUIRE(mode == NGVOL_RENDER_RM || mode == NGVOL_RENDER_RM_SHADOW || mode == NGVOL_RENDER_PT,
                "unknown render mode %d", mode);
    ra.mode = mode;
    if (opts->adaptive) {
      if (mode != NGVOL_RENDER_RM) return fail(NGVOL_EUNSUPPORTED, "adaptive marching is available in mode RM only");
      NGV_REQUIRE(mc, "adaptive marching needs macro-cells");
      NGV_REQUIRE(opts->step_max >= 1.0f && opts->step_max <= 65536.0f, "step_max must be in [1, 65536]");
      NGV_REQUIRE(opts->step_exp >= 1 && opts->step_exp <= 8, "step_exp must be in [1, 8]");
      ra.adaptive = 1;
      ra.step_max = opts->step_max;
      ra.step_exp = opts->step_exp;
    }
    if (mode != NGVOL_RENDER_RM) {
      const float* l = opts->light_dir;
      NGV_REQUIRE(std::isfinite(l[0]) && std::isfinite(l[1]) && std::isfinite(l[2]) &&
                      (l[0] != 0.0f || l[1] != 0.0f || l[2] != 0.0f),
                  "light_dir must be finite and non-zero");
      const double n2 = (double)l[0] * l[0] + (double)l[1] * l[1] + (double)l[2] * l[2];
      NGV_REQUIRE(n2 > 1e-30 && n2 < 1e30, "light_dir length out of range");
      memcpy(ra.light, l, sizeof ra.light);
      NGV_REQUIRE(aligned4(opts->d_aux), "aux must be 4-byte aligned");
      NGV_REQUIRE(mode != NGVOL_RENDER_RM_SHADOW || opts->d_aux,
                  "RM_SHADOW needs d_aux (width x height uint32) for the shading points");
      ra.aux = opts->d_aux;
    }
    if (mode == NGVOL_RENDER_PT) {
      for (int c = 0; c < 3; ++c)
        NGV_REQUIRE(std::isfinite(opts->light_radiance[c]) && std::isfinite(opts->background[c]),
                    "light_radiance and background must be finite");
      NGV_REQUIRE(std::isfinite(opts->density) && opts->density > 0.0f, "density must be positive and finite");
      NGV_REQUIRE(opts->spp >= 1 && opts->spp <= 256, "spp must be in [1, 256]");
      NGV_REQUIRE(opts->rr_depth >= 0, "rr_depth must be >= 0");
      NGV_REQUIRE(opts->max_depth >= 1 && opts->max_depth <= 1024, "max_depth must be in [1, 1024]");
      memcpy(ra.radiance, opts->light_radiance, sizeof ra.radiance);
      memcpy(ra.background, opts->background, sizeof ra.background);
      ra.density = opts->density;
      ra.spp = opts->spp;
      ra.rr_depth = opts->rr_depth;
      ra.max_depth = opts->max_depth;
    }
  }
  if (mc)
    if (int rc = resolve_mc(mc, ra.mc, false, true)) return rc;
  memcpy(ra.cam, cam, sizeof ra.cam);
  ra.lut = lut;
  ra.width = W;
  ra.height = H;
  ra.dt = dt;
  ra.seed = seed;
  ra.rgba = rgba;
  ra.n_geo = n_geo;
  ra.n_used = n_used;
  ra.queue = reinterpret_cast<unsigned int*>(ws);
  ra.counters = reinterpret_cast<unsigned long long*>(counters);
  return hip_check(launch_render(plan, tables_of(plan, w), w->params + plan->md.n_table, ra, st), "render launch", st);
}

int ngvol_render(const ngvol_plan* plan, const ngvol_weights* w, const ngvol_camera* cam, const float* lut, int32_t W,
                 int32_t H, float dt, uint32_t seed, const ngvol_macrocells* mc, float* rgba, uint32_t* n_geo,
                 uint32_t* n_used, ngvol_render_counters* counters, void* ws, size_t ws_bytes, hipStream_t st) {
  return ngvol_render_ex(plan, w, cam, lut, W, H, dt, seed, mc, nullptr, rgba, n_geo, n_used, counters, ws, ws_bytes,
                         st);
}

// ---------------------------------------------------------------------------
// Batches of independent volumes.
// ---------------------------------------------------------------------------
}  // extern "C"

struct ngvol_multi {
  int k;
  ngvol_plan plan0;  // shape shared by the group (precision, widths, device)
  ngvol_plan plans[NGVOL_MULTI_MAX];  // copies, for per-model launches
  ngvol::ModelDesc* table;  // device
  uint32_t* next_item;      // device work counter of the persistent query, after the table
  int blocks_per_cu;  // 0: one single-model launch per model
  int chunk_tiles;
  // batched training: the models' steps run on these streams, forked from
  // and joined back to the caller's stream
  static constexpr int kStreams = 4;
  hipStream_t streams[kStreams] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kStreams] = {};
};

namespace {
void multi_release(ngvol_multi* g) {
  for (int j = 0; j < ngvol_multi::kStreams; ++j) {
    if (g->ev_join[j]) (void)hipEventDestroy(g->ev_join[j]);
    if (g->streams[j]) (void)hipStreamDestroy(g->streams[j]);
  }
  if (g->ev_fork) (void)hipEventDestroy(g->ev_fork);
  delete g;
}
}  // namespace

namespace {

int multi_args(const ngvol_multi* g, const ngvol_weights* w, const float* const* xyz, const int64_t* n,
               float* const* out, int chunk_tiles, MultiArgs& a, bool& f16) {
  NGV_REQUIRE(w && xyz && n && out, "w, xyz, n and out must be non-NULL host arrays");
  memset(&a, 0, sizeof a);
  a.k = g->k;
  a.chunk_tiles = chunk_tiles;
  a.item_prefix[0] = 0;
  f16 = w[0].table_f16 != nullptr;
  for (int i = 0; i < g->k; ++i) {
    if (int rc = check_weights(&w[i])) return rc;
    NGV_REQUIRE((w[i].table_f16 != nullptr) == f16, "either every model or none has FP16 tables");
    NGV_REQUIRE(n[i] >= 0 && n[i] < ((int64_t)1 << 31), "n[%d] out of range", i);
    NGV_REQUIRE(n[i] == 0 || (xyz[i] && out[i] && aligned4(xyz[i]) && aligned4(out[i])),
                "xyz[%d] and out[%d] must be non-NULL and 4-byte aligned", i, i);
    a.params[i] = w[i].params;
    a.f16[i] = reinterpret_cast<const __half*>(w[i].table_f16);
    a.xyz[i] = xyz[i];
    a.out[i] = out[i];
    a.n[i] = n[i];
    const int64_t tiles = (n[i] + 15) / 16;
    a.item_prefix[i + 1] = a.item_prefix[i] + (tiles + chunk_tiles - 1) / chunk_tiles;
  }
  return NGVOL_OK;
}


// The group's queries: one persistent launch over all models
// (blocks_per_cu > 0), or back-to-back single-model launches (0), which
// the autotuner picks when the models are large enough for one launch each
// to fill the GPU.
hipError_t multi_launch(const ngvol_multi* g, const ngvol_weights* w, const MultiArgs& a, bool f16, int bpc,
                        hipStream_t st) {
  if (bpc > 0) return launch_multi_infer(&g->plan0, g->table, a, f16, bpc, g->next_item, st);
  for (int i = 0; i < g->k; ++i) {
    if (a.n[i] == 0) continue;
    const ngvol_plan* p = &g->plans[i];
    hipError_t e = launch_infer(p, tables_of(p, &w[i]), w[i].params + p->md.n_table, a.xyz[i], nullptr, a.n[i],
                                a.out[i], st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
}  // namespace

extern "C" {

// the k descriptors, then (at a 256-byte boundary) the persistent query's
// work counter
static size_t multi_counter_offset(int32_t k) {
  return ((size_t)(k > 0 ? k : 0) * sizeof(ngvol::ModelDesc) + 255) / 256 * 256;
}

size_t ngvol_multi_table_bytes(int32_t k) { return multi_counter_offset(k) + 256; }

int ngvol_multi_create(const ngvol_plan* const* plans, int32_t k, void* d_table, size_t table_bytes, hipStream_t st,
                       ngvol_multi** out) {
  NGV_REQUIRE(out && plans, "plans and out must be non-NULL");
  *out = nullptr;
  NGV_REQUIRE(k >= 1 && k <= NGVOL_MULTI_MAX, "k must be in [1, %d]", NGVOL_MULTI_MAX);
  NGV_REQUIRE(d_table && aligned16(d_table) && table_bytes >= ngvol_multi_table_bytes(k),
              "d_table must hold ngvol_multi_table_bytes(k) bytes, 16-byte aligned");
  for (int i = 0; i < k; ++i) {
    if (int rc = check_plan(plans[i])) return rc;
    const ngvol_plan* p = plans[i];
    const ngvol_plan* q = plans[0];
    if (p->layout.precision != q->layout.precision || p->md.F != q->md.F || p->kin != q->kin ||
        p->md.width != q->md.width || p->md.n_hidden != q->md.n_hidden)
      return fail(NGVOL_EUNSUPPORTED, "model %d differs from model 0 in precision, features, input width or MLP", i);
  }
  if (plans[0]->md.F != 2) return fail(NGVOL_EUNSUPPORTED, "batched launches support n_features = 2");
  ngvol_multi* g = new (std::nothrow) ngvol_multi;
  if (!g) return fail(NGVOL_ENOMEM, "out of host memory");
  g->k = k;
  g->plan0 = *plans[0];
  for (int i = 0; i < k; ++i) g->plans[i] = *plans[i];
  g->table = reinterpret_cast<ngvol::ModelDesc*>(d_table);
  g->next_item = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(d_table) + multi_counter_offset(k));
  // untuned shape: few workgroups per compute unit, since the models' random
  // gathers evict each other's lines when many are in flight (16 models of
  // 2^20 queries: 6.2 ms at 1 per CU, 6.6 at 2, 7.1 at 4, 8.1 at 8)
  g->blocks_per_cu = 2;
  g->chunk_tiles = 16;
  ngvol::ModelDesc host[NGVOL_MULTI_MAX];
  for (int i = 0; i < k; ++i) host[i] = plans[i]->md;
  hipError_t e = hipMemcpyAsync(d_table, host, sizeof(ngvol::ModelDesc) * k, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming);
  for (int j = 0; j < ngvol_multi::kStreams && e == hipSuccess; ++j) {
    e = hipStreamCreateWithFlags(&g->streams[j], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g->ev_join[j], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    multi_release(g);
    return hip_check(e, "multi group set-up", st);
  }
  *out = g;
  return NGVOL_OK;
}

int ngvol_multi_destroy(ngvol_multi* g) {
  if (g) {
    for (int j = 0; j < ngvol_multi::kStreams; ++j)
      if (g->streams[j]) (void)hipStreamSynchronize(g->streams[j]);
    multi_release(g);
  }
  return NGVOL_OK;
}

int ngvol_multi_train_step(const ngvol_multi* g, const ngvol_train_state* states, const ngvol_batch* batches,
                           const ngvol_adam* adam, float loss_scale, hipStream_t st) {
  NGV_REQUIRE(g && states && batches, "group, states and batches must be non-NULL");
  BatchArgs ba[NGVOL_MULTI_MAX];
  TrainWorkspace ws[NGVOL_MULTI_MAX];
  for (int i = 0; i < g->k; ++i)
    if (int rc = train_prepare(&g->plans[i], &states[i], &batches[i], adam, loss_scale, ba[i], ws[i])) return rc;
  for (int i = 0; i < g->k; ++i)
    for (int j = 0; j < i; ++j)
      NGV_REQUIRE(states[i].workspace != states[j].workspace && states[i].params != states[j].params,
                  "models %d and %d share a training state", j, i);
  const int ns = g->k < ngvol_multi::kStreams ? g->k : ngvol_multi::kStreams;
  hipError_t e = hipEventRecord(g->ev_fork, st);
  for (int j = 0; j < ns && e == hipSuccess; ++j) e = hipStreamWaitEvent(g->streams[j], g->ev_fork, 0);
  for (int i = 0; i < g->k && e == hipSuccess; ++i)
    e = train_enqueue(&g->plans[i], &states[i], ba[i], ws[i], adam, loss_scale, g->streams[i % ns]);
  for (int j = 0; j < ns && e == hipSuccess; ++j) {
    e = hipEventRecord(g->ev_join[j], g->streams[j]);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, g->ev_join[j], 0);
  }
  return hip_check(e, "multi train_step launch", st);
}

int ngvol_multi_infer(const ngvol_multi* g, const ngvol_weights* w, const float* const* xyz, const int64_t* n,
                      float* const* out, hipStream_t st) {
  NGV_REQUIRE(g, "group is NULL");
  MultiArgs a;
  bool f16 = false;
  if (int rc = multi_args(g, w, xyz, n, out, g->chunk_tiles > 0 ? g->chunk_tiles : 16, a, f16)) return rc;
  if (a.item_prefix[g->k] == 0) return NGVOL_OK;
  return hip_check(multi_launch(g, w, a, f16, g->blocks_per_cu, st), "multi_infer launch", st);
}

int ngvol_multi_autotune(ngvol_multi* g, const ngvol_weights* w, const float* const* xyz, const int64_t* n,
                         float* const* out, hipStream_t st, int32_t* bpc_out, int32_t* chunk_out) {
  NGV_REQUIRE(g, "group is NULL");
  static const int kBpc[] = {1, 2, 4, 8};
  static const int kChunk[] = {16, 64, 256};  // multiples of 4 tiles: every wave of a workgroup gets a group
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float best = 1e30f;
  int best_b = g->blocks_per_cu, best_c = g->chunk_tiles;
  for (int bi = 0; bi < 4 && e == hipSuccess; ++bi)
    for (int ci = 0; ci < 3 && e == hipSuccess; ++ci) {
      MultiArgs a;
      bool f16 = false;
      if (int rc = multi_args(g, w, xyz, n, out, kChunk[ci], a, f16)) {
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        return rc;
      }
      if (a.item_prefix[g->k] == 0) break;
      e = multi_launch(g, w, a, f16, kBpc[bi], st);  // warm-up
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      for (int r = 0; r < 2 && e == hipSuccess; ++r) e = multi_launch(g, w, a, f16, kBpc[bi], st);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && ms < best) {
        best = ms;
        best_b = kBpc[bi];
        best_c = kChunk[ci];
      }
    }
  // one single-model launch per model
  if (e == hipSuccess) {
    MultiArgs a;
    bool f16 = false;
    if (int rc = multi_args(g, w, xyz, n, out, 16, a, f16)) {
      hipEventDestroy(e0);
      hipEventDestroy(e1);
      return rc;
    }
    e = multi_launch(g, w, a, f16, 0, st);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < 2 && e == hipSuccess; ++r) e = multi_launch(g, w, a, f16, 0, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && ms < best) {
      best = ms;
      best_b = 0;
      best_c = 0;
    }
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (e != hipSuccess) return hip_check(e, "multi autotune", st);
  g->blocks_per_cu = best_b;
  g->chunk_tiles = best_c;
  if (bpc_out) *bpc_out = best_b;
  if (chunk_out) *chunk_out = best_c;
  return NGVOL_OK;
}

}  // extern "C"
