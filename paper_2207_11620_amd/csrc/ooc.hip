// Out-of-core sampling (Section 4.1): training samples of a volume larger
// than memory, drawn from a buffer of R randomly chosen blocks of which S are
// replaced before every sampling step.
//
// The paper keeps the block buffer in host memory and samples on the CPU.
// Here the buffer is in HBM (R = 65,536 blocks of 64 KB is 4 GiB of the
// 288 GB) and a kernel draws the samples, so a step's only host work is
// reading the S new blocks.  The blocks come from a bricked copy of the
// volume (one 64 KB record per block, ghost layer included, written by
// ngvol_ooc_brick_file), so a block is one pread.  Host threads read a chunk
// of records into pinned staging; one copy moves the chunk to a device
// staging area and a placement kernel puts each record into its slot, both on
// the library's own copy stream, so the transfer overlaps whatever the caller
// runs after the refresh (the training step of the previous samples).  Two
// pinned halves alternate so that reading the next chunk overlaps the copy of
// the last one.
#include <errno.h>
#include <fcntl.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <algorithm>
#include <new>
#include <thread>
#include <vector>

#include "ngvol.h"
#include "device_common.hpp"

namespace ngvol {
int api_fail(int code, const char* msg);
int api_hip_check(hipError_t e, const char* what, hipStream_t st);
}  // namespace ngvol

using namespace ngvol;

namespace {

constexpr char kMagic[8] = {'N', 'G', 'V', 'B', 'R', 'I', 'C', 'K'};
constexpr int64_t kHeaderBytes = 4096;

struct BrickHeader {
  char magic[8];
  int32_t version, dims[3], dtype, block, grid[3];
  int64_t n_blocks, record_bytes;
};

size_t dtype_bytes(int dtype) { return dtype == NGVOL_DT_F16 ? 2 : 4; }

int64_t record_bytes_of(int block, int dtype) {
  const int64_t e = (int64_t)(block + 2) * (block + 2) * (block + 2) * (int64_t)dtype_bytes(dtype);
  return (e + 4095) / 4096 * 4096;
}

bool pread_all(int fd, void* dst, size_t n, int64_t off) {
  char* p = static_cast<char*>(dst);
  while (n > 0) {
    const ssize_t r = pread(fd, p, n, (off_t)off);
    if (r < 0 && errno == EINTR) continue;
    if (r <= 0) return false;
    p += r;
    n -= (size_t)r;
    off += r;
  }
  return true;
}

bool pwrite_all(int fd, const void* src, size_t n, int64_t off) {
  const char* p = static_cast<const char*>(src);
  while (n > 0) {
    const ssize_t r = pwrite(fd, p, n, (off_t)off);
    if (r < 0 && errno == EINTR) continue;
    if (r <= 0) return false;
    p += r;
    n -= (size_t)r;
    off += r;
  }
  return true;
}

// host counter generator, the same definition as the device's
uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
uint64_t host_rng(uint64_t seed, uint32_t stream, uint64_t index) {
  return mix64((seed ^ ((uint64_t)stream << 56)) + (index + 1ull) * 0x9E3779B97F4A7C15ull);
}
__host__ __device__ inline int64_t pick(uint64_t r, int64_t n) { return (int64_t)(((r >> 40) * (uint64_t)n) >> 24); }

// Device buffer: [R records][staging: S records + S (slot, block) pairs][slot table R int32].
struct OocLayout {
  size_t slots_off, stage_off, table_off, total;
};
OocLayout layout_of(int64_t R, int64_t S, int64_t rec) {
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  OocLayout L;
  L.slots_off = 0;
  L.stage_off = up((size_t)R * (size_t)rec);
  L.table_off = L.stage_off + up((size_t)S * (size_t)rec + 8 * (size_t)S);
  L.total = L.table_off + up(4 * (size_t)R);
  return L;
}

struct OocSampleArgs {
  const unsigned char* slots;
  const int32_t* table;
  int64_t R, rec_elems, step, B;
  uint64_t seed;
  int32_t dims[3], grid[3], block;
  float* xyz;
  float* y;
};

}  // namespace

struct ngvol_ooc {
  int fd = -1;
  BrickHeader h{};
  int64_t R = 0, S = 0, last_step = -1;
  uint64_t seed = 0;
  int n_threads = 1, device = 0;
  std::vector<int32_t> slot_block;
  unsigned char* pinned = nullptr;  // two halves of S records + S (slot, block) pairs
  size_t half_bytes = 0;
  int next_half = 0;  // the pinned half the next chunk uses
  hipStream_t copy = nullptr;
  hipEvent_t ev_ready = nullptr, ev_done = nullptr, ev_half[2] = {nullptr, nullptr};
  // the next step's records, read in the background after a refresh
  std::thread prefetch;
  int64_t pf_step = -1;
  int pf_half = 0;
  bool pf_ok = false;
  std::vector<int32_t> pf_slot, pf_blk;
};

namespace {

// One workgroup per record: copy it from the staging area into its slot.
__global__ void k_ooc_place(const unsigned char* __restrict__ stage, int64_t n, int64_t rec,
                            unsigned char* __restrict__ slots, int32_t* __restrict__ table) {
  const int64_t r = blockIdx.x;
  if (r >= n) return;
  const int32_t* list = reinterpret_cast<const int32_t*>(stage + n * rec);
  const int32_t slot = list[2 * r], blk = list[2 * r + 1];
  const uint4* src = reinterpret_cast<const uint4*>(stage + r * rec);
  uint4* dst = reinterpret_cast<uint4*>(slots + (int64_t)slot * rec);
  for (int64_t i = threadIdx.x; i < rec / 16; i += blockDim.x) dst[i] = src[i];
  if (threadIdx.x == 0) table[slot] = blk;
}

__device__ __forceinline__ uint64_t rng64(uint64_t seed, uint32_t stream, uint64_t index) {
  return sm64_mix((seed ^ ((uint64_t)stream << 56)) + (index + 1ull) * 0x9E3779B97F4A7C15ull);
}

// Sample i of the step: slot, voxel and jitter from the counter generator,
// then the in-core sampler's arithmetic on the block's record (the block and
// its ghost layer hold voxels origin-1 .. origin+b per axis).
template <typename T>
__global__ void __launch_bounds__(256) k_ooc_sample(OocSampleArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.B) return;
  const uint64_t base = (uint64_t)(a.step * a.B + i) * 8u;
  const int64_t slot = pick(rng64(a.seed, 10u, base), a.R);
  const int32_t blk = a.table[slot];
  const T* rec = reinterpret_cast<const T*>(a.slots) + slot * a.rec_elems;
  const int64_t g0 = a.grid[0], g1 = a.grid[1];
  const int64_t bc[3] = {blk % g0, (blk / g0) % g1, blk / (g0 * g1)};
  const int b = a.block, e = b + 2;
  float x[3];
  int l0[3];
  float t[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const int64_t origin = bc[ax] * b;
    const int64_t ext = a.dims[ax] - origin < b ? a.dims[ax] - origin : b;
    const int64_t v = origin + pick(rng64(a.seed, 10u, base + 1u + (uint64_t)ax), ext);
    const float u = (float)(uint32_t)(rng64(a.seed, 10u, base + 4u + (uint64_t)ax) >> 40) * 0x1p-24f;
    x[ax] = __fdiv_rn(__fadd_rn((float)v, u), (float)a.dims[ax]);
    // the in-core sampler's cell and weight
    const float uu = x[ax] * (float)a.dims[ax] - 0.5f;
    float fl = floorf(uu);
    fl = fminf(fmaxf(fl, 0.0f), (float)(a.dims[ax] - 2));
    t[ax] = fminf(fmaxf(uu - fl, 0.0f), 1.0f);
    l0[ax] = (int)fl - (int)origin + 1;  // in [0, b]: the record covers origin-1 .. origin+b
  }
  const int64_t sy = e, sz = (int64_t)e * e;
  const int64_t o = l0[0] + sy * l0[1] + sz * l0[2];
  float c[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) c[k] = load_vox<T>(rec, (size_t)(o + (k & 1) + sy * ((k >> 1) & 1) + sz * ((k >> 2) & 1)));
  const float c00 = __builtin_fmaf(t[0], c[1] - c[0], c[0]);
  const float c10 = __builtin_fmaf(t[0], c[3] - c[2], c[2]);
  const float c01 = __builtin_fmaf(t[0], c[5] - c[4], c[4]);
  const float c11 = __builtin_fmaf(t[0], c[7] - c[6], c[6]);
  const float c0 = __builtin_fmaf(t[1], c10 - c00, c00);
  const float c1 = __builtin_fmaf(t[1], c11 - c01, c01);
  a.y[i] = __builtin_fmaf(t[2], c1 - c0, c0);
  a.xyz[3 * i + 0] = x[0];
  a.xyz[3 * i + 1] = x[1];
  a.xyz[3 * i + 2] = x[2];
}

// The loads of a step: (slot, block), all R slots at step 0, S from step 1.
void loads_of(const ngvol_ooc* o, int64_t step, std::vector<int32_t>& slot, std::vector<int32_t>& blk) {
  const int64_t R = o->R, S = o->S, nb = o->h.n_blocks;
  const int64_t n = step == 0 ? R : S;
  slot.resize((size_t)n);
  blk.resize((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t j = step == 0 ? i : R + (step - 1) * S + i;
    slot[(size_t)i] = (int32_t)(step == 0 ? i : ((step - 1) * S + i) % R);
    blk[(size_t)i] = (int32_t)pick(host_rng(o->seed, 9u, (uint64_t)j), nb);
  }
}

// Reads n records into a pinned half on the reader threads and appends the
// (slot, block) list the placement kernel reads.
bool read_chunk(const ngvol_ooc* o, unsigned char* half, const int32_t* slot, const int32_t* blk, int64_t n) {
  const int64_t rec = o->h.record_bytes;
  const int nt = (int)std::min<int64_t>(o->n_threads, n);
  std::vector<int> ok((size_t)nt, 1);
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&, t]() {
      for (int64_t i = t; i < n; i += nt)
        if (!pread_all(o->fd, half + (size_t)i * (size_t)rec, (size_t)rec, kHeaderBytes + (int64_t)blk[i] * rec))
          ok[(size_t)t] = 0;
    });
  for (auto& th : pool) th.join();
  int32_t* list = reinterpret_cast<int32_t*>(half + (size_t)n * (size_t)rec);
  for (int64_t i = 0; i < n; ++i) {
    list[2 * i] = slot[i];
    list[2 * i + 1] = blk[i];
  }
  for (int v : ok)
    if (!v) return false;
  return true;
}

// One staged chunk to the device: copy, then the placement kernel, on the
// copy stream; the half is free again once ev_half[h] has passed.
hipError_t enqueue_chunk(ngvol_ooc* o, int h, int64_t n, unsigned char* base, const OocLayout& L) {
  const int64_t rec = o->h.record_bytes;
  unsigned char* stage = base + L.stage_off;
  hipError_t e = hipMemcpyAsync(stage, o->pinned + (size_t)h * o->half_bytes, (size_t)n * (size_t)rec + 8 * (size_t)n,
                                hipMemcpyHostToDevice, o->copy);
  if (e == hipSuccess) e = hipEventRecord(o->ev_half[h], o->copy);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_ooc_place, dim3((unsigned)n), dim3(256), 0, o->copy, stage, n, rec, base + L.slots_off,
                       reinterpret_cast<int32_t*>(base + L.table_off));
    e = hipGetLastError();
  }
  return e;
}

void join_prefetch(ngvol_ooc* o) {
  if (o->prefetch.joinable()) o->prefetch.join();
}

// Reads step `step`'s records into the next half in the background.
void start_prefetch(ngvol_ooc* o, int64_t step) {
  const int h = o->next_half;
  o->next_half ^= 1;
  o->pf_half = h;
  o->pf_step = step;
  o->pf_ok = false;
  o->prefetch = std::thread([o, h, step]() {
    (void)hipSetDevice(o->device);
    if (hipEventSynchronize(o->ev_half[h]) != hipSuccess) return;  // its last copy has finished
    loads_of(o, step, o->pf_slot, o->pf_blk);
    o->pf_ok = read_chunk(o, o->pinned + (size_t)h * o->half_bytes, o->pf_slot.data(), o->pf_blk.data(),
                          (int64_t)o->pf_slot.size());
  });
}

}  // namespace

extern "C" {

int ngvol_ooc_brick_file(const char* raw_path, const int32_t dims[3], int32_t dtype, int32_t block,
                         const char* bricked_path) {
  if (!raw_path || !bricked_path || !dims) return api_fail(NGVOL_EINVAL, "paths and dims must be non-NULL");
  if (dtype != NGVOL_DT_F32 && dtype != NGVOL_DT_F16) return api_fail(NGVOL_EINVAL, "dtype must be F32 or F16");
  if (block < 2 || block > 254) return api_fail(NGVOL_EINVAL, "block must be in [2, 254]");
  for (int a = 0; a < 3; ++a)
    if (dims[a] < 2 || dims[a] > (1 << 20)) return api_fail(NGVOL_EINVAL, "dims must be in [2, 2^20]");
  const size_t esz = dtype_bytes(dtype);
  const int64_t Dx = dims[0], Dy = dims[1], Dz = dims[2];
  const int64_t slice = Dx * Dy * (int64_t)esz;
  BrickHeader h{};
  memcpy(h.magic, kMagic, 8);
  h.version = 1;
  for (int a = 0; a < 3; ++a) {
    h.dims[a] = dims[a];
    h.grid[a] = (dims[a] + block - 1) / block;
  }
  h.dtype = dtype;
  h.block = block;
  h.n_blocks = (int64_t)h.grid[0] * h.grid[1] * h.grid[2];
  h.record_bytes = record_bytes_of(block, dtype);
  if (h.n_blocks >= ((int64_t)1 << 31)) return api_fail(NGVOL_EINVAL, "too many blocks");
  const int in = open(raw_path, O_RDONLY);
  if (in < 0) return api_fail(NGVOL_EINVAL, "cannot open the raw volume");
  if (lseek(in, 0, SEEK_END) < (off_t)(slice * Dz)) {
    close(in);
    return api_fail(NGVOL_EINVAL, "raw volume shorter than dims x dtype");
  }
  const int out = open(bricked_path, O_WRONLY | O_CREAT | O_TRUNC, 0644);
  if (out < 0) {
    close(in);
    return api_fail(NGVOL_EINVAL, "cannot create the bricked file");
  }
  int rc = NGVOL_OK;
  const int e = block + 2;
  std::vector<unsigned char> hdr(kHeaderBytes, 0);
  memcpy(hdr.data(), &h, sizeof h);
  std::vector<unsigned char> slab, recbuf;
  try {
    slab.resize((size_t)e * (size_t)slice);
    recbuf.resize((size_t)h.record_bytes);
  } catch (const std::bad_alloc&) {
    close(in);
    close(out);
    return api_fail(NGVOL_ENOMEM, "host memory for the brick slab");
  }
  if (!pwrite_all(out, hdr.data(), hdr.size(), 0)) rc = api_fail(NGVOL_EINVAL, "write failed");
  for (int64_t bz = 0; bz < h.grid[2] && rc == NGVOL_OK; ++bz) {
    // slices origin-1 .. origin+b of this row of blocks, clamped
    for (int k = 0; k < e && rc == NGVOL_OK; ++k) {
      const int64_t z = std::min(std::max(bz * block - 1 + k, (int64_t)0), Dz - 1);
      if (!pread_all(in, slab.data() + (size_t)k * slice, (size_t)slice, z * slice))
        rc = api_fail(NGVOL_EINVAL, "read of the raw volume failed");
    }
    for (int64_t by = 0; by < h.grid[1] && rc == NGVOL_OK; ++by)
      for (int64_t bx = 0; bx < h.grid[0] && rc == NGVOL_OK; ++bx) {
        std::fill(recbuf.begin(), recbuf.end(), 0);
        for (int k = 0; k < e; ++k)
          for (int j = 0; j < e; ++j) {
            const int64_t yv = std::min(std::max(by * block - 1 + j, (int64_t)0), Dy - 1);
            for (int i = 0; i < e; ++i) {
              const int64_t xv = std::min(std::max(bx * block - 1 + i, (int64_t)0), Dx - 1);
              memcpy(recbuf.data() + ((size_t)(k * e + j) * e + i) * esz,
                     slab.data() + (size_t)k * slice + (size_t)(yv * Dx + xv) * esz, esz);
            }
          }
        const int64_t id = bx + h.grid[0] * (by + h.grid[1] * bz);
        if (!pwrite_all(out, recbuf.data(), recbuf.size(), kHeaderBytes + id * h.record_bytes))
          rc = api_fail(NGVOL_EINVAL, "write of a record failed");
      }
  }
  close(in);
  if (close(out) != 0 && rc == NGVOL_OK) rc = api_fail(NGVOL_EINVAL, "closing the bricked file failed");
  return rc;
}

int ngvol_ooc_open(const char* bricked_path, int64_t R, int64_t S, uint64_t seed, int32_t n_threads,
                   ngvol_ooc** out) {
  if (!bricked_path || !out) return api_fail(NGVOL_EINVAL, "path and out must be non-NULL");
  *out = nullptr;
  if (R < 1 || R >= ((int64_t)1 << 31) || S < 1 || S > R) return api_fail(NGVOL_EINVAL, "need 1 <= S <= R < 2^31");
  if (n_threads < 1 || n_threads > 64) return api_fail(NGVOL_EINVAL, "n_threads must be in [1, 64]");
  ngvol_ooc* o = new (std::nothrow) ngvol_ooc;
  if (!o) return api_fail(NGVOL_ENOMEM, "host memory");
  auto bail = [&](int code, const char* msg) {
    ngvol_ooc_close(o);
    return api_fail(code, msg);
  };
  o->fd = open(bricked_path, O_RDONLY);
  if (o->fd < 0) return bail(NGVOL_EINVAL, "cannot open the bricked file");
  if (!pread_all(o->fd, &o->h, sizeof o->h, 0) || memcmp(o->h.magic, kMagic, 8) != 0 || o->h.version != 1)
    return bail(NGVOL_EINVAL, "not a bricked volume file");
  const BrickHeader& h = o->h;
  if ((h.dtype != NGVOL_DT_F32 && h.dtype != NGVOL_DT_F16) || h.block < 2 || h.block > 254 ||
      h.record_bytes != record_bytes_of(h.block, h.dtype) ||
      h.n_blocks != (int64_t)h.grid[0] * h.grid[1] * h.grid[2] || h.n_blocks < 1)
    return bail(NGVOL_EINVAL, "corrupt bricked file header");
  for (int a = 0; a < 3; ++a)
    if (h.dims[a] < 2 || h.grid[a] != (h.dims[a] + h.block - 1) / h.block)
      return bail(NGVOL_EINVAL, "corrupt bricked file header");
  if (lseek(o->fd, 0, SEEK_END) < (off_t)(kHeaderBytes + h.n_blocks * h.record_bytes))
    return bail(NGVOL_EINVAL, "bricked file is truncated");
  o->R = R;
  o->S = S;
  o->seed = seed;
  o->n_threads = n_threads;
  if (hipGetDevice(&o->device) != hipSuccess) return bail(NGVOL_EDEVICE, "no current device");
  try {
    o->slot_block.assign((size_t)R, -1);
  } catch (const std::bad_alloc&) {
    return bail(NGVOL_ENOMEM, "host memory for the slot table");
  }
  o->half_bytes = (size_t)S * (size_t)h.record_bytes + 8 * (size_t)S;
  if (hipHostMalloc((void**)&o->pinned, 2 * o->half_bytes, hipHostMallocDefault) != hipSuccess) {
    o->pinned = nullptr;
    return bail(NGVOL_ENOMEM, "pinned host staging");
  }
  if (hipStreamCreateWithFlags(&o->copy, hipStreamNonBlocking) != hipSuccess) {
    o->copy = nullptr;
    return bail(NGVOL_EDEVICE, "copy stream");
  }
  hipEvent_t* evs[4] = {&o->ev_ready, &o->ev_done, &o->ev_half[0], &o->ev_half[1]};
  for (hipEvent_t* e : evs)
    if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
      *e = nullptr;
      return bail(NGVOL_EDEVICE, "events");
    }
  for (hipEvent_t e : {o->ev_done, o->ev_half[0], o->ev_half[1]})
    if (hipEventRecord(e, o->copy) != hipSuccess) return bail(NGVOL_EDEVICE, "events");
  *out = o;
  return NGVOL_OK;
}

int ngvol_ooc_close(ngvol_ooc* o) {
  if (!o) return NGVOL_OK;
  join_prefetch(o);
  if (o->copy) (void)hipStreamSynchronize(o->copy);
  for (hipEvent_t e : {o->ev_ready, o->ev_done, o->ev_half[0], o->ev_half[1]})
    if (e) (void)hipEventDestroy(e);
  if (o->copy) (void)hipStreamDestroy(o->copy);
  if (o->pinned) (void)hipHostFree(o->pinned);
  if (o->fd >= 0) close(o->fd);
  delete o;
  return NGVOL_OK;
}

int ngvol_ooc_get_info(const ngvol_ooc* o, ngvol_ooc_info* out) {
  if (!o || !out) return api_fail(NGVOL_EINVAL, "ooc and out must be non-NULL");
  for (int a = 0; a < 3; ++a) {
    out->dims[a] = o->h.dims[a];
    out->grid[a] = o->h.grid[a];
  }
  out->dtype = o->h.dtype;
  out->block = o->h.block;
  out->n_blocks = o->h.n_blocks;
  out->record_bytes = o->h.record_bytes;
  out->R = o->R;
  out->S = o->S;
  return NGVOL_OK;
}

size_t ngvol_ooc_device_bytes(const ngvol_ooc* o) {
  if (!o) return 0;
  return layout_of(o->R, o->S, o->h.record_bytes).total;
}

int ngvol_ooc_refresh(ngvol_ooc* o, int64_t step, void* d_buf, hipStream_t stream) {
  if (!o || !d_buf) return api_fail(NGVOL_EINVAL, "ooc and buffer must be non-NULL");
  if (((uintptr_t)d_buf & 15u) != 0) return api_fail(NGVOL_EINVAL, "buffer must be 16-byte aligned");
  if (step < 0 || (step != 0 && step != o->last_step + 1))
    return api_fail(NGVOL_EINVAL, "refresh steps must follow each other (0, 1, 2, ...)");
  join_prefetch(o);
  const bool have = o->pf_step == step && step >= 1 && o->pf_ok;
  o->pf_step = -1;
  const OocLayout L = layout_of(o->R, o->S, o->h.record_bytes);
  unsigned char* base = static_cast<unsigned char*>(d_buf);
  // copies start after the caller's earlier work on `stream`
  if (int rc = api_hip_check(hipEventRecord(o->ev_ready, stream), "ooc refresh", stream)) return rc;
  if (int rc = api_hip_check(hipStreamWaitEvent(o->copy, o->ev_ready, 0), "ooc refresh", stream)) return rc;
  std::vector<int32_t> slot, blk;
  if (have) {
    // read in the background after the previous refresh
    slot.swap(o->pf_slot);
    blk.swap(o->pf_blk);
    if (int rc = api_hip_check(enqueue_chunk(o, o->pf_half, (int64_t)slot.size(), base, L), "ooc refresh copy",
                               o->copy))
      return rc;
  } else {
    loads_of(o, step, slot, blk);
    const int64_t n_loads = (int64_t)slot.size();
    for (int64_t c0 = 0; c0 < n_loads; c0 += o->S) {
      const int64_t n = std::min(o->S, n_loads - c0);
      const int hh = o->next_half;
      o->next_half ^= 1;
      if (int rc = api_hip_check(hipEventSynchronize(o->ev_half[hh]), "ooc staging", stream)) return rc;
      if (!read_chunk(o, o->pinned + (size_t)hh * o->half_bytes, slot.data() + c0, blk.data() + c0, n))
        return api_fail(NGVOL_EINVAL, "read of a block record failed");
      if (int rc = api_hip_check(enqueue_chunk(o, hh, n, base, L), "ooc refresh copy", o->copy)) return rc;
    }
  }
  if (int rc = api_hip_check(hipEventRecord(o->ev_done, o->copy), "ooc refresh", stream)) return rc;
  for (size_t i = 0; i < slot.size(); ++i) o->slot_block[(size_t)slot[i]] = blk[i];
  o->last_step = step;
  start_prefetch(o, step + 1);
  return NGVOL_OK;
}

int ngvol_ooc_sample(ngvol_ooc* o, int64_t step, int64_t B, const void* d_buf, float* d_xyz, float* d_target,
                     hipStream_t stream) {
  if (!o || !d_buf || !d_xyz || !d_target) return api_fail(NGVOL_EINVAL, "arguments must be non-NULL");
  if (B < 0 || B >= ((int64_t)1 << 31)) return api_fail(NGVOL_EINVAL, "B out of range");
  if (((uintptr_t)d_buf & 15u) != 0 || ((uintptr_t)d_xyz & 3u) != 0 || ((uintptr_t)d_target & 3u) != 0)
    return api_fail(NGVOL_EINVAL, "buffer 16-byte, outputs 4-byte aligned");
  if (o->last_step < 0) return api_fail(NGVOL_EINVAL, "sample before the first refresh");
  if (step < 0) return api_fail(NGVOL_EINVAL, "step must be >= 0");
  if (B == 0) return NGVOL_OK;
  if (int rc = api_hip_check(hipStreamWaitEvent(stream, o->ev_done, 0), "ooc sample", stream)) return rc;
  const OocLayout L = layout_of(o->R, o->S, o->h.record_bytes);
  const unsigned char* base = static_cast<const unsigned char*>(d_buf);
  OocSampleArgs a;
  a.slots = base + L.slots_off;
  a.table = reinterpret_cast<const int32_t*>(base + L.table_off);
  a.R = o->R;
  a.rec_elems = o->h.record_bytes / (int64_t)dtype_bytes(o->h.dtype);
  a.step = step;
  a.B = B;
  a.seed = o->seed;
  for (int ax = 0; ax < 3; ++ax) {
    a.dims[ax] = o->h.dims[ax];
    a.grid[ax] = o->h.grid[ax];
  }
  a.block = o->h.block;
  a.xyz = d_xyz;
  a.y = d_target;
  const unsigned grid = (unsigned)((B + 255) / 256);
  if (o->h.dtype == NGVOL_DT_F16)
    hipLaunchKernelGGL(k_ooc_sample<__half>, dim3(grid), dim3(256), 0, stream, a);
  else
    hipLaunchKernelGGL(k_ooc_sample<float>, dim3(grid), dim3(256), 0, stream, a);
  return api_hip_check(hipGetLastError(), "ooc sample launch", stream);
}

int ngvol_ooc_slots(const ngvol_ooc* o, int32_t* host_slot_block) {
  if (!o || !host_slot_block) return api_fail(NGVOL_EINVAL, "arguments must be non-NULL");
  memcpy(host_slot_block, o->slot_block.data(), sizeof(int32_t) * o->slot_block.size());
  return NGVOL_OK;
}

}  // extern "C"
