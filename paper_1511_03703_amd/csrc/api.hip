// Library-wide glue of libens: error text, per-device context, kernel timing
// with HIP events, and the copy / triad kernels used to calibrate bandwidth.
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace ens {

thread_local char g_last_error[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
}

// ------------------------------------------------------------ device ctx ---

static std::mutex g_ctx_mu;
static std::vector<DeviceCtx*> g_ctx;

DeviceCtx* device_ctx() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  if ((int)g_ctx.size() <= dev) g_ctx.resize(dev + 1, nullptr);
  if (!g_ctx[dev]) {
    DeviceCtx* c = new DeviceCtx();
    c->device = dev;
    if (hipHostMalloc((void**)&c->host_flag, 64 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
        hipStreamCreateWithFlags(&c->work_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess) {
      delete c;
      return nullptr;
    }
    g_ctx[dev] = c;
  }
  return g_ctx[dev];
}

bool ensure_side_streams(DeviceCtx* c, int count) {
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  while ((int)c->side.size() < count) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return false;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipStreamDestroy(s);
      return false;
    }
    c->side.push_back(s);
    c->side_ev.push_back(e);
  }
  return true;
}

// Release every device's context (see ens_shutdown).  Returns the first
// HIP error met, after releasing what it can.
static hipError_t release_contexts() {
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  hipError_t first = hipSuccess;
  auto keep = [&](hipError_t e) {
    if (first == hipSuccess && e != hipSuccess) first = e;
  };
  int cur = 0;
  const bool have_cur = hipGetDevice(&cur) == hipSuccess;
  for (DeviceCtx*& c : g_ctx) {
    if (!c) continue;
    keep(hipSetDevice(c->device));
    keep(hipStreamSynchronize(c->work_stream));
    for (hipStream_t st : c->side) keep(hipStreamSynchronize(st));
    for (hipEvent_t e : c->side_ev) keep(hipEventDestroy(e));
    for (hipStream_t st : c->side) keep(hipStreamDestroy(st));
    keep(hipEventDestroy(c->ev_in));
    keep(hipEventDestroy(c->ev_out));
    keep(hipStreamDestroy(c->work_stream));
    keep(hipHostFree(c->host_flag));
    delete c;
    c = nullptr;
  }
  g_ctx.clear();
  if (have_cur) keep(hipSetDevice(cur));
  return first;
}

// ------------------------------------------------------------- profiling ---

struct PendingPair {
  hipEvent_t a, b;
  int kernel;
  double bytes;
};

static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<hipEvent_t> g_free_events;
static std::vector<PendingPair> g_pending;
static hipEvent_t g_open[ENS_K_COUNT];
static bool g_open_valid[ENS_K_COUNT];
static std::vector<float> g_ms[ENS_K_COUNT];    // one duration per launch
static std::vector<double> g_by[ENS_K_COUNT];   // algorithmic bytes per launch

static hipEvent_t take_event() {
  if (!g_free_events.empty()) {
    hipEvent_t e = g_free_events.back();
    g_free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Profiling paused on this thread (ProfPause): no event is taken or created.
static thread_local int g_prof_paused = 0;
ProfPause::ProfPause() { ++g_prof_paused; }
ProfPause::~ProfPause() { --g_prof_paused; }

void prof_begin(int k, hipStream_t st) {
  if (!g_prof_on || g_prof_paused || k < 0 || k >= ENS_K_COUNT) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEvent_t e = take_event();
  if (!e) return;
  (void)hipEventRecord(e, st);
  g_open[k] = e;
  g_open_valid[k] = true;
}

void prof_end(int k, hipStream_t st, double bytes) {
  if (!g_prof_on || g_prof_paused || k < 0 || k >= ENS_K_COUNT) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_open_valid[k]) return;
  hipEvent_t e = take_event();
  if (!e) return;
  (void)hipEventRecord(e, st);
  g_pending.push_back({g_open[k], e, k, bytes});
  g_open_valid[k] = false;
}

void prof_collect() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  std::vector<PendingPair> keep;
  for (auto& p : g_pending) {
    if (hipEventQuery(p.b) != hipSuccess) {
      keep.push_back(p);
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      g_ms[p.kernel].push_back(ms);
      g_by[p.kernel].push_back(p.bytes);
    }
    g_free_events.push_back(p.a);
    g_free_events.push_back(p.b);
  }
  g_pending.swap(keep);
}

// --------------------------------------------------------- stream kernels ---

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Launch shapes of the stream kernels, measured on the box over 4 GiB: the
// streams that write run fastest with one 16-byte chunk (or one FP64
// element) per lane and a workgroup per 256 of them (copy 6.4 TB/s, triad
// 5.4, pure write 6.8), against 4.6, 4.7 and 5.1 TB/s for the same loops
// over a grid capped at 8192 workgroups; the pure read fastest with
// kReadU chunks in flight per lane over contiguous 16 KB per workgroup
// (7.0 TB/s, against 6.8 for 16 per lane over the capped grid and 5.4 for
// one per lane).  Grids above kMaxStreamBlocks fall back to striding.
constexpr int64_t kMaxStreamBlocks = (int64_t)1 << 23;  // 2^31 lanes
constexpr int kReadU = 4;
static_assert(ENS_STREAM_READ_CHUNK_BYTES == 16 * 256 * kReadU, "read chunk of one workgroup");

static unsigned stream_blocks(int64_t items) {
  int64_t b = (items + 255) / 256;
  if (b > kMaxStreamBlocks) b = kMaxStreamBlocks;
  return (unsigned)(b < 1 ? 1 : b);
}

__global__ __launch_bounds__(256) void k_copy16(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                 int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    dst[i] = __builtin_nontemporal_load(src + i);
}

// Pure read stream: every 16-byte chunk read once (non-temporal, as the
// products read their values); workgroup b reads the kReadU * 256 chunks
// from b * kReadU * 256 on (lane t: t, t + 256, ...) and folds them by XOR
// into out[b].
__global__ __launch_bounds__(256) void k_read16(const u32x4* __restrict__ src, int64_t n16,
                                                uint32_t* __restrict__ out) {
  __shared__ uint32_t red[256];
  const u32x4 zero = {0u, 0u, 0u, 0u};
  const int64_t base = (int64_t)blockIdx.x * 256 * kReadU + threadIdx.x;
  u32x4 v[kReadU];
#pragma unroll
  for (int u = 0; u < kReadU; ++u) {
    const int64_t i = base + (int64_t)u * 256;
    v[u] = i < n16 ? __builtin_nontemporal_load(src + i) : zero;
  }
  u32x4 a = zero;
#pragma unroll
  for (int u = 0; u < kReadU; ++u) a ^= v[u];
  red[threadIdx.x] = a[0] ^ a[1] ^ a[2] ^ a[3];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] ^= red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Pure write stream: every 16-byte chunk written once with an ordinary
// store (as the assemblies write their values).
__global__ __launch_bounds__(256) void k_write16(u32x4* __restrict__ dst, int64_t n16, uint32_t value) {
  const u32x4 v = {value, value ^ 1u, value ^ 2u, value ^ 3u};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = v;
}

__global__ __launch_bounds__(256) void k_triad(double* __restrict__ a, const double* __restrict__ b,
                                                const double* __restrict__ c, double q, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = b[i] + q * c[i];
}

}  // namespace ens

using namespace ens;

extern "C" {

const char* ens_last_error(void) { return g_last_error; }

const char* ens_status_string(ens_status st) {
  switch (st) {
    case ENS_OK: return "ok";
    case ENS_W_NOT_CONVERGED: return "some sample did not converge";
    case ENS_E_ARG: return "invalid argument";
    case ENS_E_UNSUPPORTED: return "unsupported ensemble size or dtype";
    case ENS_E_HIP: return "HIP runtime error";
    case ENS_E_NOMEM: return "workspace too small";
    case ENS_E_RANGE: return "size out of range";
    default: return "unknown status";
  }
}

int32_t ens_abi_version(void) { return 1; }

ens_status ens_shutdown(void) {
  // the profiling events: wait for the pending pairs, keep their
  // durations, then destroy every event (the durations stay queryable)
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& p : g_pending) (void)hipEventSynchronize(p.b);
  }
  prof_collect();
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = false;
    for (hipEvent_t e : g_free_events) (void)hipEventDestroy(e);
    g_free_events.clear();
    for (int k = 0; k < ENS_K_COUNT; ++k)
      if (g_open_valid[k]) {
        (void)hipEventDestroy(g_open[k]);
        g_open_valid[k] = false;
      }
  }
  const hipError_t e = release_contexts();
  if (e != hipSuccess) {
    set_error("ens_shutdown: %s", hipGetErrorString(e));
    return ENS_E_HIP;
  }
  return ENS_OK;
}

ens_status ens_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t stream) {
  ENS_ARG_CHECK(src && dst, "null pointer");
  ENS_ARG_CHECK(bytes % 16 == 0, "bytes must be a multiple of 16");
  ENS_ARG_CHECK(aligned16(src) && aligned16(dst), "buffers must be 16-byte aligned");
  if (bytes == 0) return ENS_OK;
  const int64_t n16 = (int64_t)(bytes / 16);
  hipLaunchKernelGGL(k_copy16, dim3(stream_blocks(n16)), dim3(256), 0, stream, (const u32x4*)src, (u32x4*)dst,
                     n16);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

ens_status ens_stream_read(const void* src, size_t bytes, uint32_t* out, hipStream_t stream) {
  ENS_ARG_CHECK(src && out, "null pointer");
  ENS_ARG_CHECK(bytes % 16 == 0, "bytes must be a multiple of 16");
  ENS_ARG_CHECK(aligned16(src), "src must be 16-byte aligned");
  if (bytes == 0) return ENS_OK;
  const int64_t n16 = (int64_t)(bytes / 16);
  const int64_t blocks = (n16 + 256 * kReadU - 1) / (256 * kReadU);
  if (blocks > kMaxStreamBlocks) {
    set_error("stream read of %zu bytes exceeds %lld workgroups", bytes, (long long)kMaxStreamBlocks);
    return ENS_E_RANGE;
  }
  hipLaunchKernelGGL(k_read16, dim3((unsigned)blocks), dim3(256), 0, stream, (const u32x4*)src, n16, out);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

ens_status ens_stream_write(void* dst, size_t bytes, uint32_t value, hipStream_t stream) {
  ENS_ARG_CHECK(dst, "null pointer");
  ENS_ARG_CHECK(bytes % 16 == 0, "bytes must be a multiple of 16");
  ENS_ARG_CHECK(aligned16(dst), "dst must be 16-byte aligned");
  if (bytes == 0) return ENS_OK;
  const int64_t n16 = (int64_t)(bytes / 16);
  hipLaunchKernelGGL(k_write16, dim3(stream_blocks(n16)), dim3(256), 0, stream, (u32x4*)dst, n16, value);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

ens_status ens_stream_triad(double* a, const double* b, const double* c, double q, int64_t n,
                            hipStream_t stream) {
  ENS_ARG_CHECK(a && b && c && n >= 0, "bad triad arguments");
  if (n == 0) return ENS_OK;
  hipLaunchKernelGGL(k_triad, dim3(stream_blocks(n)), dim3(256), 0, stream, a, b, c, q, n);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

// Events are created here, ahead of the timed work, so that no event
// creation falls inside a measured region (each costs host time).
constexpr size_t kProfEventPool = 1024;

ens_status ens_prof_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  while (g_prof_on && g_free_events.size() + 2 * g_pending.size() < kProfEventPool) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) break;
    g_free_events.push_back(e);
  }
  return ENS_OK;
}

ens_status ens_prof_reset(void) {
  prof_collect();
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (int k = 0; k < ENS_K_COUNT; ++k) {
    g_ms[k].clear();
    g_by[k].clear();
  }
  return ENS_OK;
}

ens_status ens_prof_query(int32_t kernel_id, double* total_ms, int64_t* launches, double* bytes) {
  ENS_ARG_CHECK(kernel_id >= 0 && kernel_id < ENS_K_COUNT, "kernel id");
  prof_collect();
  std::lock_guard<std::mutex> lk(g_prof_mu);
  const std::vector<float>& d = g_ms[kernel_id];
  double tot = 0.0, by = 0.0;
  int64_t cnt = 0;
  if (!d.empty()) {
    const float longest = *std::max_element(d.begin(), d.end());
    for (size_t i = 0; i < d.size(); ++i)
      if (d[i] >= 0.05f * longest) {  // launches that found no work return at once
        tot += d[i];
        by += g_by[kernel_id][i];
        ++cnt;
      }
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = cnt;
  if (bytes) *bytes = by;
  return ENS_OK;
}

}  // extern "C"
