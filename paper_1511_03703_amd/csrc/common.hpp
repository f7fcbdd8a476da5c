// Internal helpers shared by the HIP sources of libens (never part of the ABI).
//
// Layout conventions of the ensemble (commuted) system, Eq. kron_sys_commuted:
// a matrix value is an s-long ensemble stored contiguously, values[k*s + e];
// a vector entry likewise, x[i*s + e].  One 16-byte load therefore carries
// V = 16/sizeof(T) consecutive samples of one entry, and the s samples of an
// entry are spread over L = s/V consecutive lanes of a 64-wide wavefront.
#pragma once

#include <vector>

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/ens.h"

namespace ens {

// ---------------------------------------------------------------- status ---

extern thread_local char g_last_error[512];
void set_error(const char* fmt, ...);

#define ENS_HIP_TRY(expr)                                                          \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) {                                                        \
      ::ens::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e),      \
                       __FILE__, __LINE__);                                        \
      return ENS_E_HIP;                                                            \
    }                                                                              \
  } while (0)

#define ENS_LAUNCH_CHECK()                                                         \
  do {                                                                             \
    hipError_t _e = hipGetLastError();                                             \
    if (_e != hipSuccess) {                                                        \
      ::ens::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(_e),  \
                       __FILE__, __LINE__);                                        \
      return ENS_E_HIP;                                                            \
    }                                                                              \
  } while (0)

#define ENS_ARG_CHECK(cond, msg)                                                   \
  do {                                                                             \
    if (!(cond)) {                                                                 \
      ::ens::set_error("invalid argument: %s", msg);                               \
      return ENS_E_ARG;                                                            \
    }                                                                              \
  } while (0)

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// ----------------------------------------------------------- vector types ---

template <typename T, int N>
struct vec_t {
  typedef T type __attribute__((ext_vector_type(N)));
};

template <typename T>
struct pack {
  static constexpr int V = 16 / (int)sizeof(T);  // samples per 16-byte load
  typedef typename vec_t<T, V>::type type;
};

// Lanes that hold the same samples of different entries must be combined
// when a per-sample sum is needed: with L lanes per entry these lanes are
// L, 2L, ... apart, so butterfly over offsets L..32.
template <int L>
__device__ inline double wave_sum_stride(double v) {
#pragma unroll
  for (int off = L; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Ensemble sizes compiled into the library (explicit instantiation).
inline bool supported_s(int s) { return s == 4 || s == 8 || s == 16 || s == 32; }

// Workgroup size of every kernel: 4 wavefronts.
constexpr int kBlock = 256;

// Per-device pinned scalars and events kept for the life of the process.
constexpr int kMaxSideStreams = 32;

struct DeviceCtx {
  int device = -1;
  int32_t* host_flag = nullptr;         // pinned [64], for the once-per-chunk polls
  hipStream_t work_stream = nullptr;    // non-default stream for graph capture
  hipEvent_t ev_in = nullptr, ev_out = nullptr;  // joins with the caller's stream
  // streams of the concurrent one-sample baseline (default priority),
  // created on first use, with one event each to join the caller's stream
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> side_ev;
};
DeviceCtx* device_ctx();
// Make sure the context holds at least `count` side streams.
bool ensure_side_streams(DeviceCtx* c, int count);

// Profiling of the hot kernels with HIP events recorded on the launch stream.
void prof_begin(int kernel_id, hipStream_t st);
void prof_end(int kernel_id, hipStream_t st, double bytes);
void prof_collect();  // resolve pending event pairs (call after a stream sync)
// While one lives, prof_begin / prof_end do nothing on this thread (for
// entry points that must not create events).
struct ProfPause {
  ProfPause();
  ~ProfPause();
};

}  // namespace ens
