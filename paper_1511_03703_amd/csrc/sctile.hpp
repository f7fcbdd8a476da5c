// One-sample CRS product (Fig. "crs") over row tiles read by the whole
// workgroup, the default of the scalar baseline (lanes_per_row = 0).
//
// A workgroup owns ScShape<T>::rows consecutive rows.  Their entries are
// contiguous in the CRS arrays, so the 256 lanes read values and column
// indices in coalesced sweeps (entry base + t + 256 u for lane t), every
// load of a lane issued before any gather, multiply each value by its
// gathered x and leave the products in LDS; lane r < rows then adds its
// row's products in ascending entry order.  A row of 27 entries thus keeps
// every lane of the read busy, where a fixed group of lanes per row idles
// some of them and has only one or two entries in flight per lane.  A tile
// whose rows hold more than ScShape<T>::cap entries is summed by lane r
// straight from global memory, in the same order and with the same
// rounding.  Tile shapes from sweeps at 128^3 (27 entries a row): FP64 64
// rows (32: 13 % slower, 128: 31 % slower), FP32 32 rows (64: 8 % slower).
#pragma once

#include "common.hpp"

namespace ens {

constexpr int kScThreads = 256;

// rows of a tile and the entries its LDS holds
template <typename T>
struct ScShape;
template <>
struct ScShape<double> {
  static constexpr int rows = 64, cap = 2048;
};
template <>
struct ScShape<float> {
  static constexpr int rows = 32, cap = 1024;
};

template <typename T>
struct ScTileLds {
  static constexpr int R = ScShape<T>::rows, CAP = ScShape<T>::cap;
  static_assert(CAP % kScThreads == 0 && R <= kScThreads, "scalar tile shape");
  int32_t rp[R + 1];
  T prod[CAP];
};

// a * b rounded once: contraction is off here, so the product is never
// fused with the sum it feeds (the staged products pass through LDS and
// cannot be)
__device__ inline double sc_mul(double a, double b) {
#pragma clang fp contract(off)
  return a * b;
}
__device__ inline float sc_mul(float a, float b) {
#pragma clang fp contract(off)
  return a * b;
}

// Row r0 + threadIdx.x of the tile starting at row r0: returns its product
// sum and sets *has_row, or returns 0 with *has_row false for lanes past
// the tile's rows.  Every lane of the workgroup must call it.
template <typename T>
__device__ inline T sc_tile_row(ScTileLds<T>& t, int n, const int32_t* __restrict__ rp,
                                const int32_t* __restrict__ ci, const T* __restrict__ vals,
                                const T* __restrict__ x, int64_t r0, bool* has_row) {
  constexpr int R = ScTileLds<T>::R, CAP = ScTileLds<T>::CAP;
  const int rows = (int)((int64_t)n - r0 < R ? (int64_t)n - r0 : R);
  for (int i = threadIdx.x; i <= rows; i += kScThreads) t.rp[i] = rp[r0 + i];
  __syncthreads();
  const int64_t base = t.rp[0];
  const int64_t cnt = (int64_t)t.rp[rows] - base;
  const bool staged = cnt <= CAP;  // the same for every lane
  if (staged) {
    constexpr int U = CAP / kScThreads;
    T v[U];
    int32_t c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = threadIdx.x + kScThreads * u;
      if (k < cnt) {
        v[u] = __builtin_nontemporal_load(vals + base + k);
        c[u] = ci[base + k];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = threadIdx.x + kScThreads * u;
      if (k < cnt) t.prod[k] = sc_mul(v[u], x[c[u]]);
    }
  }
  __syncthreads();
  const int r = threadIdx.x;
  *has_row = r < rows;
  T s = 0;
  if (r < rows) {
    const int64_t k0 = t.rp[r], k1 = t.rp[r + 1];
    if (staged)
      for (int64_t k = k0; k < k1; ++k) s += t.prod[k - base];
    else
      for (int64_t k = k0; k < k1; ++k) s += sc_mul(vals[k], x[ci[k]]);
  }
  return s;
}

}  // namespace ens
