// Ensemble and scalar CRS products as standalone entry points, and the
// layout change between the commuted and the sample-major ensemble layouts.
#include "rowops.hpp"
#include "sctile.hpp"

namespace ens {

// One workgroup of 256 lanes = 4 wavefronts, each on RPW consecutive rows;
// the tile's row offsets and column indices staged in LDS.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_ens_spmv(int n, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci, const T* __restrict__ vals,
                                                  const T* __restrict__ x, T* __restrict__ y) {
  using M = EnsMap<T, S>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane % M::L;
  const int64_t row = ((int64_t)blockIdx.x * 4 + wave) * M::RPW + lane / M::L;
  constexpr int R = 4 * M::RPW;
  __shared__ RowTileLds<R> tile;
  const bool staged = stage_row_tile(tile, n, rp, ci, (int64_t)blockIdx.x * R);
  if (row >= n) return;
  typename M::vt acc = tile_row_product<T, S>(tile, staged, (int)(row - (int64_t)blockIdx.x * R), ci, vals, x, sub);
  store_stream((typename M::vt*)y + row * M::L + sub, acc);
}

// Scalar CRS (Fig. "crs") with G lanes per row: lane g sums entries
// k0+g, k0+g+G, ...; the G partial sums are then combined by a butterfly.
template <typename T, int G>
__global__ __launch_bounds__(256) void k_scalar_spmv(int n, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, const T* __restrict__ vals,
                                                     const T* __restrict__ x, T* __restrict__ y) {
  const int g = threadIdx.x % G;
  const int64_t row = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
  const bool ok = row < n;
  T acc = 0;
  if (ok) {
    const int64_t k1 = rp[row + 1];
    for (int64_t k = rp[row] + g; k < k1; k += G) acc += __builtin_nontemporal_load(vals + k) * x[ci[k]];
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (ok && g == 0) y[row] = acc;
}

// Scalar CRS over row tiles read by the whole workgroup (lanes_per_row 0).
template <typename T>
__global__ __launch_bounds__(kScThreads) void k_scalar_spmv_tile(int n, const int32_t* __restrict__ rp,
                                                                const int32_t* __restrict__ ci,
                                                                const T* __restrict__ vals,
                                                                const T* __restrict__ x, T* __restrict__ y) {
  __shared__ ScTileLds<T> t;
  const int64_t r0 = (int64_t)blockIdx.x * ScShape<T>::rows;
  bool has = false;
  const T v = sc_tile_row<T>(t, n, rp, ci, vals, x, r0, &has);
  if (has) y[r0 + threadIdx.x] = v;
}

__global__ __launch_bounds__(256) void k_relayout(const double* __restrict__ src, double* __restrict__ dst,
                                                  int64_t rows, int s, int to_sm) {
  const int64_t total = rows * s;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    // t indexes the destination
    if (to_sm) {
      const int64_t e = t / rows, r = t % rows;
      dst[t] = src[r * s + e];
    } else {
      const int64_t r = t / s, e = t % s;
      dst[t] = src[e * rows + r];
    }
  }
}

template <typename T, int S>
static ens_status launch_ens_spmv(const ens_graph* g, const void* vals, const void* x, void* y,
                                  hipStream_t st) {
  using M = EnsMap<T, S>;
  const int64_t rows_per_block = 4 * M::RPW;
  const int64_t blocks = (g->n + rows_per_block - 1) / rows_per_block;
  if (blocks == 0) return ENS_OK;
  hipLaunchKernelGGL((k_ens_spmv<T, S>), dim3((unsigned)blocks), dim3(256), 0, st, g->n, g->row_ptr, g->col_idx,
                     (const T*)vals, (const T*)x, (T*)y);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

template <typename T>
static ens_status launch_scalar_spmv(const ens_graph* g, const void* vals, const void* x, void* y, int G,
                                     hipStream_t st) {
  if (g->n == 0) return ENS_OK;
  if (G == 0) {
    const int64_t tiles = (g->n + ScShape<T>::rows - 1) / ScShape<T>::rows;
    hipLaunchKernelGGL((k_scalar_spmv_tile<T>), dim3((unsigned)tiles), dim3(kScThreads), 0, st, g->n, g->row_ptr,
                       g->col_idx, (const T*)vals, (const T*)x, (T*)y);
    ENS_LAUNCH_CHECK();
    return ENS_OK;
  }
  const int64_t blocks = (g->n * G + 255) / 256;
  switch (G) {
#define ENS_SC_CASE(GG)                                                                                   \
  case GG:                                                                                                \
    hipLaunchKernelGGL((k_scalar_spmv<T, GG>), dim3((unsigned)blocks), dim3(256), 0, st, g->n, g->row_ptr, \
                       g->col_idx, (const T*)vals, (const T*)x, (T*)y);                                   \
    break;
    ENS_SC_CASE(4)
    ENS_SC_CASE(8)
    ENS_SC_CASE(16)
    ENS_SC_CASE(32)
    ENS_SC_CASE(64)
#undef ENS_SC_CASE
    default:
      set_error("lanes_per_row %d not supported", G);
      return ENS_E_ARG;
  }
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

ens_status check_graph(const ens_graph* g) {
  ENS_ARG_CHECK(g, "null graph");
  ENS_ARG_CHECK(g->n >= 0 && g->nnz >= 0 && g->nnz <= INT32_MAX, "graph sizes out of range");
  ENS_ARG_CHECK(g->n == 0 || g->row_ptr, "null row_ptr");
  ENS_ARG_CHECK(g->nnz == 0 || g->col_idx, "null col_idx");
  return ENS_OK;
}

}  // namespace ens

using namespace ens;

extern "C" {

ens_status ens_spmv(const ens_graph* graph, int32_t s, ens_dtype dtype, const void* values, const void* x,
                    void* y, hipStream_t stream) {
  ens_status st = check_graph(graph);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK((values || graph->nnz == 0) && ((x && y) || graph->n == 0), "null pointer");
  ENS_ARG_CHECK(aligned16(values) && aligned16(x) && aligned16(y), "ensemble buffers must be 16-byte aligned");
  ENS_ARG_CHECK(x != y || graph->n == 0, "y must not alias x");
  if (!supported_s(s)) {
    set_error("ensemble size %d not compiled in", s);
    return ENS_E_UNSUPPORTED;
  }
  const double w = dtype == ENS_F64 ? 8.0 : 4.0;
  const int kid = dtype == ENS_F64 ? ENS_K_SPMV_F64 : ENS_K_SPMV_F32;
  const double bytes = (double)graph->nnz * (s * w + 4.0) + 4.0 * (graph->n + 1) + 2.0 * graph->n * s * w;
  prof_begin(kid, stream);
  if (dtype == ENS_F64) {
    switch (s) {
      case 4: st = launch_ens_spmv<double, 4>(graph, values, x, y, stream); break;
      case 8: st = launch_ens_spmv<double, 8>(graph, values, x, y, stream); break;
      case 16: st = launch_ens_spmv<double, 16>(graph, values, x, y, stream); break;
      case 32: st = launch_ens_spmv<double, 32>(graph, values, x, y, stream); break;
    }
  } else if (dtype == ENS_F32) {
    switch (s) {
      case 4: st = launch_ens_spmv<float, 4>(graph, values, x, y, stream); break;
      case 8: st = launch_ens_spmv<float, 8>(graph, values, x, y, stream); break;
      case 16: st = launch_ens_spmv<float, 16>(graph, values, x, y, stream); break;
      case 32: st = launch_ens_spmv<float, 32>(graph, values, x, y, stream); break;
    }
  } else {
    set_error("unknown dtype %d", (int)dtype);
    return ENS_E_UNSUPPORTED;
  }
  prof_end(kid, stream, bytes);
  return st;
}

ens_status ens_scalar_spmv(const ens_graph* graph, ens_dtype dtype, const void* values, const void* x, void* y,
                           int32_t lanes_per_row, hipStream_t stream) {
  ens_status st = check_graph(graph);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK((values || graph->nnz == 0) && ((x && y && x != y) || graph->n == 0), "null or aliased pointer");
  ENS_ARG_CHECK(lanes_per_row >= 0, "lanes_per_row must be 0 (row tiles) or 4, 8, 16, 32, 64");
  const int G = lanes_per_row;
  const double w = dtype == ENS_F64 ? 8.0 : 4.0;
  const double bytes = (double)graph->nnz * (w + 4.0) + 4.0 * (graph->n + 1) + 2.0 * graph->n * w;
  prof_begin(ENS_K_SCALAR_SPMV, stream);
  if (dtype == ENS_F64) st = launch_scalar_spmv<double>(graph, values, x, y, G, stream);
  else if (dtype == ENS_F32) st = launch_scalar_spmv<float>(graph, values, x, y, G, stream);
  else {
    set_error("unknown dtype %d", (int)dtype);
    return ENS_E_UNSUPPORTED;
  }
  prof_end(ENS_K_SCALAR_SPMV, stream, bytes);
  return st;
}

ens_status ens_relayout(const double* src, double* dst, int64_t rows, int32_t s, int32_t to_sample_major,
                        hipStream_t stream) {
  ENS_ARG_CHECK(src && dst && src != dst && rows >= 0 && s >= 1, "bad relayout arguments");
  int64_t total = rows * s;
  if (total == 0) return ENS_OK;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_relayout, dim3((unsigned)blocks), dim3(256), 0, stream, src, dst, rows, s, to_sample_major);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

}  // extern "C"
