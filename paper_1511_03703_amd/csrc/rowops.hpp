// Device building blocks of the ensemble sparse products (Sec. 2).
//
// Fig. "ensemble_crs" puts the sample loop innermost: for each stored entry
// the column index is read once and the s-long ensembles of the value and of
// x[col] are contiguous.  On a 64-wide wavefront we map that inner loop onto
// lanes: one 16-byte load holds V = 16/sizeof(T) samples, L = s/V lanes
// cover one entry's ensemble, and a wavefront works on 64/L rows at once.
// Every lane walks its row's entries in ascending order, so each sample's
// sum is formed in the order of the listing (with fused multiply-adds).
//   s=32 FP32: L=8, 8 rows/wave     s=32 FP64: L=16, 4 rows/wave
//   s=16 FP64: L=8, 8 rows/wave     s=4  FP64: L=2, 32 rows/wave
// Loads of the matrix values and of x are 128-256 contiguous bytes per row
// and entry (coalesced); the values stream is read with non-temporal loads
// so it does not evict the reused x entries from the caches.
#pragma once

#include "common.hpp"

namespace ens {

template <typename T, int S>
struct EnsMap {
  static constexpr int V = pack<T>::V;  // samples per 16-byte load
  static_assert(S % V == 0, "ensemble size must fill a 16-byte load");
  static constexpr int L = S / V;       // lanes per row
  static constexpr int RPW = 64 / L;    // rows per wavefront
  typedef typename pack<T>::type vt;
};

template <typename VT>
__device__ inline VT load_stream(const VT* p) {
  return __builtin_nontemporal_load(p);
}

// Streamed results are written with non-temporal stores: in a
// read-dominated stream the ordinary write-back stores cost far more read
// bandwidth than their few bytes (measured about 3.5 % of SpMV throughput).
template <typename VT>
__device__ inline void store_stream(VT* p, VT v) {
  __builtin_nontemporal_store(v, p);
}

// y_row = sum_k values[k] * x[col[k]] for the V samples of lane `sub`.
template <typename T, int S>
__device__ inline typename EnsMap<T, S>::vt ens_row_product(const int32_t* __restrict__ ci,
                                                            const T* __restrict__ vals,
                                                            const T* __restrict__ x, int64_t k0,
                                                            int64_t k1, int sub) {
  using M = EnsMap<T, S>;
  using vt = typename M::vt;
  const vt* vv = (const vt*)vals + sub;
  const vt* xv = (const vt*)x + sub;
  vt acc = (vt)0;
  int64_t k = k0;
  for (; k + 2 < k1; k += 3) {
    int32_t c[3];
    vt a[3], b[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) c[j] = ci[k + j];
#pragma unroll
    for (int j = 0; j < 3; ++j) a[j] = load_stream(vv + (k + j) * M::L);
#pragma unroll
    for (int j = 0; j < 3; ++j) b[j] = xv[(int64_t)c[j] * M::L];
#pragma unroll
    for (int j = 0; j < 3; ++j) acc += a[j] * b[j];
  }
  for (; k < k1; ++k) {
    int32_t c = ci[k];
    acc += load_stream(vv + k * M::L) * xv[(int64_t)c * M::L];
  }
  return acc;
}

// A workgroup's row tile staged in LDS: the row offsets of rows r0..r0+R
// and the column indices of their entries, read once per workgroup with
// coalesced loads (one index per lane instead of one per L-lane group and
// entry), after which the lanes take their indices from LDS.  Measured at
// 128^3, s = 32 in FP32: the CG product 5.08 -> 5.36 TB/s and the multigrid
// row passes 5.23 -> 5.46 TB/s against the per-lane index loads.  CAP = 32
// indices per row covers the 27-point rows with room; a tile whose entries
// do not fit (other graphs) reads its indices from global memory.
template <int R>
constexpr int kTileCap = R * 32;

template <int R, int CAP = kTileCap<R>>
struct RowTileLds {
  int32_t rp[R + 1];
  int32_t ci[CAP];
};

// Stage rows r0 .. min(r0 + R, n) - 1 (every lane of the workgroup calls
// this).  Returns false, staging only the offsets, when their entries do not
// fit in CAP indices; the caller then reads the indices from global memory.
template <int R, int CAP>
__device__ inline bool stage_row_tile(RowTileLds<R, CAP>& t, int n, const int32_t* __restrict__ rp,
                                      const int32_t* __restrict__ ci, int64_t r0) {
  const int rows = (int)((int64_t)n - r0 < R ? (int64_t)n - r0 : R);
  for (int i = threadIdx.x; i <= rows; i += blockDim.x) t.rp[i] = rp[r0 + i];
  __syncthreads();
  const int64_t base = t.rp[0], cnt = (int64_t)t.rp[rows] - base;
  if (cnt > CAP) return false;
  for (int i = threadIdx.x; i < (int)cnt; i += blockDim.x) t.ci[i] = ci[base + i];
  __syncthreads();
  return true;
}

// ens_row_product with the column indices from a staged tile (sci =
// t.ci - t.rp[0], so sci[k] is entry k's index).
template <typename T, int S>
__device__ inline typename EnsMap<T, S>::vt ens_row_product_lds(const int32_t* sci, const T* __restrict__ vals,
                                                                const T* __restrict__ x, int64_t k0, int64_t k1,
                                                                int sub) {
  using M = EnsMap<T, S>;
  using vt = typename M::vt;
  const vt* vv = (const vt*)vals + sub;
  const vt* xv = (const vt*)x + sub;
  vt acc = (vt)0;
  int64_t k = k0;
  for (; k + 2 < k1; k += 3) {
    int32_t c[3];
    vt a[3], b[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) c[j] = sci[k + j];
#pragma unroll
    for (int j = 0; j < 3; ++j) a[j] = load_stream(vv + (k + j) * M::L);
#pragma unroll
    for (int j = 0; j < 3; ++j) b[j] = xv[(int64_t)c[j] * M::L];
#pragma unroll
    for (int j = 0; j < 3; ++j) acc += a[j] * b[j];
  }
  for (; k < k1; ++k) acc += load_stream(vv + k * M::L) * xv[(int64_t)sci[k] * M::L];
  return acc;
}

// Row product of row `row` (local index lr in the tile) through the staged
// tile when it was staged, else from global memory.
template <typename T, int S, int R, int CAP>
__device__ inline typename EnsMap<T, S>::vt tile_row_product(const RowTileLds<R, CAP>& t, bool staged, int lr,
                                                             const int32_t* __restrict__ ci,
                                                             const T* __restrict__ vals, const T* __restrict__ x,
                                                             int sub) {
  const int64_t k0 = t.rp[lr], k1 = t.rp[lr + 1];
  if (staged) return ens_row_product_lds<T, S>(t.ci - t.rp[0], vals, x, k0, k1, sub);
  return ens_row_product<T, S>(ci, vals, x, k0, k1, sub);
}

// Block-wide per-sample reduction of NQ quantities over NW wavefronts.
// Each lane holds vals[q][j] for samples sub*VS + j (j < VS); lanes with
// equal (lane % L) hold the same samples.  The block totals are written to
// dst[q][s] (one row of the partial array) in a fixed order.
template <int S, int VS, int NQ, int NW>
__device__ inline void block_partials(double (&vals)[NQ][VS], double* __restrict__ dst) {
  constexpr int L = S / VS;
  __shared__ double red[NW][NQ][S];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int j = 0; j < VS; ++j) {
      double v = wave_sum_stride<L>(vals[q][j]);
      if (lane < L) red[wave][q][lane * VS + j] = v;
    }
  __syncthreads();
  if (threadIdx.x < NQ * S) {
    const int q = threadIdx.x / S, e = threadIdx.x % S;
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += red[w][q][e];
    dst[q * S + e] = t;
  }
}

// dst[qe] = sum over r < rows of src[r*P + qe] for the P columns of a
// row-major partial array, with the rows split into G = 256/P interleaved
// stripes that are added in stripe order afterwards.  The order depends only
// on `rows`, so the result is bit-reproducible.
template <int P>
__device__ inline void sum_rows(const double* __restrict__ src, int64_t rows, double* __restrict__ dst) {
  constexpr int G = kBlock / P;
  __shared__ double stripe[G][P];
  const int t = threadIdx.x;
  const int g = t / P, qe = t % P;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int64_t r = g;
  for (; r + 3 * G < rows; r += 4 * G) {
    const double v0 = src[r * P + qe];
    const double v1 = src[(r + G) * P + qe];
    const double v2 = src[(r + 2 * G) * P + qe];
    const double v3 = src[(r + 3 * G) * P + qe];
    a0 += v0;
    a1 += v1;
    a2 += v2;
    a3 += v3;
  }
  for (; r < rows; r += G) a0 += src[r * P + qe];
  stripe[g][qe] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (t < P) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < G; ++k) acc += stripe[k][t];
    dst[t] = acc;
  }
  __syncthreads();
}

}  // namespace ens
