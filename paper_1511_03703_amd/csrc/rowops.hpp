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
  for (; k + 8 < k1; k += 9) {
    int32_t c[9];
    vt a[9], b[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) c[j] = ci[k + j];
#pragma unroll
    for (int j = 0; j < 9; ++j) a[j] = load_stream(vv + (k + j) * M::L);
#pragma unroll
    for (int j = 0; j < 9; ++j) b[j] = xv[(int64_t)c[j] * M::L];
#pragma unroll
    for (int j = 0; j < 9; ++j) acc += a[j] * b[j];
  }
  for (; k < k1; ++k) {
    int32_t c = ci[k];
    acc += load_stream(vv + k * M::L) * xv[(int64_t)c * M::L];
  }
  return acc;
}

// Lanes that hold the same V samples (of different rows / entries) are L
// apart; sum a double over them.
template <int L>
__device__ inline double sum_same_samples(double v) {
  return wave_sum_stride<L>(v);
}

// Block-wide per-sample reduction of NQ quantities.  Each lane holds
// vals[q][j] for samples sub*VS + j (j < VS); lanes with equal (lane % L)
// hold the same samples.  Block totals land in part[blockIdx.x][q][s] in a
// fixed order (deterministic).
template <int S, int VS, int NQ>
__device__ inline void block_partials(double (&vals)[NQ][VS], double* __restrict__ part) {
  constexpr int L = S / VS;
  __shared__ double red[kBlock / 64][NQ][S];
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
    for (int w = 0; w < kBlock / 64; ++w) t += red[w][q][e];
    part[((int64_t)blockIdx.x * NQ + q) * S + e] = t;
  }
}

// Returns true in exactly one block: the last to finish writing its
// partials.  Release/acquire at device scope makes the other blocks'
// partials visible to it across the XCD L2 caches.
__device__ inline bool last_block_done(uint32_t* counter) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t prev = atomicAdd(counter, 1u);
    s_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (s_last) __threadfence();
  return s_last != 0;
}

// In the last block: tot[q][e] = sum over blocks of part[b][q][e], in
// ascending block order within each of G interleaved stripes, stripes then
// combined in order (deterministic for a fixed grid size).
template <int S, int NQ>
__device__ inline void final_totals(const double* __restrict__ part, int nblocks, double* __restrict__ tot) {
  constexpr int P = NQ * S;
  constexpr int G = kBlock / P > 0 ? kBlock / P : 1;
  __shared__ double stripe[G][P];
  const int t = threadIdx.x;
  if (t < G * P) {
    const int g = t / P, qe = t % P;
    double acc = 0.0;
    const volatile double* vp = part;
    for (int b = g; b < nblocks; b += G) acc += vp[(int64_t)b * P + qe];
    stripe[g][qe] = acc;
  }
  __syncthreads();
  if (t < P) {
    double acc = 0.0;
#pragma unroll
    for (int g = 0; g < G; ++g) acc += stripe[g][t];
    tot[t] = acc;
  }
  __syncthreads();
}

}  // namespace ens
