// Device side of the Jacobi-CG: per-sample state, the finalize step of each
// reduction, and the bodies of the fused CG kernels.  Each body takes the
// block index it works on and the row of the partial array it writes, so the
// same code runs one ensemble per launch (cg.hip) or many sample groups per
// launch (batch.hip).
#pragma once

#include "rowops.hpp"

namespace ens {

constexpr int kMaxS = 32;

enum CgOp { OP_START = 0, OP_RHO = 1, OP_ALPHA = 2, OP_UPDATE = 3, OP_TRUE = 4, OP_OUTER = 5, OP_UPDATE_R = 6,
            OP_BETA = 7 };

struct Ctl {
  double rho[kMaxS], alpha[kMaxS], beta[kMaxS], tol2[kMaxS], bnorm2[kMaxS];
  double rel_res[kMaxS], orr_prev[kMaxS];
  int32_t active[kMaxS], oactive[kMaxS], iters[kMaxS], oiters[kMaxS], kiter[kMaxS], status[kMaxS];
  int32_t zero_b[kMaxS];
  int32_t compacted[kMaxS];  // the sample finished in the compacted ensemble
  int32_t n_active, n_oactive;
  double rtol, inner_rtol;
  int32_t max_iter, inner_max_iter, max_outer, mixed;
  int32_t coupled;
  int32_t xnz;  // set when the initial guess has a nonzero entry
  double tot[2 * kMaxS];
};

// ------------------------------------------------------------- finalize ---

// Coupled mode (the solve of the whole commuted system, Sec. 3.4 and 3.7):
// the CG scalars use the ensemble sums of the inner products, added here in
// sample order by every thread alike, so all samples take the same alpha,
// beta and stopping decision; true residuals stay per sample.
template <int S>
__device__ void finalize(Ctl* c, int op, int arg) {
  const int e = threadIdx.x;
  if (e < S) {
    double t0 = c->tot[e], t1 = c->tot[S + e];
    if (c->coupled && op != OP_TRUE && op != OP_OUTER) {
      t0 = 0.0;
      t1 = 0.0;
      for (int j = 0; j < S; ++j) {
        t0 += c->tot[j];
        t1 += c->tot[S + j];
      }
    }
    switch (op) {
      case OP_START: {  // t0 = |b - A x0|^2, t1 = |b|^2
        c->bnorm2[e] = t1;
        c->tol2[e] = c->rtol * c->rtol * t1;
        c->iters[e] = 0;
        c->oiters[e] = 0;
        c->kiter[e] = 0;
        c->zero_b[e] = (t1 == 0.0);
        c->active[e] = 0;
        if (t1 == 0.0) {
          c->status[e] = ENS_SAMPLE_CONVERGED;
        } else if (!isfinite(t0) || !isfinite(t1)) {
          c->status[e] = ENS_SAMPLE_NONFINITE;
        } else if (t0 <= c->tol2[e]) {
          c->status[e] = ENS_SAMPLE_CONVERGED;
        } else {
          c->status[e] = ENS_SAMPLE_MAXITER;
          c->active[e] = 1;
        }
        break;
      }
      case OP_RHO: {  // t0 = r.z
        if (c->active[e]) {
          c->kiter[e] = 0;
          if (!isfinite(t0)) {
            c->status[e] = ENS_SAMPLE_NONFINITE;
            c->active[e] = 0;
            c->oactive[e] = 0;
          } else {
            c->rho[e] = t0;
          }
        }
        break;
      }
      case OP_ALPHA: {  // t0 = p.q
        if (c->active[e]) {
          const double rho = c->rho[e];
          if (!isfinite(t0) || !isfinite(rho)) {
            c->status[e] = ENS_SAMPLE_NONFINITE;
            c->active[e] = 0;
            c->oactive[e] = 0;
          } else if (!(t0 > 0.0)) {
            c->status[e] = ENS_SAMPLE_BREAKDOWN;
            c->active[e] = 0;
            c->oactive[e] = 0;
          } else {
            c->alpha[e] = rho / t0;
          }
        }
        break;
      }
      case OP_UPDATE: {  // t0 = r.z, t1 = r.r
        if (c->active[e]) {
          c->iters[e] += 1;
          c->kiter[e] += 1;
          const int cap = c->mixed ? c->inner_max_iter : c->max_iter;
          if (!isfinite(t0) || !isfinite(t1)) {
            c->status[e] = ENS_SAMPLE_NONFINITE;
            c->active[e] = 0;
            c->oactive[e] = 0;
          } else if (t1 <= c->tol2[e]) {
            c->active[e] = 0;
            if (!c->mixed) c->status[e] = ENS_SAMPLE_CONVERGED;
          } else if (c->kiter[e] >= cap) {
            c->active[e] = 0;
            if (!c->mixed) c->status[e] = ENS_SAMPLE_MAXITER;
          } else {
            c->beta[e] = t0 / c->rho[e];
            c->rho[e] = t0;
          }
        }
        break;
      }
      case OP_UPDATE_R: {  // t1 = r.r after x += alpha p, r -= alpha q (preconditioner applied next)
        if (c->active[e]) {
          c->iters[e] += 1;
          c->kiter[e] += 1;
          const int cap = c->mixed ? c->inner_max_iter : c->max_iter;
          if (!isfinite(t1)) {
            c->status[e] = ENS_SAMPLE_NONFINITE;
            c->active[e] = 0;
            c->oactive[e] = 0;
          } else if (t1 <= c->tol2[e]) {
            c->active[e] = 0;
            if (!c->mixed) c->status[e] = ENS_SAMPLE_CONVERGED;
          } else if (c->kiter[e] >= cap) {
            c->active[e] = 0;
            if (!c->mixed) c->status[e] = ENS_SAMPLE_MAXITER;
          }
        }
        break;
      }
      case OP_BETA: {  // t0 = r.z with z = M r
        if (c->active[e]) {
          if (!isfinite(t0)) {
            c->status[e] = ENS_SAMPLE_NONFINITE;
            c->active[e] = 0;
            c->oactive[e] = 0;
          } else {
            c->beta[e] = t0 / c->rho[e];
            c->rho[e] = t0;
          }
        }
        break;
      }
      case OP_TRUE: {  // t0 = |b - A x|^2, t1 = |b|^2
        c->rel_res[e] = t1 > 0.0 ? sqrt(t0 / t1) : sqrt(t0);
        break;
      }
      case OP_OUTER: {  // t0 = |b - A x|^2, t1 = |b|^2, arg = refinement step
        const int o = arg;
        if (o == 0) {
          c->bnorm2[e] = t1;
          c->zero_b[e] = (t1 == 0.0);
          c->oactive[e] = (t1 != 0.0);
          c->status[e] = t1 == 0.0 ? ENS_SAMPLE_CONVERGED : ENS_SAMPLE_MAXITER;
          c->iters[e] = 0;
          c->oiters[e] = 0;
          c->orr_prev[e] = INFINITY;
        }
        c->rel_res[e] = t1 > 0.0 ? sqrt(t0 / t1) : 0.0;
        c->active[e] = 0;
        if (c->oactive[e]) {
          const double rt = c->rtol;
          if (!isfinite(t0)) {
            c->status[e] = ENS_SAMPLE_NONFINITE;
            c->oactive[e] = 0;
          } else if (t0 <= rt * rt * t1) {
            c->status[e] = ENS_SAMPLE_CONVERGED;
            c->oactive[e] = 0;
          } else if (o >= 1 && t0 > 0.25 * c->orr_prev[e]) {
            c->status[e] = ENS_SAMPLE_STAGNATED;
            c->oactive[e] = 0;
          } else if (o >= c->max_outer) {
            c->status[e] = ENS_SAMPLE_MAXITER;
            c->oactive[e] = 0;
          } else {
            const double it = c->inner_rtol * c->inner_rtol * t0;
            const double fl = 0.09 * rt * rt * t1;
            c->tol2[e] = it > fl ? it : fl;
            c->active[e] = 1;
            c->oiters[e] += 1;
          }
          c->orr_prev[e] = t0;
        }
        break;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int na = 0, no = 0;
    for (int j = 0; j < S; ++j) {
      na += c->active[j];
      no += c->oactive[j];
    }
    c->n_active = na;
    c->n_oactive = no;
  }
}

// Streaming kernels process kU chunks per thread: all loads of a thread
// are issued before its stores, so the in-order memory counter never makes
// a load wait for an earlier store.  Vectors that a launch reads once (r,
// z, p, q, x, D^-1, b) are read with non-temporal loads and written with
// non-temporal stores: at the sizes here each is larger than the caches,
// and ordinary accesses evicted the lines the products reuse (the gathered
// x, the column indices); measured at 128^3, s = 32 in FP32, the CG
// product 5.36 -> 5.60 TB/s with its own code unchanged.
constexpr int kU = 4;

// Streaming kernels treat an [n][S] vector as chunks of V = min(16/sizeof(T),
// S) consecutive samples of one row (one 16-byte load for S >= 4; a single
// element for the one-sample path).  Lanes L = S/V apart hold the same
// samples.
template <typename T, int S>
struct VecMap {
  static constexpr int V = pack<T>::V < S ? pack<T>::V : S;
  static constexpr int VS = V;
  static constexpr int L = S / V;
  typedef typename vec_t<T, V>::type vt;
  __device__ static inline int sample(int sub, int v) { return sub * V + v; }
  __device__ static inline int slot(int v) { return v; }
};

static __global__ void k_ctl_init(Ctl* c, double rtol, double inner_rtol, int max_iter, int inner_max_iter,
                                  int max_outer, int mixed, int coupled) {
  if (threadIdx.x == 0) {
    c->rtol = rtol;
    c->inner_rtol = inner_rtol;
    c->max_iter = max_iter;
    c->inner_max_iter = inner_max_iter;
    c->max_outer = max_outer;
    c->mixed = mixed;
    c->coupled = coupled;
    c->xnz = 0;
    c->n_active = 0;
    c->n_oactive = 0;
  }
  if (threadIdx.x < kMaxS) {
    const int e = threadIdx.x;
    c->active[e] = 0;
    c->oactive[e] = 0;
    c->iters[e] = 0;
    c->oiters[e] = 0;
    c->kiter[e] = 0;
    c->status[e] = ENS_SAMPLE_MAXITER;
    c->zero_b[e] = 0;
    c->compacted[e] = 0;
    c->rel_res[e] = 0.0;
  }
}

// dinv[i][e] = 1 / A_ii[e] for the rows of block `blk` (256 (row, sample)
// pairs per block).
template <typename T, int S>
__device__ inline void diag_inv_body(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                     const T* __restrict__ vals, T* __restrict__ dinv, int64_t blk) {
  const int64_t t = blk * blockDim.x + threadIdx.x;
  const int64_t row = t / S;
  const int e = (int)(t % S);
  if (row >= n) return;
  T d = (T)0;
  for (int64_t k = rp[row]; k < rp[row + 1]; ++k)
    if (ci[k] == row) d = vals[k * S + e];
  dinv[row * S + e] = (T)1 / d;
}

// r = b - A x in FP64 for the row tile `blk` (NW wavefronts), optionally
// stored (rounded to TR), with the block's partials |r|^2 and |b|^2 written
// to dst[2][S].
template <int S, typename TR, int NW>
__device__ inline void residual_body(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                     const double* __restrict__ vals, const double* __restrict__ x,
                                     const double* __restrict__ b, TR* __restrict__ rout, int64_t blk,
                                     double* __restrict__ dst, bool x_zero = false) {
  using M = EnsMap<double, S>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane % M::L;
  double acc[2][M::V];
#pragma unroll
  for (int j = 0; j < M::V; ++j) acc[0][j] = acc[1][j] = 0.0;
  const int64_t row = (blk * NW + wave) * M::RPW + lane / M::L;
  constexpr int R = NW * M::RPW;
  __shared__ RowTileLds<R> tile;
  const bool staged = !x_zero && stage_row_tile(tile, n, rp, ci, blk * R);
  if (row < n) {
    typename M::vt ax = x_zero ? (typename M::vt)0.0
                               : tile_row_product<double, S>(tile, staged, (int)(row - blk * R), ci, vals, x, sub);
    typename M::vt bv = load_stream((const typename M::vt*)b + row * M::L + sub);
    typename M::vt r = bv - ax;
#pragma unroll
    for (int j = 0; j < M::V; ++j) {
      acc[0][j] = r[j] * r[j];
      acc[1][j] = bv[j] * bv[j];
    }
    if (rout) {
      typename vec_t<TR, M::V>::type rv;
#pragma unroll
      for (int j = 0; j < M::V; ++j) rv[j] = (TR)r[j];
      store_stream((typename vec_t<TR, M::V>::type*)(rout + row * S + sub * M::V), rv);
    }
  }
  block_partials<S, M::V, 2, NW>(acc, dst);
}

// z = D^-1 r, p = z (all samples); optionally zero the solution vector;
// partials r.z and r.r of chunk block `blk` to dst[2][S].
template <typename T, int S>
__device__ inline void cg_start_body(int64_t nchunks, const T* __restrict__ r, const T* __restrict__ dinv,
                                     T* __restrict__ p, T* __restrict__ xzero, int64_t blk,
                                     double* __restrict__ dst) {
  using M = VecMap<T, S>;
  using vt = typename M::vt;
  double acc[2][M::VS];
#pragma unroll
  for (int j = 0; j < M::VS; ++j) acc[0][j] = acc[1][j] = 0.0;
  const int64_t base = blk * kBlock * kU + threadIdx.x;
  vt rv[kU], dv[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int64_t i = base + u * kBlock;
    if (i < nchunks) {
      rv[u] = load_stream((const vt*)r + i);
      dv[u] = load_stream((const vt*)dinv + i);
    }
  }
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int64_t i = base + u * kBlock;
    if (i < nchunks) {
      vt z = dv[u] * rv[u];
      store_stream((vt*)p + i, z);
      if (xzero) ((vt*)xzero)[i] = (vt)0;
#pragma unroll
      for (int v = 0; v < M::V; ++v) {
        acc[0][M::slot(v)] += (double)rv[u][v] * (double)z[v];
        acc[1][M::slot(v)] += (double)rv[u][v] * (double)rv[u][v];
      }
    }
  }
  block_partials<S, M::VS, 2, kBlock / 64>(acc, dst);
}

// A: q = A p for row tile `blk` (NW wavefronts), partials p.q to dst[S].
template <typename T, int S, int NW>
__device__ inline void spmv_dot_body(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                     const T* __restrict__ vals, const T* __restrict__ p, T* __restrict__ q,
                                     int64_t blk, double* __restrict__ dst) {
  using M = EnsMap<T, S>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane % M::L;
  double acc[1][M::V];
#pragma unroll
  for (int j = 0; j < M::V; ++j) acc[0][j] = 0.0;
  const int64_t row = (blk * NW + wave) * M::RPW + lane / M::L;
  constexpr int R = NW * M::RPW;
  __shared__ RowTileLds<R> tile;
  const bool staged = stage_row_tile(tile, n, rp, ci, blk * R);
  if (row < n) {
    typename M::vt qv = tile_row_product<T, S>(tile, staged, (int)(row - blk * R), ci, vals, p, sub);
    store_stream((typename M::vt*)q + row * M::L + sub, qv);
    typename M::vt pv = ((const typename M::vt*)p)[row * M::L + sub];
#pragma unroll
    for (int j = 0; j < M::V; ++j) acc[0][j] = (double)pv[j] * (double)qv[j];
  }
  block_partials<S, M::V, 1, NW>(acc, dst);
}

// B: x += alpha p; r -= alpha q; z = D^-1 r for chunk block `blk`; partials
// r.z, r.r to dst[2][S].  Samples that are not active stay frozen.
template <typename T, int S>
__device__ inline void update_body(int64_t nchunks, T* __restrict__ x, const T* __restrict__ p,
                                   const T* __restrict__ q, T* __restrict__ r, const T* __restrict__ dinv,
                                   const Ctl* c, int64_t blk, double* __restrict__ dst) {
  using M = VecMap<T, S>;
  using vt = typename M::vt;
  const int sub = (threadIdx.x & 63) % M::L;
  vt al;
  int act[M::V];
#pragma unroll
  for (int v = 0; v < M::V; ++v) {
    const int e = M::sample(sub, v);
    act[v] = c->active[e];
    al[v] = act[v] ? (T)c->alpha[e] : (T)0;
  }
  double acc[2][M::VS];
#pragma unroll
  for (int j = 0; j < M::VS; ++j) acc[0][j] = acc[1][j] = 0.0;
  const int64_t base = blk * kBlock * kU + threadIdx.x;
  vt pv[kU], qv[kU], rv[kU], xv[kU], dv[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int64_t i = base + u * kBlock;
    if (i < nchunks) {
      pv[u] = load_stream((const vt*)p + i);
      qv[u] = load_stream((const vt*)q + i);
      rv[u] = load_stream((const vt*)r + i);
      xv[u] = load_stream((const vt*)x + i);
      dv[u] = load_stream((const vt*)dinv + i);
    }
  }
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int64_t i = base + u * kBlock;
    if (i < nchunks) {
      vt xn = xv[u] + al * pv[u];
      vt rn = rv[u] - al * qv[u];
#pragma unroll
      for (int v = 0; v < M::V; ++v)  // converged or stopped samples stay frozen
        if (!act[v]) {
          xn[v] = xv[u][v];
          rn[v] = rv[u][v];
        }
      xv[u] = xn;
      rv[u] = rn;
      vt z = dv[u] * rn;
#pragma unroll
      for (int v = 0; v < M::V; ++v) {
        const double rr = act[v] ? (double)rn[v] : 0.0;
        acc[0][M::slot(v)] += rr * (double)z[v];
        acc[1][M::slot(v)] += rr * rr;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int64_t i = base + u * kBlock;
    if (i < nchunks) {
      store_stream((vt*)x + i, xv[u]);
      store_stream((vt*)r + i, rv[u]);
    }
  }
  block_partials<S, M::VS, 2, kBlock / 64>(acc, dst);
}

// C: p = D^-1 r + beta p for the samples still active, chunk block `blk`.
template <typename T, int S>
__device__ inline void pupdate_body(int64_t nchunks, const T* __restrict__ r, const T* __restrict__ dinv,
                                    T* __restrict__ p, const Ctl* c, int64_t blk) {
  using M = VecMap<T, S>;
  using vt = typename M::vt;
  const int sub = (threadIdx.x & 63) % M::L;
  vt be;
  int act[M::V];
  bool any = false;
#pragma unroll
  for (int v = 0; v < M::V; ++v) {
    const int e = M::sample(sub, v);
    act[v] = c->active[e];
    be[v] = act[v] ? (T)c->beta[e] : (T)0;
    any |= act[v] != 0;
  }
  if (!any) return;
  const int64_t base = blk * kBlock * kU + threadIdx.x;
  vt pv[kU], rv[kU], dv[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int64_t i = base + u * kBlock;
    if (i < nchunks) {
      pv[u] = load_stream((const vt*)p + i);
      rv[u] = load_stream((const vt*)r + i);
      dv[u] = load_stream((const vt*)dinv + i);
    }
  }
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int64_t i = base + u * kBlock;
    if (i < nchunks) {
      vt pn = dv[u] * rv[u] + be * pv[u];
#pragma unroll
      for (int v = 0; v < M::V; ++v)  // inactive samples keep their p
        if (!act[v]) pn[v] = pv[u][v];
      store_stream((vt*)p + i, pn);
    }
  }
}

// Multigrid-preconditioned iteration, update half: x += alpha p; r -= alpha
// q for the active samples; partials (0, r.r) of chunk block `blk` to dst.
template <typename T, int S>
__device__ inline void update_r_body(int64_t nchunks, T* __restrict__ x, const T* __restrict__ p,
                                     const T* __restrict__ q, T* __restrict__ r, const Ctl* c, int64_t blk,
                                     double* __restrict__ dst) {
  using M = VecMap<T, S>;
  using vt = typename M::vt;
  const int sub = (threadIdx.x & 63) % M::L;
  vt al;
  int act[M::V];
#pragma unroll
  for (int v = 0; v < M::V; ++v) {
    const int e = M::sample(sub, v);
    act[v] = c->active[e];
    al[v] = act[v] ? (T)c->alpha[e] : (T)0;
  }
  double acc[2][M::VS];
#pragma unroll
  for (int j = 0; j < M::VS; ++j) acc[0][j] = acc[1][j] = 0.0;
  const int64_t base = blk * kBlock * kU + threadIdx.x;
  vt pv[kU], qv[kU], rv[kU], xv[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int64_t i = base + u * kBlock;
    if (i < nchunks) {
      pv[u] = load_stream((const vt*)p + i);
      qv[u] = load_stream((const vt*)q + i);
      rv[u] = load_stream((const vt*)r + i);
      xv[u] = load_stream((const vt*)x + i);
    }
  }
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int64_t i = base + u * kBlock;
    if (i < nchunks) {
      vt xn = xv[u] + al * pv[u];
      vt rn = rv[u] - al * qv[u];
#pragma unroll
      for (int v = 0; v < M::V; ++v)
        if (!act[v]) {
          xn[v] = xv[u][v];
          rn[v] = rv[u][v];
        }
      xv[u] = xn;
      rv[u] = rn;
#pragma unroll
      for (int v = 0; v < M::V; ++v) {
        const double rr = act[v] ? (double)rn[v] : 0.0;
        acc[1][M::slot(v)] += rr * rr;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int64_t i = base + u * kBlock;
    if (i < nchunks) {
      store_stream((vt*)x + i, xv[u]);
      store_stream((vt*)r + i, rv[u]);
    }
  }
  block_partials<S, M::VS, 2, kBlock / 64>(acc, dst);
}

// Partials (r.z, 0) of chunk block `blk`; with pz, also p = z (start).
template <typename T, int S>
__device__ inline void rz_body(int64_t nchunks, const T* __restrict__ r, const T* __restrict__ z,
                               T* __restrict__ pz, int64_t blk, double* __restrict__ dst) {
  using M = VecMap<T, S>;
  using vt = typename M::vt;
  double acc[2][M::VS];
#pragma unroll
  for (int j = 0; j < M::VS; ++j) acc[0][j] = acc[1][j] = 0.0;
  const int64_t base = blk * kBlock * kU + threadIdx.x;
  vt rv[kU], zv[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int64_t i = base + u * kBlock;
    if (i < nchunks) {
      rv[u] = load_stream((const vt*)r + i);
      zv[u] = load_stream((const vt*)z + i);
    }
  }
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int64_t i = base + u * kBlock;
    if (i < nchunks) {
      if (pz) store_stream((vt*)pz + i, zv[u]);
#pragma unroll
      for (int v = 0; v < M::V; ++v) acc[0][M::slot(v)] += (double)rv[u][v] * (double)zv[u][v];
    }
  }
  block_partials<S, M::VS, 2, kBlock / 64>(acc, dst);
}

// p = z + beta p for the samples still active.
template <typename T, int S>
__device__ inline void pupdate_z_body(int64_t nchunks, const T* __restrict__ z, T* __restrict__ p,
                                      const Ctl* c, int64_t blk) {
  using M = VecMap<T, S>;
  using vt = typename M::vt;
  const int sub = (threadIdx.x & 63) % M::L;
  vt be;
  int act[M::V];
  bool any = false;
#pragma unroll
  for (int v = 0; v < M::V; ++v) {
    const int e = M::sample(sub, v);
    act[v] = c->active[e];
    be[v] = act[v] ? (T)c->beta[e] : (T)0;
    any |= act[v] != 0;
  }
  if (!any) return;
  const int64_t base = blk * kBlock * kU + threadIdx.x;
  vt pv[kU], zv[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int64_t i = base + u * kBlock;
    if (i < nchunks) {
      pv[u] = load_stream((const vt*)p + i);
      zv[u] = load_stream((const vt*)z + i);
    }
  }
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int64_t i = base + u * kBlock;
    if (i < nchunks) {
      vt pn = zv[u] + be * pv[u];
#pragma unroll
      for (int v = 0; v < M::V; ++v)
        if (!act[v]) pn[v] = pv[u][v];
      store_stream((vt*)p + i, pn);
    }
  }
}

// c->xnz = 1 if any of the `total` entries of x is nonzero (every block
// that finds one stores the same value).
// total is n * S with S >= 4, so x is read as 16-byte pairs, four loads in
// flight per lane.
__device__ inline void x_nonzero_body(int64_t total, const double* __restrict__ x, Ctl* c) {
  const int64_t nv = total / 2, stride = (int64_t)gridDim.x * blockDim.x;
  const double2* __restrict__ xv = (const double2*)x;
  int any = 0;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < nv; i += 4 * stride) {
    const double2 a = xv[i], b = xv[i + stride], d = xv[i + 2 * stride], e = xv[i + 3 * stride];
    any |= (a.x != 0.0) | (a.y != 0.0) | (b.x != 0.0) | (b.y != 0.0) | (d.x != 0.0) | (d.y != 0.0) |
           (e.x != 0.0) | (e.y != 0.0);
  }
  for (; i < nv; i += stride) {
    const double2 a = xv[i];
    any |= (a.x != 0.0) | (a.y != 0.0);
  }
  if (__syncthreads_or(any) && threadIdx.x == 0) c->xnz = 1;
}

// x = 0 for samples whose right-hand side is zero.
template <int S>
__device__ inline void zero_where_body(int64_t total, double* __restrict__ x, const Ctl* c, int64_t i0,
                                       int64_t stride) {
  for (int64_t i = i0; i < total; i += stride)
    if (c->zero_b[i % S]) x[i] = 0.0;
}

}  // namespace ens
