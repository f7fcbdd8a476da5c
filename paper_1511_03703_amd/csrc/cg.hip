// Ensemble Jacobi-preconditioned CG with per-sample scalars, its FP32-in-FP64
// iterative-refinement form, and the one-sample-at-a-time baseline.
//
// Sec. 3.4 runs CG on the ensemble system and notes that a solver only sees
// inner products; for the commuted Kronecker system the ensemble inner
// product first forms sum_i u_i^T v_i (x) e_i, one value per sample.  We keep
// exactly that per-sample vector and give every sample its own alpha, beta,
// rho and convergence mask, so sample e follows its own scalar CG iteration
// (the block-diagonal structure of Eq. kron_sys) while all samples share one
// pass over the graph.  The preconditioner is the diagonal instance of the
// ensemble preconditioner M_c = sum_i M_i (x) e_i e_i^T of Sec. 3.5.
//
// One iteration is three fused kernels:
//   A: q = A p and the per-sample partials of p.q   -> alpha_e (last block)
//   B: x += alpha p, r -= alpha q, z = D^-1 r, partials of r.z and r.r
//                                                   -> masks, beta_e (last block)
//   C: p = z + beta p
// Reductions are two-level and deterministic: wave butterflies between lanes
// holding the same samples, a fixed-order LDS sum per block, and the block
// partials summed in a fixed order by the last block to finish.  That block
// also updates the per-sample scalars and the count of active samples; every
// kernel returns immediately when the count is zero, and the host reads the
// count once per chunk of iterations, so the loop ends on the device.
#include "rowops.hpp"

namespace ens {

constexpr int kMaxS = 32;

enum CgOp { OP_START = 0, OP_RHO = 1, OP_ALPHA = 2, OP_UPDATE = 3, OP_TRUE = 4, OP_OUTER = 5 };

struct Ctl {
  double rho[kMaxS], alpha[kMaxS], beta[kMaxS], tol2[kMaxS], bnorm2[kMaxS];
  double rel_res[kMaxS], orr_prev[kMaxS];
  int32_t active[kMaxS], oactive[kMaxS], iters[kMaxS], oiters[kMaxS], kiter[kMaxS], status[kMaxS];
  int32_t zero_b[kMaxS];
  int32_t n_active, n_oactive;
  uint32_t counter[4];               // last-group counters, one per reduction site
  uint32_t gcount[4][kMaxGroups];    // per-group arrival counters
  double rtol, inner_rtol;
  int32_t max_iter, inner_max_iter, max_outer, mixed;
  double tot[2 * kMaxS];
};

// ------------------------------------------------------------- finalize ---

template <int S>
__device__ void finalize(Ctl* c, int op, int arg) {
  const int e = threadIdx.x;
  if (e < S) {
    const double t0 = c->tot[e], t1 = c->tot[S + e];
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

// Finishes a reduction site: block partials, grid total, finalize.  The
// partial buffer holds kMaxPartBlocks block rows followed by kMaxGroups
// group rows of NQ*S doubles.
template <int S, int VS, int NQ>
__device__ inline void reduce_site(double (&vals)[NQ][VS], double* __restrict__ part, Ctl* c, int site, int op,
                                   int arg) {
  block_partials<S, VS, NQ>(vals, part);
  double* gpart = part + (int64_t)kMaxPartBlocks * NQ * S;
  if (grid_total<NQ * S>(part, gpart, c->gcount[site], &c->counter[site], c->tot)) {
    if (NQ == 1 && threadIdx.x < S) c->tot[S + threadIdx.x] = 0.0;
    __syncthreads();
    finalize<S>(c, op, arg);
  }
}

// --------------------------------------------------------- vector mapping ---

// Streaming kernels treat an [n][S] vector as chunks of V = min(16/sizeof(T),
// S) consecutive samples of one row (one 16-byte load for S >= 4; a single
// element for the one-sample path).  Lanes L = S/V apart hold the same
// samples, and a grid-stride loop keeps each lane on the same samples.
template <typename T, int S>
struct VecMap {
  static constexpr int V = pack<T>::V < S ? pack<T>::V : S;
  static constexpr int VS = V;
  static constexpr int L = S / V;
  typedef typename vec_t<T, V>::type vt;
  __device__ static inline int sample(int sub, int v) { return sub * V + v; }
  __device__ static inline int slot(int v) { return v; }
};

// ------------------------------------------------------------ kernels ---

__global__ void k_ctl_init(Ctl* c, double rtol, double inner_rtol, int max_iter, int inner_max_iter,
                           int max_outer, int mixed) {
  if (threadIdx.x == 0) {
    c->rtol = rtol;
    c->inner_rtol = inner_rtol;
    c->max_iter = max_iter;
    c->inner_max_iter = inner_max_iter;
    c->max_outer = max_outer;
    c->mixed = mixed;
    c->n_active = 0;
    c->n_oactive = 0;
    for (int i = 0; i < 4; ++i) c->counter[i] = 0;
  }
  for (int i = threadIdx.x; i < 4 * kMaxGroups; i += blockDim.x) c->gcount[i / kMaxGroups][i % kMaxGroups] = 0;
  if (threadIdx.x < kMaxS) {
    const int e = threadIdx.x;
    c->active[e] = 0;
    c->oactive[e] = 0;
    c->iters[e] = 0;
    c->oiters[e] = 0;
    c->kiter[e] = 0;
    c->status[e] = ENS_SAMPLE_MAXITER;
    c->zero_b[e] = 0;
    c->rel_res[e] = 0.0;
  }
}

// dinv[i][e] = 1 / A_ii[e]
template <typename T, int S>
__global__ __launch_bounds__(256) void k_diag_inv(int n, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci, const T* __restrict__ vals,
                                                  T* __restrict__ dinv) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = t / S;
  const int e = (int)(t % S);
  if (row >= n) return;
  T d = (T)0;
  for (int64_t k = rp[row]; k < rp[row + 1]; ++k)
    if (ci[k] == row) d = vals[k * S + e];
  dinv[row * S + e] = (T)1 / d;
}

// r = b - A x in FP64 for every sample (ensemble layout), optionally stored
// (rounded to TR), with partials |r|^2 and |b|^2.
template <int S, typename TR>
__global__ __launch_bounds__(256) void k_residual(int n, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci, const double* __restrict__ vals,
                                                  const double* __restrict__ x, const double* __restrict__ b,
                                                  TR* __restrict__ rout, Ctl* c, double* __restrict__ part, int op,
                                                  int arg) {
  using M = EnsMap<double, S>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane % M::L;
  double acc[2][M::V];
#pragma unroll
  for (int j = 0; j < M::V; ++j) acc[0][j] = acc[1][j] = 0.0;
  const int64_t tiles = ((int64_t)n + 4 * M::RPW - 1) / (4 * M::RPW);
#pragma unroll 1
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t row = (tile * 4 + wave) * M::RPW + lane / M::L;
    if (row < n) {
      typename M::vt ax = ens_row_product<double, S>(ci, vals, x, rp[row], rp[row + 1], sub);
      typename M::vt bv = ((const typename M::vt*)b)[row * M::L + sub];
      typename M::vt r = bv - ax;
#pragma unroll
      for (int j = 0; j < M::V; ++j) {
        acc[0][j] += r[j] * r[j];
        acc[1][j] += bv[j] * bv[j];
      }
      if (rout) {
#pragma unroll
        for (int j = 0; j < M::V; ++j) rout[row * S + sub * M::V + j] = (TR)r[j];
      }
    }
  }
  reduce_site<S, M::V, 2>(acc, part, c, 0, op, arg);
}

// z = D^-1 r, p = z (all samples); optionally zero the solution vector;
// partials r.z and r.r; finalize OP_RHO.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_cg_start(int64_t nchunks, const T* __restrict__ r,
                                                  const T* __restrict__ dinv, T* __restrict__ p,
                                                  T* __restrict__ xzero, Ctl* c, double* __restrict__ part) {
  using M = VecMap<T, S>;
  using vt = typename M::vt;
  const int sub = (threadIdx.x & 63) % M::L;
  double acc[2][M::VS];
#pragma unroll
  for (int j = 0; j < M::VS; ++j) acc[0][j] = acc[1][j] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nchunks; i += stride) {
    vt rv = ((const vt*)r)[i], dv = ((const vt*)dinv)[i];
    vt z = dv * rv;
    ((vt*)p)[i] = z;
    if (xzero) ((vt*)xzero)[i] = (vt)0;
#pragma unroll
    for (int v = 0; v < M::V; ++v) {
      acc[0][M::slot(v)] += (double)rv[v] * (double)z[v];
      acc[1][M::slot(v)] += (double)rv[v] * (double)rv[v];
    }
  }
  (void)sub;
  reduce_site<S, M::VS, 2>(acc, part, c, 1, OP_RHO, 0);
}

// A: q = A p, partials p.q, finalize alpha.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_cg_spmv_dot(int n, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, const T* __restrict__ vals,
                                                     const T* __restrict__ p, T* __restrict__ q, Ctl* c,
                                                     double* __restrict__ part) {
  if (c->n_active == 0) return;
  using M = EnsMap<T, S>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane % M::L;
  double acc[1][M::V];
#pragma unroll
  for (int j = 0; j < M::V; ++j) acc[0][j] = 0.0;
  const int64_t tiles = ((int64_t)n + 4 * M::RPW - 1) / (4 * M::RPW);
#pragma unroll 1
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t row = (tile * 4 + wave) * M::RPW + lane / M::L;
    if (row < n) {
      typename M::vt qv = ens_row_product<T, S>(ci, vals, p, rp[row], rp[row + 1], sub);
      ((typename M::vt*)q)[row * M::L + sub] = qv;
      typename M::vt pv = ((const typename M::vt*)p)[row * M::L + sub];
#pragma unroll
      for (int j = 0; j < M::V; ++j) acc[0][j] += (double)pv[j] * (double)qv[j];
    }
  }
  reduce_site<S, M::V, 1>(acc, part, c, 2, OP_ALPHA, 0);
}

// B: x += alpha p; r -= alpha q; z = D^-1 r; partials r.z, r.r; finalize.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_cg_update(int64_t nchunks, T* __restrict__ x, const T* __restrict__ p,
                                                   const T* __restrict__ q, T* __restrict__ r,
                                                   const T* __restrict__ dinv, Ctl* c, double* __restrict__ part,
                                                   int k) {
  if (c->n_active == 0) return;
  using M = VecMap<T, S>;
  using vt = typename M::vt;
  const int sub = (threadIdx.x & 63) % M::L;
  vt al;
  bool any = false;
  int act[M::V];
#pragma unroll
  for (int v = 0; v < M::V; ++v) {
    const int e = M::sample(sub, v);
    act[v] = c->active[e];
    al[v] = act[v] ? (T)c->alpha[e] : (T)0;
    any |= act[v] != 0;
  }
  double acc[2][M::VS];
#pragma unroll
  for (int j = 0; j < M::VS; ++j) acc[0][j] = acc[1][j] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (any) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nchunks; i += stride) {
      vt pv = ((const vt*)p)[i], qv = ((const vt*)q)[i], rv = ((const vt*)r)[i], xv = ((const vt*)x)[i];
      vt dv = ((const vt*)dinv)[i];
      xv += al * pv;
      rv -= al * qv;
      vt z = dv * rv;
      ((vt*)x)[i] = xv;
      ((vt*)r)[i] = rv;
#pragma unroll
      for (int v = 0; v < M::V; ++v) {
        if (act[v]) {
          acc[0][M::slot(v)] += (double)rv[v] * (double)z[v];
          acc[1][M::slot(v)] += (double)rv[v] * (double)rv[v];
        }
      }
    }
  }
  reduce_site<S, M::VS, 2>(acc, part, c, 3, OP_UPDATE, k);
}

// C: p = D^-1 r + beta p for the samples still active.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_cg_pupdate(int64_t nchunks, const T* __restrict__ r,
                                                    const T* __restrict__ dinv, T* __restrict__ p, Ctl* c) {
  if (c->n_active == 0) return;
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
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nchunks; i += stride) {
    vt rv = ((const vt*)r)[i], dv = ((const vt*)dinv)[i], pv = ((const vt*)p)[i];
    vt pn = dv * rv + be * pv;
#pragma unroll
    for (int v = 0; v < M::V; ++v)  // inactive samples keep their p
      if (!act[v]) pn[v] = pv[v];
    ((vt*)p)[i] = pn;
  }
}

// x += d for the samples still in refinement (FP64 += FP32 correction).
template <int S>
__global__ __launch_bounds__(256) void k_ir_update(int64_t total, double* __restrict__ x,
                                                   const float* __restrict__ d, const Ctl* c) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int e = (int)(i % S);
    if (c->oactive[e]) x[i] += (double)d[i];
  }
}

// x = 0 for samples whose right-hand side is zero.
template <int S>
__global__ __launch_bounds__(256) void k_zero_where(int64_t total, double* __restrict__ x, const Ctl* c) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    if (c->zero_b[i % S]) x[i] = 0.0;
  }
}

// ----------------------------------------------- one-sample (scalar) path ---

// residual with G lanes per row (scalar CRS)
template <int G>
__global__ __launch_bounds__(256) void k_residual_scalar(int n, const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci,
                                                         const double* __restrict__ vals,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ b, double* __restrict__ rout,
                                                         Ctl* c, double* __restrict__ part, int op) {
  const int g = threadIdx.x % G;
  double acc[2][1] = {{0.0}, {0.0}};
  const int64_t rows_per_iter = (int64_t)gridDim.x * (256 / G);
  for (int64_t row = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G; row < n; row += rows_per_iter) {
    double s = 0.0;
    for (int64_t k = rp[row] + g; k < rp[row + 1]; k += G) s += __builtin_nontemporal_load(vals + k) * x[ci[k]];
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (g == 0) {
      const double r = b[row] - s;
      if (rout) rout[row] = r;
      acc[0][0] += r * r;
      acc[1][0] += b[row] * b[row];
    }
  }
  reduce_site<1, 1, 2>(acc, part, c, 0, op, 0);
}

template <int G>
__global__ __launch_bounds__(256) void k_cg_spmv_dot_scalar(int n, const int32_t* __restrict__ rp,
                                                            const int32_t* __restrict__ ci,
                                                            const double* __restrict__ vals,
                                                            const double* __restrict__ p, double* __restrict__ q,
                                                            Ctl* c, double* __restrict__ part) {
  if (c->n_active == 0) return;
  const int g = threadIdx.x % G;
  double acc[1][1] = {{0.0}};
  const int64_t rows_per_iter = (int64_t)gridDim.x * (256 / G);
  for (int64_t row = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G; row < n; row += rows_per_iter) {
    double s = 0.0;
    for (int64_t k = rp[row] + g; k < rp[row + 1]; k += G) s += __builtin_nontemporal_load(vals + k) * p[ci[k]];
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (g == 0) {
      q[row] = s;
      acc[0][0] += p[row] * s;
    }
  }
  reduce_site<1, 1, 1>(acc, part, c, 2, OP_ALPHA, 0);
}

// ------------------------------------------------------------ host side ---

struct Work {
  Ctl* ctl;
  double* part;
  void* vec[5];
};

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t ws_layout(int64_t n, int s, bool mixed, Work* w, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? base + off : nullptr;
    off += round256(bytes);
    return p;
  };
  Ctl* ctl = (Ctl*)take(sizeof(Ctl));
  double* part = (double*)take((size_t)(kMaxPartBlocks + kMaxGroups) * 2 * kMaxS * sizeof(double));
  const size_t vb = (size_t)n * s * (mixed ? sizeof(float) : sizeof(double));
  void* v[5];
  for (int i = 0; i < 5; ++i) v[i] = take(vb);
  if (w) {
    w->ctl = ctl;
    w->part = part;
    for (int i = 0; i < 5; ++i) w->vec[i] = v[i];
  }
  return off;
}

static int stream_blocks(int64_t items) {
  int64_t b = (items + kBlock - 1) / kBlock;
  if (b > kStreamBlocks) b = kStreamBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

static int row_blocks(int64_t n, int rows_per_tile) {
  int64_t b = (n + rows_per_tile - 1) / rows_per_tile;
  if (b > kStreamBlocks) b = kStreamBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

static ens_status poll_active(Ctl* ctl, bool outer, hipStream_t st, int32_t* out) {
  DeviceCtx* cx = device_ctx();
  if (!cx) {
    set_error("device context unavailable");
    return ENS_E_HIP;
  }
  ENS_HIP_TRY(hipMemcpyAsync(cx->host_flag, outer ? &ctl->n_oactive : &ctl->n_active, sizeof(int32_t),
                             hipMemcpyDeviceToHost, st));
  ENS_HIP_TRY(hipStreamSynchronize(st));
  prof_collect();
  *out = *cx->host_flag;
  return ENS_OK;
}

// CG loop on already-initialised state; x is the solution (FP64 CG) or
// the correction d (refinement inner solve).
template <typename T, int S>
static ens_status cg_loop(const ens_graph* g, const T* vals, T* x, T* r, T* p, T* q, T* dinv, Work& w,
                          int max_iter, int check_every, hipStream_t st) {
  using M = EnsMap<T, S>;
  const int64_t nchunks = (int64_t)g->n * S / VecMap<T, S>::V;
  const int vb = stream_blocks(nchunks);
  const int sb = row_blocks(g->n, 4 * M::RPW);
  const int kid = sizeof(T) == 8 ? ENS_K_SPMV_F64 : ENS_K_SPMV_F32;
  const double w_ = sizeof(T);
  const double spmv_bytes = (double)g->nnz * (S * w_ + 4.0) + 4.0 * (g->n + 1) + 2.0 * g->n * S * w_;
  for (int k0 = 0; k0 < max_iter; k0 += check_every) {
    const int k1 = k0 + check_every < max_iter ? k0 + check_every : max_iter;
    for (int k = k0 + 1; k <= k1; ++k) {
      prof_begin(kid, st);
      hipLaunchKernelGGL((k_cg_spmv_dot<T, S>), dim3(sb), dim3(kBlock), 0, st, g->n, g->row_ptr, g->col_idx, vals,
                         p, q, w.ctl, w.part);
      prof_end(kid, st, spmv_bytes);
      hipLaunchKernelGGL((k_cg_update<T, S>), dim3(vb), dim3(kBlock), 0, st, nchunks, x, p, q, r, dinv, w.ctl,
                         w.part, k);
      hipLaunchKernelGGL((k_cg_pupdate<T, S>), dim3(vb), dim3(kBlock), 0, st, nchunks, r, dinv, p, w.ctl);
    }
    ENS_LAUNCH_CHECK();
    int32_t act = 0;
    ens_status s2 = poll_active(w.ctl, false, st, &act);
    if (s2 != ENS_OK) return s2;
    if (act == 0) break;
  }
  return ENS_OK;
}

static ens_status read_stats(Ctl* ctl, int s, ens_cg_stat* stats, hipStream_t st) {
  Ctl h;
  ENS_HIP_TRY(hipMemcpyAsync(&h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  ENS_HIP_TRY(hipStreamSynchronize(st));
  prof_collect();
  ens_status rc = ENS_OK;
  for (int e = 0; e < s; ++e) {
    stats[e].iters = h.iters[e];
    stats[e].outer_iters = h.oiters[e];
    stats[e].status = h.status[e];
    stats[e].reserved = 0;
    stats[e].rel_res = h.rel_res[e];
    if (h.status[e] != ENS_SAMPLE_CONVERGED) rc = ENS_W_NOT_CONVERGED;
  }
  return rc;
}

template <int S>
static ens_status cg_fp64(const ens_graph* g, const double* vals, const double* b, double* x,
                          const ens_cg_opts& o, Work& w, hipStream_t st) {
  using M = EnsMap<double, S>;
  double* r = (double*)w.vec[0];
  double* p = (double*)w.vec[1];
  double* q = (double*)w.vec[2];
  double* dinv = (double*)w.vec[3];
  const int64_t n = g->n;
  const int64_t total = n * S;
  const int sb = row_blocks(n, 4 * M::RPW);
  const int vb = stream_blocks(total / VecMap<double, S>::V);
  hipLaunchKernelGGL((k_diag_inv<double, S>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g->n,
                     g->row_ptr, g->col_idx, vals, dinv);
  hipLaunchKernelGGL((k_residual<S, double>), dim3(sb), dim3(kBlock), 0, st, g->n, g->row_ptr, g->col_idx, vals, x,
                     b, r, w.ctl, w.part, (int)OP_START, 0);
  hipLaunchKernelGGL(k_zero_where<S>, dim3(stream_blocks(total)), dim3(kBlock), 0, st, total, x, w.ctl);
  hipLaunchKernelGGL((k_cg_start<double, S>), dim3(vb), dim3(kBlock), 0, st, total / VecMap<double, S>::V, r, dinv, p,
                     (double*)nullptr, w.ctl, w.part);
  ENS_LAUNCH_CHECK();
  ens_status rc = cg_loop<double, S>(g, vals, x, r, p, q, dinv, w, o.max_iter, o.check_every, st);
  if (rc != ENS_OK) return rc;
  hipLaunchKernelGGL((k_residual<S, double>), dim3(sb), dim3(kBlock), 0, st, g->n, g->row_ptr, g->col_idx, vals, x,
                     b, (double*)nullptr, w.ctl, w.part, (int)OP_TRUE, 0);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

template <int S>
static ens_status cg_mixed(const ens_graph* g, const double* vals, const float* vals32, const double* b, double* x,
                           const ens_cg_opts& o, Work& w, hipStream_t st) {
  using M = EnsMap<double, S>;
  float* r = (float*)w.vec[0];
  float* p = (float*)w.vec[1];
  float* q = (float*)w.vec[2];
  float* dinv = (float*)w.vec[3];
  float* d = (float*)w.vec[4];
  const int64_t n = g->n;
  const int64_t total = n * S;
  const int sb = row_blocks(n, 4 * M::RPW);
  const int vb = stream_blocks(total / VecMap<float, S>::V);
  hipLaunchKernelGGL((k_diag_inv<float, S>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g->n,
                     g->row_ptr, g->col_idx, vals32, dinv);
  ENS_LAUNCH_CHECK();
  for (int outer = 0;; ++outer) {
    hipLaunchKernelGGL((k_residual<S, float>), dim3(sb), dim3(kBlock), 0, st, g->n, g->row_ptr, g->col_idx, vals,
                       x, b, r, w.ctl, w.part, (int)OP_OUTER, outer);
    if (outer == 0) hipLaunchKernelGGL(k_zero_where<S>, dim3(stream_blocks(total)), dim3(kBlock), 0, st, total, x,
                                       w.ctl);
    ENS_LAUNCH_CHECK();
    int32_t act = 0;
    ens_status rc = poll_active(w.ctl, true, st, &act);
    if (rc != ENS_OK) return rc;
    if (act == 0) break;
    hipLaunchKernelGGL((k_cg_start<float, S>), dim3(vb), dim3(kBlock), 0, st, total / VecMap<float, S>::V, r, dinv, p, d,
                       w.ctl, w.part);
    ENS_LAUNCH_CHECK();
    rc = cg_loop<float, S>(g, vals32, d, r, p, q, dinv, w, o.inner_max_iter, o.check_every, st);
    if (rc != ENS_OK) return rc;
    hipLaunchKernelGGL(k_ir_update<S>, dim3(stream_blocks(total)), dim3(kBlock), 0, st, total, x, d, w.ctl);
    ENS_LAUNCH_CHECK();
  }
  return ENS_OK;
}

template <int G>
static ens_status cg_scalar_one(const ens_graph* g, const double* vals, const double* b, double* x,
                                const ens_cg_opts& o, Work& w, hipStream_t st) {
  double* r = (double*)w.vec[0];
  double* p = (double*)w.vec[1];
  double* q = (double*)w.vec[2];
  double* dinv = (double*)w.vec[3];
  const int64_t n = g->n;
  const int rb = row_blocks(n, 256 / G);
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, st, w.ctl, o.rtol, o.inner_rtol, o.max_iter,
                     o.inner_max_iter, o.max_outer, 0);
  hipLaunchKernelGGL((k_diag_inv<double, 1>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g->n, g->row_ptr,
                     g->col_idx, vals, dinv);
  hipLaunchKernelGGL(k_residual_scalar<G>, dim3(rb), dim3(kBlock), 0, st, g->n, g->row_ptr, g->col_idx, vals, x, b,
                     r, w.ctl, w.part, (int)OP_START);
  hipLaunchKernelGGL(k_zero_where<1>, dim3(stream_blocks(n)), dim3(kBlock), 0, st, n, x, w.ctl);
  hipLaunchKernelGGL((k_cg_start<double, 1>), dim3(stream_blocks(n)), dim3(kBlock), 0, st, n, r, dinv, p,
                     (double*)nullptr, w.ctl, w.part);
  ENS_LAUNCH_CHECK();
  const int vb = stream_blocks(n);
  for (int k0 = 0; k0 < o.max_iter; k0 += o.check_every) {
    const int k1 = k0 + o.check_every < o.max_iter ? k0 + o.check_every : o.max_iter;
    for (int k = k0 + 1; k <= k1; ++k) {
      prof_begin(ENS_K_SCALAR_SPMV, st);
      hipLaunchKernelGGL(k_cg_spmv_dot_scalar<G>, dim3(rb), dim3(kBlock), 0, st, g->n, g->row_ptr, g->col_idx,
                         vals, p, q, w.ctl, w.part);
      prof_end(ENS_K_SCALAR_SPMV, st, (double)g->nnz * 12.0 + 4.0 * (n + 1) + 16.0 * n);
      hipLaunchKernelGGL((k_cg_update<double, 1>), dim3(vb), dim3(kBlock), 0, st, n, x, p, q, r, dinv, w.ctl,
                         w.part, k);
      hipLaunchKernelGGL((k_cg_pupdate<double, 1>), dim3(vb), dim3(kBlock), 0, st, n, r, dinv, p, w.ctl);
    }
    ENS_LAUNCH_CHECK();
    int32_t act = 0;
    ens_status rc = poll_active(w.ctl, false, st, &act);
    if (rc != ENS_OK) return rc;
    if (act == 0) break;
  }
  hipLaunchKernelGGL(k_residual_scalar<G>, dim3(rb), dim3(kBlock), 0, st, g->n, g->row_ptr, g->col_idx, vals, x, b,
                     (double*)nullptr, w.ctl, w.part, (int)OP_TRUE);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

ens_status check_graph(const ens_graph* g);

static ens_cg_opts normalized(const ens_cg_opts* in) {
  ens_cg_opts o = *in;
  if (o.max_iter <= 0) o.max_iter = 10000;
  if (o.inner_max_iter <= 0) o.inner_max_iter = 10000;
  if (o.max_outer <= 0) o.max_outer = 10;
  if (o.check_every <= 0) o.check_every = 16;
  if (!(o.inner_rtol > 0.0)) o.inner_rtol = 1e-4;
  return o;
}

}  // namespace ens

using namespace ens;

extern "C" {

ens_status ens_cg_workspace_bytes(const ens_graph* graph, int32_t s, const ens_cg_opts* opts, size_t* bytes) {
  ens_status st = check_graph(graph);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK(opts && bytes, "null argument");
  if (!supported_s(s)) {
    set_error("ensemble size %d not compiled in", s);
    return ENS_E_UNSUPPORTED;
  }
  *bytes = ws_layout(graph->n, s, opts->mixed != 0, nullptr, nullptr);
  return ENS_OK;
}

ens_status ens_cg(const ens_graph* graph, int32_t s, const double* values, const float* values32, const double* b,
                  double* x, const ens_cg_opts* opts, void* workspace, size_t ws_bytes, ens_cg_stat* stats,
                  hipStream_t stream) {
  ens_status st = check_graph(graph);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK(opts && stats, "null options or stats");
  ENS_ARG_CHECK(values && b && x && workspace, "null device pointer");
  ENS_ARG_CHECK(aligned16(values) && aligned16(b) && aligned16(x), "buffers must be 16-byte aligned");
  ENS_ARG_CHECK(((uintptr_t)workspace & 255u) == 0, "workspace must be 256-byte aligned");
  ENS_ARG_CHECK(opts->rtol >= 0.0, "rtol must be >= 0");
  ENS_ARG_CHECK(!opts->mixed || (values32 && aligned16(values32)), "mixed mode needs values32");
  if (!supported_s(s)) {
    set_error("ensemble size %d not compiled in", s);
    return ENS_E_UNSUPPORTED;
  }
  const bool mixed = opts->mixed != 0;
  const size_t need = ws_layout(graph->n, s, mixed, nullptr, nullptr);
  if (ws_bytes < need) {
    set_error("workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    return ENS_E_NOMEM;
  }
  if (graph->n == 0) {
    for (int e = 0; e < s; ++e) stats[e] = ens_cg_stat{0, 0, ENS_SAMPLE_CONVERGED, 0, 0.0};
    return ENS_OK;
  }
  Work w;
  ws_layout(graph->n, s, mixed, &w, (char*)workspace);
  ens_cg_opts o = normalized(opts);
  static_assert(kStreamBlocks <= kMaxPartBlocks, "reduction partial buffer too small");
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, stream, w.ctl, o.rtol, o.inner_rtol, o.max_iter,
                     o.inner_max_iter, o.max_outer, (int)mixed);
  ENS_LAUNCH_CHECK();
  switch (s) {
#define ENS_CG_CASE(SS)                                                                                      \
  case SS:                                                                                                   \
    st = mixed ? cg_mixed<SS>(graph, values, values32, b, x, o, w, stream)                                  \
               : cg_fp64<SS>(graph, values, b, x, o, w, stream);                                            \
    break;
    ENS_CG_CASE(4)
    ENS_CG_CASE(8)
    ENS_CG_CASE(16)
    ENS_CG_CASE(32)
#undef ENS_CG_CASE
  }
  if (st != ENS_OK) return st;
  return read_stats(w.ctl, s, stats, stream);
}

ens_status ens_scalar_cg(const ens_graph* graph, int32_t s, const double* values, const double* b, double* x,
                         const ens_cg_opts* opts, int32_t lanes_per_row, void* workspace, size_t ws_bytes,
                         ens_cg_stat* stats, hipStream_t stream) {
  ens_status st = check_graph(graph);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK(opts && stats && s >= 1, "bad arguments");
  ENS_ARG_CHECK(!opts->mixed, "the scalar baseline is FP64 only");
  ENS_ARG_CHECK(values && b && x && workspace, "null device pointer");
  ENS_ARG_CHECK(((uintptr_t)workspace & 255u) == 0, "workspace must be 256-byte aligned");
  const size_t need = ws_layout(graph->n, 1, false, nullptr, nullptr);
  if (ws_bytes < need) {
    set_error("workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    return ENS_E_NOMEM;
  }
  int G = lanes_per_row > 0 ? lanes_per_row : 8;
  Work w;
  ws_layout(graph->n, 1, false, &w, (char*)workspace);
  ens_cg_opts o = normalized(opts);
  ens_status agg = ENS_OK;
  for (int e = 0; e < s; ++e) {
    const double* ve = values + (int64_t)e * graph->nnz;
    const double* be = b + (int64_t)e * graph->n;
    double* xe = x + (int64_t)e * graph->n;
    switch (G) {
      case 4: st = cg_scalar_one<4>(graph, ve, be, xe, o, w, stream); break;
      case 8: st = cg_scalar_one<8>(graph, ve, be, xe, o, w, stream); break;
      case 16: st = cg_scalar_one<16>(graph, ve, be, xe, o, w, stream); break;
      case 32: st = cg_scalar_one<32>(graph, ve, be, xe, o, w, stream); break;
      default: set_error("lanes_per_row %d not supported", G); return ENS_E_ARG;
    }
    if (st != ENS_OK) return st;
    st = read_stats(w.ctl, 1, &stats[e], stream);
    if (st == ENS_W_NOT_CONVERGED) agg = st;
    else if (st != ENS_OK) return st;
  }
  return agg;
}

}  // extern "C"
