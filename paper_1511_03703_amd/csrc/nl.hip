// Newton's method for the nonlinear problem of Sec. 4 (Eq. diffusion_sys)
// with its Newton systems A d = F (Eq. fenl_lin_sys, A = dF/du) solved by
// restarted GMRES with right preconditioning, all samples of an ensemble at
// once in the commuted layout.
//
// With alpha != 0 the Jacobian is nonsymmetric, so CG no longer applies; the
// ensemble GMRES keeps everything per sample (Hessenberg matrix, Givens
// rotations, residual estimate, restarts and stopping decisions), the
// ensemble analogue of the per-sample CG.  Each Arnoldi step is
//   z = M v_j (Jacobi: D^-1 v_j, fused into the basis scaling; multigrid:
//   the V-cycle of the sample's diffusion operator), w = A z,
//   two classical Gram-Schmidt passes (h = V^T w, w -= V h, twice),
//   |w|, v_{j+1} = w / |w|,
// with every dot product formed as block partials and reduced in a fixed
// order by the library (no atomics, bit-reproducible).  The small per-sample
// work (rotations, back substitution, decisions) runs in one-block kernels on
// the device; the host polls one count per step.
#include <math.h>

#include "cgcore.hpp"
#include "mg.hpp"

namespace ens {

constexpr int kGmMaxRestart = 32;
constexpr int kGmChunk = 8;      // basis vectors per pass of the dot kernel
constexpr int kGmBlocks = 1024;  // grid of the streaming GMRES kernels
constexpr int kGmRed = 256;      // most first-stage blocks of a reduction

enum GmOp { GM_START = 0, GM_H1 = 1, GM_H2 = 2, GM_NORM = 3 };

struct GmCtl {
  double H[kMaxS][kGmMaxRestart + 1][kGmMaxRestart];  // rotated Hessenberg columns (R on and above the diagonal)
  double cs[kMaxS][kGmMaxRestart], sn[kMaxS][kGmMaxRestart];
  double g[kMaxS][kGmMaxRestart + 1];
  double y[kMaxS][kGmMaxRestart];
  double coef[kMaxS][kGmMaxRestart + 1];  // coefficients of the current Gram-Schmidt pass
  double scale[kMaxS];                    // 1/|w| of the next basis vector (0: idle sample)
  double bnorm[kMaxS], tol[kMaxS], rel_res[kMaxS];
  int32_t status[kMaxS], run[kMaxS], cyc[kMaxS], k[kMaxS], iters[kMaxS], cycles[kMaxS], upd[kMaxS], zx[kMaxS];
  int32_t n_run, n_cyc;
  int32_t restart, max_iter;
  double rtol;
};

struct NtCtl {
  double ref[kMaxS], fnorm[kMaxS], rel_res[kMaxS];
  double eta[kMaxS], fprev[kMaxS];  // forcing term of the coming solve; |F| of the last step
  int32_t status[kMaxS], active[kMaxS], iters[kMaxS], lin_iters[kMaxS];
  int32_t n_active;
  int32_t max_newton, forcing;
  double rtol, lin_rtol;
};

// ------------------------------------------------------------ reductions ---

// Sum rows [r0, r1) of a row-major array (row stride `stride`) over its
// first Q columns into dst[q], in an order fixed by (r0, r1, Q).
__device__ inline void sum_block_rows(const double* __restrict__ src, int64_t r0, int64_t r1, int Q, int64_t stride,
                                      double* __restrict__ dst) {
  __shared__ double stripe[kBlock];
  const int t = threadIdx.x;
  if (Q <= kBlock) {
    const int G = kBlock / Q;  // row stripes
    const int q = t % Q, gi = t / Q;
    double a = 0.0;
    if (gi < G)
      for (int64_t r = r0 + gi; r < r1; r += G) a += src[r * stride + q];
    stripe[t] = a;
    __syncthreads();
    if (t < Q) {
      double acc = 0.0;
      for (int k = 0; k < G; ++k) acc += stripe[k * Q + t];
      dst[t] = acc;
    }
    __syncthreads();
  } else {
    for (int q = t; q < Q; q += kBlock) {
      double a = 0.0;
      for (int64_t r = r0; r < r1; ++r) a += src[r * stride + q];
      dst[q] = a;
    }
    __syncthreads();
  }
}

static __global__ __launch_bounds__(kBlock) void k_gm_red1(const double* __restrict__ part, int64_t rows, int Q,
                                                           int64_t stride, double* __restrict__ out) {
  const int64_t r0 = rows * blockIdx.x / gridDim.x, r1 = rows * (blockIdx.x + 1) / gridDim.x;
  sum_block_rows(part, r0, r1, Q, stride, out + (int64_t)blockIdx.x * Q);
}

// ------------------------------------------------------------- finalize ---

template <int S>
__device__ void gm_finalize(GmCtl* c, const double* tot, int op, int arg, const int32_t* mask,
                            const double* rtol_e) {
  const int e = threadIdx.x;
  if (e < S) {
    switch (op) {
      case GM_START: {  // tot: |r|^2 [S], |b|^2 [S]; arg 0 first residual, 1 after a cycle
        if (arg == 0) {
          c->bnorm[e] = sqrt(tot[S + e]);
          c->tol[e] = (rtol_e ? rtol_e[e] : c->rtol) * c->bnorm[e];
          c->iters[e] = 0;
          c->cycles[e] = 0;
          c->zx[e] = 0;
          c->run[e] = mask ? (mask[e] != 0) : 1;
          c->status[e] = c->run[e] ? ENS_SAMPLE_MAXITER : ENS_SAMPLE_CONVERGED;
          c->rel_res[e] = 0.0;
          if (c->run[e] && c->bnorm[e] == 0.0) {
            c->status[e] = ENS_SAMPLE_CONVERGED;
            c->run[e] = 0;
            c->zx[e] = 1;
          }
        } else if (c->run[e]) {
          c->cycles[e] += 1;
        }
        if (c->run[e]) {
          const double beta = sqrt(tot[e]);
          c->rel_res[e] = beta / c->bnorm[e];
          if (!isfinite(beta)) {
            c->status[e] = ENS_SAMPLE_NONFINITE;
            c->run[e] = 0;
          } else if (beta <= c->tol[e]) {
            c->status[e] = ENS_SAMPLE_CONVERGED;
            c->run[e] = 0;
          } else if (c->iters[e] >= c->max_iter) {
            c->status[e] = ENS_SAMPLE_MAXITER;
            c->run[e] = 0;
          } else {
            c->g[e][0] = beta;
            for (int i = 1; i <= kGmMaxRestart; ++i) c->g[e][i] = 0.0;
            c->scale[e] = 1.0 / beta;
          }
        }
        c->cyc[e] = c->run[e];
        c->k[e] = 0;
        c->upd[e] = 0;
        if (!c->run[e]) c->scale[e] = 0.0;
        break;
      }
      case GM_H1:
      case GM_H2: {  // tot[i*S + e] = v_i . w for i <= arg
        const int j = arg;
        for (int i = 0; i <= j; ++i) {
          const double h = c->cyc[e] ? tot[i * S + e] : 0.0;
          c->coef[e][i] = h;
          if (c->cyc[e]) c->H[e][i][j] = (op == GM_H1) ? h : c->H[e][i][j] + h;
        }
        break;
      }
      case GM_NORM: {  // tot[e] = |w|^2 after the second pass; arg = j
        const int j = arg;
        if (c->cyc[e]) {
          const double hn = sqrt(tot[e]);
          double (*H)[kGmMaxRestart] = c->H[e];
          H[j + 1][j] = hn;
          for (int i = 0; i < j; ++i) {
            const double a = H[i][j], b = H[i + 1][j];
            H[i][j] = c->cs[e][i] * a + c->sn[e][i] * b;
            H[i + 1][j] = -c->sn[e][i] * a + c->cs[e][i] * b;
          }
          const double a = H[j][j], b = H[j + 1][j];
          const double den = sqrt(a * a + b * b);
          c->iters[e] += 1;
          c->k[e] = j + 1;
          bool end = false;
          if (!isfinite(den)) {
            c->status[e] = ENS_SAMPLE_NONFINITE;
            c->run[e] = 0;
            end = true;
          } else if (den == 0.0) {
            c->status[e] = ENS_SAMPLE_BREAKDOWN;
            c->run[e] = 0;
            end = true;
          } else {
            c->cs[e][j] = a / den;
            c->sn[e][j] = b / den;
            H[j][j] = den;
            H[j + 1][j] = 0.0;
            c->g[e][j + 1] = -c->sn[e][j] * c->g[e][j];
            c->g[e][j] = c->cs[e][j] * c->g[e][j];
            c->rel_res[e] = fabs(c->g[e][j + 1]) / c->bnorm[e];
            end = fabs(c->g[e][j + 1]) <= c->tol[e] || hn == 0.0 || j + 1 == c->restart ||
                  c->iters[e] >= c->max_iter;
          }
          if (end) {
            c->cyc[e] = 0;
            c->scale[e] = 0.0;
          } else {
            c->scale[e] = 1.0 / hn;
          }
        } else {
          c->scale[e] = 0.0;
        }
        break;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int nr = 0, nc = 0;
    for (int q = 0; q < S; ++q) {
      nr += c->run[q];
      nc += c->cyc[q];
    }
    c->n_run = nr;
    c->n_cyc = nc;
  }
}

template <int S>
static __global__ __launch_bounds__(kBlock) void k_gm_final(const double* __restrict__ part, int64_t rows, int Q,
                                                            int64_t stride, GmCtl* c, int op, int arg,
                                                            const int32_t* __restrict__ mask,
                                                            const double* __restrict__ rtol_e) {
  __shared__ double tot[(kGmMaxRestart + 1) * kMaxS];
  sum_block_rows(part, 0, rows, Q, stride, tot);
  gm_finalize<S>(c, tot, op, arg, mask, rtol_e);
}

static __global__ void k_gm_init(GmCtl* c, double rtol, int restart, int max_iter) {
  if (threadIdx.x == 0) {
    c->rtol = rtol;
    c->restart = restart;
    c->max_iter = max_iter;
    c->n_run = 0;
    c->n_cyc = 0;
  }
}

// End of a cycle: y = R^-1 g over each running sample's k steps (y = 0 for
// the others, so their solution stays as it is).
template <int S>
static __global__ void k_gm_solve(GmCtl* c) {
  const int e = threadIdx.x;
  if (e >= S) return;
  for (int i = 0; i < kGmMaxRestart; ++i) c->y[e][i] = 0.0;
  const int k = c->k[e];
  c->upd[e] = c->run[e] && k > 0;
  if (!c->upd[e]) return;
  for (int i = k - 1; i >= 0; --i) {
    double v = c->g[e][i];
    for (int l = i + 1; l < k; ++l) v -= c->H[e][i][l] * c->y[e][l];
    c->y[e][i] = v / c->H[e][i][i];
  }
}

// End of a cycle when the estimate is trusted: a running sample whose
// Arnoldi residual estimate |g_k| met its tolerance has converged (in exact
// arithmetic the estimate is the true residual of the right-preconditioned
// system); the others go on to the true residual and, if it is needed, a
// further cycle.
template <int S>
static __global__ void k_gm_accept(GmCtl* c) {
  const int e = threadIdx.x;
  if (e < S && c->run[e] && c->k[e] > 0 && fabs(c->g[e][c->k[e]]) <= c->tol[e]) {
    c->status[e] = ENS_SAMPLE_CONVERGED;
    c->run[e] = 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int nr = 0;
    for (int q = 0; q < S; ++q) nr += c->run[q];
    c->n_run = nr;
  }
}

// --------------------------------------------------------- vector kernels ---

// sum_k vals[k] z[col k] for the two samples of lane `sub`, the values (TV)
// and z (TZ) widened to FP64 as they are read; entries in ascending order.
template <int S, typename TV, typename TZ>
__device__ inline typename EnsMap<double, S>::vt gm_row_product(const int32_t* __restrict__ ci,
                                                                const TV* __restrict__ vals,
                                                                const TZ* __restrict__ z, int64_t k0, int64_t k1,
                                                                int sub) {
  using M = EnsMap<double, S>;
  using vt = typename M::vt;
  typedef typename vec_t<TV, M::V>::type at;
  typedef typename vec_t<TZ, M::V>::type zt;
  const at* vv = (const at*)vals + sub;
  const zt* zv = (const zt*)z + sub;
  vt acc = (vt)0.0;
  int64_t k = k0;
  for (; k + 2 < k1; k += 3) {
    int32_t c3[3];
    at a[3];
    zt b[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) c3[j] = ci[k + j];
#pragma unroll
    for (int j = 0; j < 3; ++j) a[j] = load_stream(vv + (k + j) * M::L);
#pragma unroll
    for (int j = 0; j < 3; ++j) b[j] = zv[(int64_t)c3[j] * M::L];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int v = 0; v < M::V; ++v) acc[v] += (double)a[j][v] * (double)b[j][v];
  }
  for (; k < k1; ++k) {
    const at a = load_stream(vv + k * M::L);
    const zt b = zv[(int64_t)ci[k] * M::L];
#pragma unroll
    for (int v = 0; v < M::V; ++v) acc[v] += (double)a[v] * (double)b[v];
  }
  return acc;
}

// w = A z: the matrix in FP64 or FP32 (TV), z in FP64 or, from an FP32
// cycle, FP32 (TZ); products and sums in FP64.
template <int S, typename TV, typename TZ>
static __global__ __launch_bounds__(kBlock) void k_gm_spmv(int n, const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const TV* __restrict__ vals, const TZ* __restrict__ z,
                                                           double* __restrict__ w) {
  using M = EnsMap<double, S>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane % M::L;
  const int64_t row = ((int64_t)blockIdx.x * (kBlock / 64) + wave) * M::RPW + lane / M::L;
  constexpr int R = (kBlock / 64) * M::RPW;
  __shared__ RowTileLds<R> tile;  // the row tile's offsets and indices, as in the CG product
  const bool staged = stage_row_tile(tile, n, rp, ci, (int64_t)blockIdx.x * R);
  if (row >= n) return;
  const int lr = (int)(row - (int64_t)blockIdx.x * R);
  const typename M::vt y = staged
                               ? gm_row_product<S, TV, TZ>(tile.ci - tile.rp[0], vals, z, tile.rp[lr], tile.rp[lr + 1], sub)
                               : gm_row_product<S, TV, TZ>(ci, vals, z, tile.rp[lr], tile.rp[lr + 1], sub);
  store_stream((typename M::vt*)w + row * M::L + sub, y);
}

// One row of the FP32-mapped product: entries k0..k1 of the row, column
// indices from ci (global memory or a staged LDS tile).
template <int S, typename TZ>
__device__ inline typename vec_t<double, 4>::type gm_v32_row(const int32_t* ci, const float* __restrict__ vals,
                                                             const TZ* __restrict__ z, int64_t k0, int64_t k1,
                                                             int sub) {
  using M = EnsMap<float, S>;
  typedef typename vec_t<float, 4>::type f4;
  typedef typename vec_t<TZ, 4>::type z4;
  typedef typename vec_t<double, 4>::type d4;
  const f4* vv = (const f4*)vals + sub;
  const TZ* zs = z + sub * 4;
  d4 acc = (d4)0.0;
  int64_t k = k0;
  for (; k + 2 < k1; k += 3) {
    int32_t c3[3];
    f4 a[3];
    z4 b[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) c3[j] = ci[k + j];
#pragma unroll
    for (int j = 0; j < 3; ++j) a[j] = load_stream(vv + (k + j) * M::L);
#pragma unroll
    for (int j = 0; j < 3; ++j) b[j] = *(const z4*)(zs + (int64_t)c3[j] * S);
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] += (double)a[j][v] * (double)b[j][v];
  }
  for (; k < k1; ++k) {
    const f4 a = load_stream(vv + k * M::L);
    const z4 b = *(const z4*)(zs + (int64_t)ci[k] * S);
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] += (double)a[v] * (double)b[v];
  }
  return acc;
}

// w = A z for an FP32 matrix with the FP32 row mapping: each lane reads 16
// bytes (4 samples) of the value stream, gathers those samples of z (FP64
// or FP32) and accumulates in FP64.
template <int S, typename TZ>
static __global__ __launch_bounds__(kBlock) void k_gm_spmv_v32(int n, const int32_t* __restrict__ rp,
                                                               const int32_t* __restrict__ ci,
                                                               const float* __restrict__ vals,
                                                               const TZ* __restrict__ z, double* __restrict__ w) {
  using M = EnsMap<float, S>;  // V = 4 samples per lane
  typedef typename vec_t<double, 4>::type d4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane % M::L;
  const int64_t row = ((int64_t)blockIdx.x * (kBlock / 64) + wave) * M::RPW + lane / M::L;
  constexpr int R = (kBlock / 64) * M::RPW;
  __shared__ RowTileLds<R> tile;  // the row tile's offsets and indices, as in the CG product
  const bool staged = stage_row_tile(tile, n, rp, ci, (int64_t)blockIdx.x * R);
  if (row >= n) return;
  const int lr = (int)(row - (int64_t)blockIdx.x * R);
  const int64_t k0 = tile.rp[lr], k1 = tile.rp[lr + 1];
  const d4 acc = staged ? gm_v32_row<S, TZ>(tile.ci - tile.rp[0], vals, z, k0, k1, sub)
                        : gm_v32_row<S, TZ>(ci, vals, z, k0, k1, sub);
  store_stream((d4*)(w + row * S + sub * 4), acc);
}

// part[blk][i*S + e] = sum over the block's chunks of V_i . w, i = 0..j.
template <int S>
static __global__ __launch_bounds__(kBlock) void k_gm_dots(int64_t nchunks, const double* __restrict__ V,
                                                           int64_t vstride, int j, const double* __restrict__ w,
                                                           double* __restrict__ part, int64_t pstride) {
  using VM = VecMap<double, S>;
  using vt = typename VM::vt;
  const int64_t step = (int64_t)gridDim.x * kBlock;
  for (int i0 = 0; i0 <= j; i0 += kGmChunk) {
    double acc[kGmChunk][VM::VS];
#pragma unroll
    for (int q = 0; q < kGmChunk; ++q)
#pragma unroll
      for (int v = 0; v < VM::VS; ++v) acc[q][v] = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nchunks; c += step) {
      const vt wv = ((const vt*)w)[c];
#pragma unroll
      for (int q = 0; q < kGmChunk; ++q)
        if (i0 + q <= j) {
          const vt vv = load_stream((const vt*)(V + (int64_t)(i0 + q) * vstride) + c);
#pragma unroll
          for (int v = 0; v < VM::V; ++v) acc[q][v] += vv[v] * wv[v];
        }
    }
    block_partials<S, VM::VS, kGmChunk, kBlock / 64>(acc, part + (int64_t)blockIdx.x * pstride + (int64_t)i0 * S);
    __syncthreads();
  }
}

// w -= sum_{i<=j} coef_i V_i per sample; with NORM the partials |w|^2.
template <int S, bool NORM>
static __global__ __launch_bounds__(kBlock) void k_gm_axpy(int64_t nchunks, const double* __restrict__ V,
                                                           int64_t vstride, int j, const GmCtl* __restrict__ c,
                                                           double* __restrict__ w, double* __restrict__ part,
                                                           int64_t pstride) {
  using VM = VecMap<double, S>;
  using vt = typename VM::vt;
  __shared__ double s_coef[kGmMaxRestart + 1][S];
  for (int t = threadIdx.x; t < (j + 1) * S; t += kBlock) s_coef[t / S][t % S] = c->coef[t % S][t / S];
  __syncthreads();
  const int sub = threadIdx.x % VM::L;
  double acc[1][VM::VS];
#pragma unroll
  for (int v = 0; v < VM::VS; ++v) acc[0][v] = 0.0;
  const int64_t step = (int64_t)gridDim.x * kBlock;
  for (int64_t ch = (int64_t)blockIdx.x * kBlock + threadIdx.x; ch < nchunks; ch += step) {
    vt wv = ((const vt*)w)[ch];
    for (int i = 0; i <= j; ++i) {
      const vt vv = load_stream((const vt*)(V + (int64_t)i * vstride) + ch);
#pragma unroll
      for (int v = 0; v < VM::V; ++v) wv[v] -= s_coef[i][VM::sample(sub, v)] * vv[v];
    }
    ((vt*)w)[ch] = wv;
    if (NORM)
#pragma unroll
      for (int v = 0; v < VM::V; ++v) acc[0][v] += wv[v] * wv[v];
  }
  if (NORM) block_partials<S, VM::VS, 1, kBlock / 64>(acc, part + (int64_t)blockIdx.x * pstride);
}

// Preconditioner forms of the GMRES kernels.
enum GmPrec { PR_MG64 = 0, PR_JACOBI = 1, PR_MG32 = 2 };

// The first pass's update w -= sum_{i<=j} coef_i V_i fused with the second
// pass's partials V_i . w on the updated w (j < JM): each V_i chunk is read
// once and kept in registers for both uses.
template <int S, int JM>
static __global__ __launch_bounds__(kBlock) void k_gm_axpy_dots(int64_t nchunks, const double* __restrict__ V,
                                                                int64_t vstride, int j, const GmCtl* __restrict__ c,
                                                                double* __restrict__ w, double* __restrict__ part,
                                                                int64_t pstride) {
  using VM = VecMap<double, S>;
  using vt = typename VM::vt;
  static_assert(JM % kGmChunk == 0, "JM must be a multiple of the partial chunk");
  __shared__ double s_coef[JM][S];
  for (int t = threadIdx.x; t < JM * S; t += kBlock) s_coef[t / S][t % S] = t / S <= j ? c->coef[t % S][t / S] : 0.0;
  __syncthreads();
  const int sub = threadIdx.x % VM::L;
  double acc[JM][VM::VS];
#pragma unroll
  for (int i = 0; i < JM; ++i)
#pragma unroll
    for (int v = 0; v < VM::VS; ++v) acc[i][v] = 0.0;
  const int64_t step = (int64_t)gridDim.x * kBlock;
  for (int64_t ch = (int64_t)blockIdx.x * kBlock + threadIdx.x; ch < nchunks; ch += step) {
    vt wv = ((const vt*)w)[ch];
    vt vv[JM];
#pragma unroll
    for (int i = 0; i < JM; ++i)
      if (i <= j) {
        vv[i] = load_stream((const vt*)(V + (int64_t)i * vstride) + ch);
#pragma unroll
        for (int v = 0; v < VM::V; ++v) wv[v] -= s_coef[i][VM::sample(sub, v)] * vv[i][v];
      }
    ((vt*)w)[ch] = wv;
#pragma unroll
    for (int i = 0; i < JM; ++i)
      if (i <= j)
#pragma unroll
        for (int v = 0; v < VM::V; ++v) acc[i][v] += vv[i][v] * wv[v];
  }
#pragma unroll
  for (int g = 0; g < JM / kGmChunk; ++g) {
    block_partials<S, VM::VS, kGmChunk, kBlock / 64>(
        *reinterpret_cast<double(*)[kGmChunk][VM::VS]>(&acc[g * kGmChunk][0]),
        part + (int64_t)blockIdx.x * pstride + (int64_t)g * kGmChunk * S);
    __syncthreads();
  }
}

// vout = w * scale (exact zeros for idle samples); then the input of the
// preconditioner: Jacobi z = D^-1 vout, FP32 cycle r32 = (float) vout.
template <int S, int PR>
static __global__ __launch_bounds__(kBlock) void k_gm_scale(int64_t nchunks, const double* __restrict__ w,
                                                            const GmCtl* __restrict__ c, double* __restrict__ vout,
                                                            const double* __restrict__ dinv,
                                                            double* __restrict__ z, float* __restrict__ r32) {
  using VM = VecMap<double, S>;
  using vt = typename VM::vt;
  typedef typename vec_t<float, VM::V>::type ft;
  const int64_t ch = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (ch >= nchunks) return;
  const int sub = threadIdx.x % VM::L;
  const vt wv = ((const vt*)w)[ch];
  vt v;
#pragma unroll
  for (int k = 0; k < VM::V; ++k) {
    const double sc = c->scale[VM::sample(sub, k)];
    v[k] = sc == 0.0 ? 0.0 : wv[k] * sc;
  }
  ((vt*)vout)[ch] = v;
  if (PR == PR_JACOBI) ((vt*)z)[ch] = ((const vt*)dinv)[ch] * v;
  if (PR == PR_MG32) {
    ft f;
#pragma unroll
    for (int k = 0; k < VM::V; ++k) f[k] = (float)v[k];
    ((ft*)r32)[ch] = f;
  }
}

// t = sum_{i<k} y_i V_i per sample.
template <int S>
static __global__ __launch_bounds__(kBlock) void k_gm_combine(int64_t nchunks, const double* __restrict__ V,
                                                              int64_t vstride, int k, const GmCtl* __restrict__ c,
                                                              double* __restrict__ t) {
  using VM = VecMap<double, S>;
  using vt = typename VM::vt;
  __shared__ double s_y[kGmMaxRestart][S];
  for (int q = threadIdx.x; q < k * S; q += kBlock) s_y[q / S][q % S] = c->y[q % S][q / S];
  __syncthreads();
  const int64_t ch = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (ch >= nchunks) return;
  const int sub = threadIdx.x % VM::L;
  vt acc = (vt)0.0;
  for (int i = 0; i < k; ++i) {
    const vt vv = load_stream((const vt*)(V + (int64_t)i * vstride) + ch);
#pragma unroll
    for (int v = 0; v < VM::V; ++v) acc[v] += s_y[i][VM::sample(sub, v)] * vv[v];
  }
  ((vt*)t)[ch] = acc;
}

// Jacobi end of a cycle: x += D^-1 t for the samples updated in it.
template <int S>
static __global__ __launch_bounds__(kBlock) void k_gm_addto(int64_t nchunks, const double* __restrict__ t,
                                                            const double* __restrict__ dinv,
                                                            const GmCtl* __restrict__ c, double* __restrict__ x) {
  using VM = VecMap<double, S>;
  using vt = typename VM::vt;
  const int64_t ch = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (ch >= nchunks) return;
  const int sub = threadIdx.x % VM::L;
  const vt tv = ((const vt*)dinv)[ch] * ((const vt*)t)[ch];
  vt xv = ((const vt*)x)[ch];
#pragma unroll
  for (int v = 0; v < VM::V; ++v)
    if (c->upd[VM::sample(sub, v)]) xv[v] += tv[v];
  ((vt*)x)[ch] = xv;
}

// Multigrid end of a cycle: x += sum_{i<k} y_i z_i for the samples updated
// in it, z_i = M v_i kept from the cycle's steps in the cycle's precision
// TZ.  With a fixed preconditioner M (V y) is that same sum, so the cycle
// ends without a further application of M.  A sample's y is zero beyond
// its own steps, where its basis vectors, and so its z, are zero.
template <int S, typename TZ>
static __global__ __launch_bounds__(kBlock) void k_gm_zupdate(int64_t nchunks, const TZ* __restrict__ Z,
                                                              int64_t zstride, int k, const GmCtl* __restrict__ c,
                                                              double* __restrict__ x) {
  using VM = VecMap<double, S>;
  using vt = typename VM::vt;
  typedef typename vec_t<TZ, VM::V>::type zt;
  __shared__ double s_y[kGmMaxRestart][S];
  for (int q = threadIdx.x; q < k * S; q += kBlock) s_y[q / S][q % S] = c->y[q % S][q / S];
  __syncthreads();
  const int64_t ch = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (ch >= nchunks) return;
  const int sub = threadIdx.x % VM::L;
  vt acc = (vt)0.0;
  for (int i = 0; i < k; ++i) {
    const zt zv = ((const zt*)(Z + (int64_t)i * zstride))[ch];
#pragma unroll
    for (int v = 0; v < VM::V; ++v) acc[v] += s_y[i][VM::sample(sub, v)] * (double)zv[v];
  }
  vt xv = ((const vt*)x)[ch];
#pragma unroll
  for (int v = 0; v < VM::V; ++v)
    if (c->upd[VM::sample(sub, v)]) xv[v] += acc[v];
  ((vt*)x)[ch] = xv;
}

// x = 0 for samples whose right-hand side is zero.
template <int S>
static __global__ __launch_bounds__(kBlock) void k_gm_zero_x(int64_t total, const GmCtl* __restrict__ c,
                                                             double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < total && c->zx[i % S]) x[i] = 0.0;
}

// r = b - A x (matrix in FP64 or FP32, widened) for the row tile, with the
// block's partials |r|^2 and |b|^2.
template <int S, typename TV, bool XZ = false>
static __global__ __launch_bounds__(kBlock) void k_gm_residual(int n, const int32_t* __restrict__ rp,
                                                               const int32_t* __restrict__ ci,
                                                               const TV* __restrict__ vals,
                                                               const double* __restrict__ x,
                                                               const double* __restrict__ b, double* __restrict__ r,
                                                               double* __restrict__ part) {
  using M = EnsMap<double, S>;
  using vt = typename M::vt;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane % M::L;
  double acc[2][M::V];
#pragma unroll
  for (int v = 0; v < M::V; ++v) acc[0][v] = acc[1][v] = 0.0;
  const int64_t row = ((int64_t)blockIdx.x * (kBlock / 64) + wave) * M::RPW + lane / M::L;
  if (row < n) {
    // XZ: x = 0 is known, so r = b without the product
    const vt ax = XZ ? (vt)0.0 : gm_row_product<S, TV, double>(ci, vals, x, rp[row], rp[row + 1], sub);
    const vt bv = ((const vt*)b)[row * M::L + sub];
    const vt rv = bv - ax;
    ((vt*)r)[row * M::L + sub] = rv;
#pragma unroll
    for (int v = 0; v < M::V; ++v) {
      acc[0][v] = rv[v] * rv[v];
      acc[1][v] = bv[v] * bv[v];
    }
  }
  block_partials<S, M::V, 2, kBlock / 64>(acc, part + (int64_t)blockIdx.x * 2 * S);
}

// dinv[i][e] = 1 / A_ii[e] in FP64 (the diagonal widened from TV).
template <int S, typename TV>
static __global__ __launch_bounds__(kBlock) void k_gm_dinv(int n, const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const TV* __restrict__ vals, double* __restrict__ dinv) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t row = t / S;
  const int e = (int)(t % S);
  if (row >= n) return;
  double d = 0.0;
  for (int64_t k = rp[row]; k < rp[row + 1]; ++k)
    if (ci[k] == row) d = (double)vals[k * S + e];
  dinv[row * S + e] = 1.0 / d;
}

// ------------------------------------------------------------ host side ---

static size_t r256(size_t b) { return (b + 255) & ~(size_t)255; }

static int64_t gm_pstride(int S, int restart) {
  const int cols = ((restart + kGmChunk - 1) / kGmChunk) * kGmChunk;
  return (int64_t)(cols < 2 ? 2 : cols) * S;
}

static int64_t row_blocks(int64_t n, int S) {
  const int64_t rpb = (kBlock / 64) * (64 / (S / 2));  // FP64 rows per block
  return (n + rpb - 1) / rpb;
}

struct GmWork {
  GmCtl* ctl;
  double *part, *part1, *rpart;
  double *V, *w, *z, *t, *dinv;
  float* r32;  // input of an FP32 cycle
  void* Z;     // z_j = M v_j of a cycle's steps: restart vectors, FP64 or (FP32 cycle) FP32
  int64_t pstride;
};

static size_t gm_layout(int64_t n, int S, int restart, GmWork* w, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += r256(bytes);
    return p;
  };
  const int64_t ps = gm_pstride(S, restart);
  GmCtl* ctl = (GmCtl*)take(sizeof(GmCtl));
  double* part = (double*)take((size_t)kGmBlocks * ps * sizeof(double));
  double* part1 = (double*)take((size_t)kGmRed * (ps > 2 * S ? ps : 2 * S) * sizeof(double));
  double* rpart = (double*)take((size_t)row_blocks(n, S) * 2 * S * sizeof(double));
  const size_t vb = (size_t)n * S * sizeof(double);
  double* V = (double*)take(vb * (size_t)(restart + 1));
  double* wv = (double*)take(vb);
  double* z = (double*)take(vb);
  double* t = (double*)take(vb);
  double* dinv = (double*)take(vb);
  float* r32 = (float*)take(vb / 2);
  void* Z = take(vb * (size_t)restart);
  if (w) *w = GmWork{ctl, part, part1, rpart, V, wv, z, t, dinv, r32, Z, ps};
  return off;
}

static unsigned grid_of(int64_t items, int64_t per) {
  const int64_t b = (items + per - 1) / per;
  return (unsigned)(b < 1 ? 1 : b);
}

static unsigned stream_grid(int64_t nchunks) {
  const int64_t b = (nchunks + kBlock - 1) / kBlock;
  return (unsigned)(b < 1 ? 1 : (b > kGmBlocks ? kGmBlocks : b));
}

// Reduce `rows` partial rows (Q columns, row stride `stride`) and run the
// finalize step.
template <int S>
static void gm_reduce(const GmWork& w, const double* part, int64_t rows, int Q, int64_t stride, int op, int arg,
                      const int32_t* mask, const double* rtol_e, hipStream_t st) {
  if (rows <= 64) {
    hipLaunchKernelGGL((k_gm_final<S>), dim3(1), dim3(kBlock), 0, st, part, rows, Q, stride, w.ctl, op, arg, mask,
                       rtol_e);
    return;
  }
  int64_t r = rows / 16;
  if (r > kGmRed) r = kGmRed;
  hipLaunchKernelGGL(k_gm_red1, dim3((unsigned)r), dim3(kBlock), 0, st, part, rows, Q, stride, w.part1);
  hipLaunchKernelGGL((k_gm_final<S>), dim3(1), dim3(kBlock), 0, st, w.part1, r, Q, (int64_t)Q, w.ctl, op, arg,
                     mask, rtol_e);
}

static ens_status read_flag(const int32_t* dev, hipStream_t st, int32_t* out) {
  DeviceCtx* cx = device_ctx();
  if (!cx) {
    set_error("device context unavailable");
    return ENS_E_HIP;
  }
  ENS_HIP_TRY(hipMemcpyAsync(cx->host_flag, dev, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  ENS_HIP_TRY(hipStreamSynchronize(st));
  prof_collect();
  *out = *cx->host_flag;
  return ENS_OK;
}

// GMRES on (graph, vals) for all samples; x in/out.  plan != nullptr:
// multigrid preconditioner, else Jacobi.  mask (device, nullable): samples
// that take part.
template <int S, typename TV>
static ens_status gmres(const ens_graph* g, const TV* vals, const double* b, double* x, double rtol, int restart,
                        int max_iter, const MgPlan* plan, const GmWork& w, const int32_t* mask,
                        const double* rtol_e, hipStream_t st, bool x_zero = false, bool trust = false) {
  const int n = g->n;
  const int64_t nchunks = (int64_t)n * S / VecMap<double, S>::V;
  const int64_t vstride = (int64_t)n * S;
  const unsigned sg = stream_grid(nchunks), eg = grid_of(nchunks, kBlock);
  const unsigned rb = (unsigned)row_blocks(n, S);
  const unsigned sb = grid_of(n, (kBlock / 64) * EnsMap<double, S>::RPW);
  const bool jac = plan == nullptr;
  const bool f32 = plan != nullptr && plan->fp32;
  const double spmv_bytes = (double)g->nnz * (S * (double)sizeof(TV) + 4.0) + 4.0 * (n + 1) + 2.0 * n * S * 8.0;
  const double vbytes = (double)n * S * 8.0;
  hipLaunchKernelGGL(k_gm_init, dim3(1), dim3(64), 0, st, w.ctl, rtol, restart, max_iter);
  if (jac) hipLaunchKernelGGL((k_gm_dinv<S, TV>), dim3(grid_of((int64_t)n * S, kBlock)), dim3(kBlock), 0, st, n,
                              g->row_ptr, g->col_idx, vals, w.dinv);
  if (x_zero)
    hipLaunchKernelGGL((k_gm_residual<S, TV, true>), dim3(rb), dim3(kBlock), 0, st, n, g->row_ptr, g->col_idx, vals,
                       x, b, w.w, w.rpart);
  else
    hipLaunchKernelGGL((k_gm_residual<S, TV>), dim3(rb), dim3(kBlock), 0, st, n, g->row_ptr, g->col_idx, vals, x, b,
                       w.w, w.rpart);
  gm_reduce<S>(w, w.rpart, rb, 2 * S, 2 * S, GM_START, 0, mask, rtol_e, st);
  hipLaunchKernelGGL((k_gm_zero_x<S>), dim3(grid_of((int64_t)n * S, kBlock)), dim3(kBlock), 0, st, (int64_t)n * S,
                     w.ctl, x);
  ENS_LAUNCH_CHECK();
  for (;;) {
    int32_t nrun = 0;
    ens_status rc = read_flag(&w.ctl->n_run, st, &nrun);
    if (rc != ENS_OK) return rc;
    if (nrun == 0) break;
    auto scale = [&](double* vout) {
      if (jac)
        hipLaunchKernelGGL((k_gm_scale<S, PR_JACOBI>), dim3(eg), dim3(kBlock), 0, st, nchunks, w.w, w.ctl, vout,
                           w.dinv, w.z, (float*)nullptr);
      else if (f32)
        hipLaunchKernelGGL((k_gm_scale<S, PR_MG32>), dim3(eg), dim3(kBlock), 0, st, nchunks, w.w, w.ctl, vout,
                           (const double*)nullptr, (double*)nullptr, w.r32);
      else
        hipLaunchKernelGGL((k_gm_scale<S, PR_MG64>), dim3(eg), dim3(kBlock), 0, st, nchunks, w.w, w.ctl, vout,
                           (const double*)nullptr, (double*)nullptr, (float*)nullptr);
    };
    scale(w.V);
    int steps = 0;
    for (int j = 0; j < restart; ++j) {
      double* vj = w.V + (int64_t)j * vstride;
      float* zj32 = (float*)w.Z + (int64_t)j * vstride;
      double* zj = jac ? w.z : (double*)w.Z + (int64_t)j * vstride;
      if (f32) mg_vcycle<float, S>(*plan, w.r32, zj32, nullptr, st);
      else if (!jac) mg_vcycle<double, S>(*plan, vj, zj, nullptr, st);
      prof_begin(ENS_K_GM_SPMV, st);
      if (sizeof(TV) == 4) {
        const unsigned sb32 = grid_of(n, (kBlock / 64) * EnsMap<float, S>::RPW);
        if (f32)
          hipLaunchKernelGGL((k_gm_spmv_v32<S, float>), dim3(sb32), dim3(kBlock), 0, st, n, g->row_ptr, g->col_idx,
                             (const float*)vals, (const float*)zj32, w.w);
        else
          hipLaunchKernelGGL((k_gm_spmv_v32<S, double>), dim3(sb32), dim3(kBlock), 0, st, n, g->row_ptr,
                             g->col_idx, (const float*)vals, (const double*)zj, w.w);
      } else {
        if (f32)
          hipLaunchKernelGGL((k_gm_spmv<S, TV, float>), dim3(sb), dim3(kBlock), 0, st, n, g->row_ptr, g->col_idx,
                             vals, (const float*)zj32, w.w);
        else
          hipLaunchKernelGGL((k_gm_spmv<S, TV, double>), dim3(sb), dim3(kBlock), 0, st, n, g->row_ptr, g->col_idx,
                             vals, (const double*)zj, w.w);
      }
      prof_end(ENS_K_GM_SPMV, st, spmv_bytes - (f32 ? 4.0 * n * S : 0.0));
      // classical Gram-Schmidt twice: h1 = V^T w, w -= V h1, h2 = V^T w,
      // w -= V h2 and |w|^2; for j < 16 the middle two passes are one kernel
      auto dots = [&]() {
        prof_begin(ENS_K_GM_ORTH, st);
        hipLaunchKernelGGL((k_gm_dots<S>), dim3(sg), dim3(kBlock), 0, st, nchunks, w.V, vstride, j, w.w, w.part,
                           w.pstride);
        prof_end(ENS_K_GM_ORTH, st, vbytes * (j + 1 + (j + kGmChunk) / kGmChunk));
      };
      dots();
      gm_reduce<S>(w, w.part, sg, (j + 1) * S, w.pstride, GM_H1, j, mask, rtol_e, st);
      prof_begin(ENS_K_GM_ORTH, st);
      if (j < 8)
        hipLaunchKernelGGL((k_gm_axpy_dots<S, 8>), dim3(sg), dim3(kBlock), 0, st, nchunks, w.V, vstride, j, w.ctl,
                           w.w, w.part, w.pstride);
      else if (j < 16)
        hipLaunchKernelGGL((k_gm_axpy_dots<S, 16>), dim3(sg), dim3(kBlock), 0, st, nchunks, w.V, vstride, j, w.ctl,
                           w.w, w.part, w.pstride);
      else
        hipLaunchKernelGGL((k_gm_axpy<S, false>), dim3(sg), dim3(kBlock), 0, st, nchunks, w.V, vstride, j, w.ctl,
                           w.w, w.part, w.pstride);
      prof_end(ENS_K_GM_ORTH, st, vbytes * (j + 3));
      if (j >= 16) dots();
      gm_reduce<S>(w, w.part, sg, (j + 1) * S, w.pstride, GM_H2, j, mask, rtol_e, st);
      prof_begin(ENS_K_GM_ORTH, st);
      hipLaunchKernelGGL((k_gm_axpy<S, true>), dim3(sg), dim3(kBlock), 0, st, nchunks, w.V, vstride, j, w.ctl, w.w,
                         w.part, w.pstride);
      prof_end(ENS_K_GM_ORTH, st, vbytes * (j + 3));
      gm_reduce<S>(w, w.part, sg, S, w.pstride, GM_NORM, j, mask, rtol_e, st);
      ENS_LAUNCH_CHECK();
      steps = j + 1;
      int32_t ncyc = 0;
      rc = read_flag(&w.ctl->n_cyc, st, &ncyc);
      if (rc != ENS_OK) return rc;
      if (ncyc == 0) break;
      scale(w.V + (int64_t)(j + 1) * vstride);
    }
    hipLaunchKernelGGL((k_gm_solve<S>), dim3(1), dim3(64), 0, st, w.ctl);
    if (jac) {
      hipLaunchKernelGGL((k_gm_combine<S>), dim3(eg), dim3(kBlock), 0, st, nchunks, w.V, vstride, steps, w.ctl, w.t);
      hipLaunchKernelGGL((k_gm_addto<S>), dim3(eg), dim3(kBlock), 0, st, nchunks, w.t, w.dinv, w.ctl, x);
    } else if (f32) {
      hipLaunchKernelGGL((k_gm_zupdate<S, float>), dim3(eg), dim3(kBlock), 0, st, nchunks, (const float*)w.Z,
                         vstride, steps, w.ctl, x);
    } else {
      hipLaunchKernelGGL((k_gm_zupdate<S, double>), dim3(eg), dim3(kBlock), 0, st, nchunks, (const double*)w.Z,
                         vstride, steps, w.ctl, x);
    }
    if (trust) {
      // samples whose estimate met the tolerance stop here; the true
      // residual is formed only if a further cycle is needed
      hipLaunchKernelGGL((k_gm_accept<S>), dim3(1), dim3(64), 0, st, w.ctl);
      ENS_LAUNCH_CHECK();
      int32_t nleft = 0;
      rc = read_flag(&w.ctl->n_run, st, &nleft);
      if (rc != ENS_OK) return rc;
      if (nleft == 0) break;
    }
    hipLaunchKernelGGL((k_gm_residual<S, TV>), dim3(rb), dim3(kBlock), 0, st, n, g->row_ptr, g->col_idx, vals, x, b,
                       w.w, w.rpart);
    gm_reduce<S>(w, w.rpart, rb, 2 * S, 2 * S, GM_START, 1, mask, rtol_e, st);
    ENS_LAUNCH_CHECK();
  }
  return ENS_OK;
}

// ----------------------------------------------------------------- Newton ---

// F norms (and, at the first step, load norms) of chunk blocks: partials
// |F|^2 and |load|^2.
template <int S>
static __global__ __launch_bounds__(kBlock) void k_nt_norms(int64_t nchunks, const double* __restrict__ F,
                                                            const double* __restrict__ load,
                                                            double* __restrict__ part, int64_t pstride) {
  using VM = VecMap<double, S>;
  using vt = typename VM::vt;
  double acc[2][VM::VS];
#pragma unroll
  for (int v = 0; v < VM::VS; ++v) acc[0][v] = acc[1][v] = 0.0;
  const int64_t step = (int64_t)gridDim.x * kBlock;
  for (int64_t ch = (int64_t)blockIdx.x * kBlock + threadIdx.x; ch < nchunks; ch += step) {
    const vt f = ((const vt*)F)[ch];
    const vt l = load ? ((const vt*)load)[ch] : (vt)0.0;
#pragma unroll
    for (int v = 0; v < VM::V; ++v) {
      acc[0][v] += f[v] * f[v];
      acc[1][v] += l[v] * l[v];
    }
  }
  block_partials<S, VM::VS, 2, kBlock / 64>(acc, part + (int64_t)blockIdx.x * pstride);
}

// Newton decisions after the residual of step k: tot = |F|^2 [S], |load|^2 [S].
template <int S>
static __global__ __launch_bounds__(kBlock) void k_nt_final(const double* __restrict__ part, int64_t rows,
                                                            int64_t stride, NtCtl* c, int k) {
  __shared__ double tot[2 * kMaxS];
  sum_block_rows(part, 0, rows, 2 * S, stride, tot);
  const int e = threadIdx.x;
  if (e < S) {
    const double fn = sqrt(tot[e]);
    if (k == 0) {
      double ref = sqrt(tot[S + e]);
      if (ref == 0.0) ref = fn;
      c->ref[e] = ref;
      c->active[e] = 1;
      c->status[e] = ENS_SAMPLE_MAXITER;
      c->iters[e] = 0;
      c->lin_iters[e] = 0;
    }
    c->fnorm[e] = fn;
    c->rel_res[e] = c->ref[e] > 0.0 ? fn / c->ref[e] : 0.0;
    if (c->active[e]) {
      if (!isfinite(fn)) {
        c->status[e] = ENS_SAMPLE_NONFINITE;
        c->active[e] = 0;
      } else if (fn <= c->rtol * c->ref[e]) {
        c->status[e] = ENS_SAMPLE_CONVERGED;
        c->active[e] = 0;
      } else if (k == c->max_newton) {
        c->status[e] = ENS_SAMPLE_MAXITER;
        c->active[e] = 0;
      }
    }
    if (c->active[e]) {
      // forcing term of this step's linear solve: fixed, or the second
      // choice of Eisenstat and Walker (gamma 0.9, exponent 2, safeguard
      // gamma eta^2 above 0.1, eta_0 = eta_max = lin_rtol, and no tighter
      // than 0.5 rtol ref / |F|)
      double eta = c->lin_rtol;
      if (c->forcing == 1 && k > 0) {
        const double gamma = 0.9;
        eta = gamma * (fn / c->fprev[e]) * (fn / c->fprev[e]);
        const double safe = gamma * c->eta[e] * c->eta[e];
        if (safe > 0.1 && safe > eta) eta = safe;
        if (eta > c->lin_rtol) eta = c->lin_rtol;
        const double floor_tol = 0.5 * c->rtol * c->ref[e] / fn;
        if (eta < floor_tol) eta = floor_tol;
      }
      c->eta[e] = eta;
      c->fprev[e] = fn;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int na = 0;
    for (int q = 0; q < S; ++q) na += c->active[q];
    c->n_active = na;
  }
}

// After the linear solve: count its iterations, stop samples whose solve
// failed, and count the Newton step of the others.
template <int S>
static __global__ void k_nt_after(NtCtl* c, const GmCtl* g) {
  const int e = threadIdx.x;
  if (e >= S || !c->active[e]) return;
  c->lin_iters[e] += g->iters[e];
  if (g->status[e] == ENS_SAMPLE_NONFINITE || g->status[e] == ENS_SAMPLE_BREAKDOWN) {
    c->status[e] = g->status[e];
    c->active[e] = 0;
  } else {
    c->iters[e] += 1;
  }
}

// u -= d for the samples that took the step.
template <int S>
static __global__ __launch_bounds__(kBlock) void k_nt_update(int64_t total, const NtCtl* __restrict__ c,
                                                             const double* __restrict__ d, double* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < total && c->active[i % S]) u[i] -= d[i];
}

static __global__ void k_nt_init(NtCtl* c, double rtol, int max_newton, int forcing, double lin_rtol) {
  if (threadIdx.x == 0) {
    c->rtol = rtol;
    c->max_newton = max_newton;
    c->forcing = forcing;
    c->lin_rtol = lin_rtol;
    c->n_active = 0;
  }
  if (threadIdx.x < kMaxS) {
    c->active[threadIdx.x] = 0;
    c->eta[threadIdx.x] = lin_rtol;
    c->fprev[threadIdx.x] = 0.0;
  }
}

static __global__ void k_fill_zero64(int64_t total, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < total) x[i] = 0.0;
}

struct NtWork {
  NtCtl* ctl;
  void* J;  // Jacobian values, FP64 or (jac32) FP32
  double *F, *load, *d, *npart;
  GmWork gm;
};

static size_t nt_layout(int64_t n, int64_t nnz, int S, int restart, bool jac32, NtWork* w, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += r256(bytes);
    return p;
  };
  NtCtl* ctl = (NtCtl*)take(sizeof(NtCtl));
  void* J = take((size_t)nnz * S * (jac32 ? sizeof(float) : sizeof(double)));
  const size_t vb = (size_t)n * S * sizeof(double);
  double* F = (double*)take(vb);
  double* load = (double*)take(vb);
  double* d = (double*)take(vb);
  double* npart = (double*)take((size_t)kGmBlocks * 2 * S * sizeof(double));
  GmWork gm;
  const size_t g = gm_layout(n, S, restart, w ? &gm : nullptr, base ? base + off : nullptr);
  off += g;
  if (w) *w = NtWork{ctl, J, F, load, d, npart, gm};
  return off;
}

template <int S>
static ens_status newton(int N, const ens_graph* g, const void* kl, const ens_nl_problem* prob, const double* xi,
                         double* u, const ens_newton_opts& o, const MgPlan* plan, NtWork& w, hipStream_t st) {
  const int64_t n = g->n;
  const int64_t total = n * S;
  const int64_t nchunks = total / VecMap<double, S>::V;
  const unsigned sg = stream_grid(nchunks);
  hipLaunchKernelGGL(k_nt_init, dim3(1), dim3(64), 0, st, w.ctl, o.rtol, o.max_newton, o.forcing, o.lin_rtol);
  ENS_LAUNCH_CHECK();
  for (int k = 0;; ++k) {
    ens_status rc = ens_nl_assemble(N, g, kl, prob, S, xi, u, o.jac32 ? nullptr : (double*)w.J,
                                    o.jac32 ? (float*)w.J : nullptr, w.F, k == 0 ? w.load : nullptr, st);
    if (rc != ENS_OK) return rc;
    hipLaunchKernelGGL((k_nt_norms<S>), dim3(sg), dim3(kBlock), 0, st, nchunks, w.F,
                       k == 0 ? (const double*)w.load : (const double*)nullptr, w.npart, (int64_t)2 * S);
    hipLaunchKernelGGL((k_nt_final<S>), dim3(1), dim3(kBlock), 0, st, w.npart, (int64_t)sg, (int64_t)2 * S, w.ctl,
                       k);
    ENS_LAUNCH_CHECK();
    int32_t na = 0;
    rc = read_flag(&w.ctl->n_active, st, &na);
    if (rc != ENS_OK) return rc;
    if (na == 0) break;
    hipLaunchKernelGGL(k_fill_zero64, dim3(grid_of(total, kBlock)), dim3(kBlock), 0, st, total, w.d);
    if (o.jac32)
      rc = gmres<S, float>(g, (const float*)w.J, w.F, w.d, o.lin_rtol, o.restart, o.lin_max_iter, plan, w.gm,
                           w.ctl->active, w.ctl->eta, st, true, true);
    else
      rc = gmres<S, double>(g, (const double*)w.J, w.F, w.d, o.lin_rtol, o.restart, o.lin_max_iter, plan, w.gm,
                            w.ctl->active, w.ctl->eta, st, true, true);
    if (rc != ENS_OK) return rc;
    hipLaunchKernelGGL((k_nt_after<S>), dim3(1), dim3(64), 0, st, w.ctl, (const GmCtl*)w.gm.ctl);
    hipLaunchKernelGGL((k_nt_update<S>), dim3(grid_of(total, kBlock)), dim3(kBlock), 0, st, total, w.ctl, w.d, u);
    ENS_LAUNCH_CHECK();
  }
  return ENS_OK;
}

}  // namespace ens

using namespace ens;

namespace {

ens_status check_graph_nl(const ens_graph* g) {
  ENS_ARG_CHECK(g && g->row_ptr && g->col_idx && g->n > 0 && g->nnz > 0, "bad graph");
  return ENS_OK;
}

// The multigrid plan of a set-up hierarchy, attached to the fine matrix its
// cycle runs on (mg_values: FP64 for an FP64 hierarchy, FP32 for an FP32
// one).
ens_status mg_plan_for(const ens_mg* mg, const ens_graph* graph, int32_t s, const void* mg_values, MgPlan* plan) {
  ENS_ARG_CHECK(mg->buffer && mg_values && aligned16(mg_values), "multigrid needs its buffer and fine matrix");
  ENS_ARG_CHECK(mg->s == s, "hierarchy built for another ensemble size");
  const int64_t nn = (int64_t)(mg->N + 1) * (mg->N + 1) * (mg->N + 1);
  ENS_ARG_CHECK(graph->n == nn, "graph is not the hierarchy's fine mesh");
  if (mg_stage(mg) < 2) {
    set_error("multigrid hierarchy not set up: call ens_mg_build and ens_mg_setup first");
    return ENS_E_ARG;
  }
  if (!mg_plan(mg->N, mg->M, s, mg->fp32 != 0, (char*)mg->buffer, plan)) {
    set_error("multigrid hierarchy of N=%d is not supported", mg->N);
    return ENS_E_UNSUPPORTED;
  }
  if (mg->bytes < plan->bytes) {
    set_error("multigrid buffer of %zu bytes is smaller than the %zu required", mg->bytes, plan->bytes);
    return ENS_E_NOMEM;
  }
  if (mg->fp32) mg_attach_fine(plan, graph->row_ptr, graph->col_idx, nullptr, (const float*)mg_values);
  else mg_attach_fine(plan, graph->row_ptr, graph->col_idx, (const double*)mg_values, nullptr);
  return ENS_OK;
}

}  // namespace

extern "C" {

ens_status ens_gmres_workspace_bytes(const ens_graph* graph, int32_t s, int32_t restart, size_t* bytes) {
  ens_status st = check_graph_nl(graph);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK(bytes, "null output");
  ENS_ARG_CHECK(restart >= 1 && restart <= kGmMaxRestart, "restart must be in 1..32");
  if (!supported_s(s)) {
    set_error("ensemble size %d not compiled in", s);
    return ENS_E_UNSUPPORTED;
  }
  *bytes = gm_layout(graph->n, s, restart, nullptr, nullptr);
  return ENS_OK;
}

ens_status ens_gmres(const ens_graph* graph, int32_t s, const double* values, const double* b, double* x,
                     const ens_gmres_opts* opts, const ens_mg* mg, const void* mg_values, void* workspace,
                     size_t ws_bytes, ens_cg_stat* stats, hipStream_t stream) {
  ens_status st = check_graph_nl(graph);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK(opts && stats, "null options or stats");
  ENS_ARG_CHECK(values && b && x && workspace, "null device pointer");
  ENS_ARG_CHECK(aligned16(values) && aligned16(b) && aligned16(x), "buffers must be 16-byte aligned");
  ENS_ARG_CHECK(((uintptr_t)workspace & 255u) == 0, "workspace must be 256-byte aligned");
  ENS_ARG_CHECK(opts->rtol >= 0.0 && opts->max_iter >= 0, "bad tolerance or iteration cap");
  ENS_ARG_CHECK(opts->restart >= 1 && opts->restart <= kGmMaxRestart, "restart must be in 1..32");
  if (!supported_s(s)) {
    set_error("ensemble size %d not compiled in", s);
    return ENS_E_UNSUPPORTED;
  }
  const size_t need = gm_layout(graph->n, s, opts->restart, nullptr, nullptr);
  if (ws_bytes < need) {
    set_error("workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    return ENS_E_NOMEM;
  }
  MgPlan plan;
  if (mg) {
    st = mg_plan_for(mg, graph, s, mg_values, &plan);
    if (st != ENS_OK) return st;
  }
  GmWork w;
  gm_layout(graph->n, s, opts->restart, &w, (char*)workspace);
  switch (s) {
#define ENS_GM_CASE(SS)                                                                                       \
  case SS:                                                                                                    \
    st = gmres<SS, double>(graph, values, b, x, opts->rtol, opts->restart, opts->max_iter, mg ? &plan : nullptr, \
                           w, nullptr, nullptr, stream);                                                      \
    break;
    ENS_GM_CASE(4)
    ENS_GM_CASE(8)
    ENS_GM_CASE(16)
    ENS_GM_CASE(32)
#undef ENS_GM_CASE
  }
  if (st != ENS_OK) return st;
  GmCtl* h = (GmCtl*)malloc(sizeof(GmCtl));
  if (!h) {
    set_error("host allocation failed");
    return ENS_E_NOMEM;
  }
  hipError_t he = hipMemcpyAsync(h, w.ctl, sizeof(GmCtl), hipMemcpyDeviceToHost, stream);
  if (he == hipSuccess) he = hipStreamSynchronize(stream);
  if (he != hipSuccess) {
    free(h);
    set_error("reading the GMRES state failed: %s", hipGetErrorString(he));
    return ENS_E_HIP;
  }
  prof_collect();
  ens_status rc = ENS_OK;
  for (int e = 0; e < s; ++e) {
    stats[e].iters = h->iters[e];
    stats[e].outer_iters = h->cycles[e];
    stats[e].status = h->status[e];
    stats[e].compacted = 0;
    stats[e].rel_res = h->rel_res[e];
    if (h->status[e] != ENS_SAMPLE_CONVERGED) rc = ENS_W_NOT_CONVERGED;
  }
  free(h);
  return rc;
}

ens_status ens_newton_workspace_bytes(const ens_graph* graph, int32_t s, const ens_newton_opts* opts,
                                      size_t* bytes) {
  ens_status st = check_graph_nl(graph);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK(bytes && opts, "null output or options");
  ENS_ARG_CHECK(opts->restart >= 1 && opts->restart <= kGmMaxRestart, "restart must be in 1..32");
  if (!supported_s(s)) {
    set_error("ensemble size %d not compiled in", s);
    return ENS_E_UNSUPPORTED;
  }
  *bytes = nt_layout(graph->n, graph->nnz, s, opts->restart, opts->jac32 != 0, nullptr, nullptr);
  return ENS_OK;
}

ens_status ens_newton(int32_t N, const ens_graph* graph, const void* kl, const ens_nl_problem* problem, int32_t s,
                      const double* xi, double* u, const ens_newton_opts* opts, const ens_mg* mg,
                      const void* mg_values, void* workspace, size_t ws_bytes, ens_newton_stat* stats,
                      hipStream_t stream) {
  ens_status st = check_graph_nl(graph);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK(problem && opts && stats, "null problem, options or stats");
  ENS_ARG_CHECK(u && workspace && aligned16(u), "null or misaligned device pointer");
  ENS_ARG_CHECK(((uintptr_t)workspace & 255u) == 0, "workspace must be 256-byte aligned");
  ENS_ARG_CHECK(opts->rtol >= 0.0 && opts->lin_rtol >= 0.0, "tolerances must be >= 0");
  ENS_ARG_CHECK(opts->max_newton >= 0 && opts->lin_max_iter >= 0, "iteration caps must be >= 0");
  ENS_ARG_CHECK(opts->restart >= 1 && opts->restart <= kGmMaxRestart, "restart must be in 1..32");
  ENS_ARG_CHECK(opts->forcing == 0 || opts->forcing == 1, "forcing must be 0 (fixed) or 1 (adaptive)");
  const int64_t nn = (int64_t)(N + 1) * (N + 1) * (N + 1);
  ENS_ARG_CHECK(N >= 1 && graph->n == nn, "graph is not the N^3 mesh's graph");
  if (!supported_s(s)) {
    set_error("ensemble size %d not compiled in", s);
    return ENS_E_UNSUPPORTED;
  }
  const size_t need = nt_layout(graph->n, graph->nnz, s, opts->restart, opts->jac32 != 0, nullptr, nullptr);
  if (ws_bytes < need) {
    set_error("workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    return ENS_E_NOMEM;
  }
  MgPlan plan;
  if (mg) {
    ENS_ARG_CHECK(mg->N == N && mg->M == problem->M, "hierarchy built for another mesh or M");
    st = mg_plan_for(mg, graph, s, mg_values, &plan);
    if (st != ENS_OK) return st;
  }
  NtWork w;
  nt_layout(graph->n, graph->nnz, s, opts->restart, opts->jac32 != 0, &w, (char*)workspace);
  switch (s) {
#define ENS_NT_CASE(SS)                                                                           \
  case SS:                                                                                        \
    st = newton<SS>(N, graph, kl, problem, xi, u, *opts, mg ? &plan : nullptr, w, stream);        \
    break;
    ENS_NT_CASE(4)
    ENS_NT_CASE(8)
    ENS_NT_CASE(16)
    ENS_NT_CASE(32)
#undef ENS_NT_CASE
  }
  if (st != ENS_OK) return st;
  NtCtl h;
  ENS_HIP_TRY(hipMemcpyAsync(&h, w.ctl, sizeof(NtCtl), hipMemcpyDeviceToHost, stream));
  ENS_HIP_TRY(hipStreamSynchronize(stream));
  prof_collect();
  ens_status rc = ENS_OK;
  for (int e = 0; e < s; ++e) {
    stats[e].newton_iters = h.iters[e];
    stats[e].lin_iters = h.lin_iters[e];
    stats[e].status = h.status[e];
    stats[e].reserved = 0;
    stats[e].rel_res = h.rel_res[e];
    if (h.status[e] != ENS_SAMPLE_CONVERGED) rc = ENS_W_NOT_CONVERGED;
  }
  return rc;
}

}  // extern "C"
