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
// One iteration is three fused streaming kernels plus two small reduction
// kernels after each of the first two:
//   A: q = A p and per-block partials of p.q          -> alpha_e
//   B: x += alpha p, r -= alpha q, z = D^-1 r, partials of r.z and r.r
//                                                      -> masks, beta_e, rho_e
//   C: p = z + beta p
// Reductions are deterministic: wave butterflies between lanes holding the
// same samples, a fixed-order LDS sum per block, then the block partials are
// summed by a striped first stage and a one-block final stage, each in a
// fixed order, and the final stage updates the per-sample scalars and the
// count of active samples.  Producing kernels publish their partials by
// ending (no device-scope fences inside kernels: on this part a fence
// writes back and invalidates the XCD's L2, which costs more than the
// launch it saves).  Every kernel of the iteration returns immediately when
// the active count is zero, and the host reads the count once per chunk of
// iterations, so the loop ends on the device.
#include <mutex>
#include <vector>

#include "cgcore.hpp"
#include "mg.hpp"
#include "sctile.hpp"

namespace ens {

// First reduction stage: at most this many blocks, each summing >= 64 rows.
constexpr int kRedBlocks = 128;

// Stage 1: rows split into gridDim.x contiguous ranges, block b sums its
// range (fixed order) into out[b][P].
template <int P>
__global__ __launch_bounds__(256) void k_reduce_stage1(const double* __restrict__ part, int64_t nrows,
                                                       double* __restrict__ out, const Ctl* c, int gate) {
  if (gate && c->n_active == 0) return;
  const int64_t chunk = (nrows + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = r0 + chunk < nrows ? r0 + chunk : nrows;
  sum_rows<P>(part + r0 * P, r1 > r0 ? r1 - r0 : 0, out + (int64_t)blockIdx.x * P);
}

// Stage 2: one block sums the stage-1 rows in order and updates the
// per-sample state.
template <int S, int NQ>
__global__ __launch_bounds__(256) void k_reduce_final(const double* __restrict__ rows, int64_t nrows, Ctl* c,
                                                      int op, int arg, int gate) {
  if (gate && c->n_active == 0) return;
  sum_rows<NQ * S>(rows, nrows, c->tot);
  if (NQ == 1 && threadIdx.x < S) c->tot[S + threadIdx.x] = 0.0;
  __syncthreads();
  finalize<S>(c, op, arg);
}

// ------------------------------------------------------------ kernels ---

template <typename T, int S>
__global__ __launch_bounds__(256) void k_diag_inv(int n, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci, const T* __restrict__ vals,
                                                  T* __restrict__ dinv) {
  diag_inv_body<T, S>(n, rp, ci, vals, dinv, blockIdx.x);
}

// Wavefronts per workgroup of the CG product and the FP64 residual: 8
// (a row tile twice as deep as the cycle's row passes) measured 1.2 % (FP32)
// and 1.9 % (FP64) faster than 4 at 128^3, s = 32; the cycle's passes gain
// under 1 % in FP32 and lose 2.7 % in FP64 from it, and keep 4.
constexpr int kProdWaves = 8;

// One row tile per block (kProdWaves wavefronts).
template <int S, typename TR>
__global__ __launch_bounds__(64 * kProdWaves) void k_residual(int n, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci, const double* __restrict__ vals,
                                                  const double* __restrict__ x, const double* __restrict__ b,
                                                  TR* __restrict__ rout, double* __restrict__ part,
                                                  const Ctl* xflag) {
  // a zero initial guess (xflag->xnz == 0) makes r = b without the product
  const bool x_zero = xflag && xflag->xnz == 0;
  residual_body<S, TR, kProdWaves>(n, rp, ci, vals, x, b, rout, blockIdx.x, part + (int64_t)blockIdx.x * 2 * S,
                                   x_zero);
}

static __global__ __launch_bounds__(256) void k_x_nonzero(int64_t total, const double* __restrict__ x, Ctl* c) {
  x_nonzero_body(total, x, c);
}

template <typename T, int S>
__global__ __launch_bounds__(256) void k_cg_start(int64_t nchunks, const T* __restrict__ r,
                                                  const T* __restrict__ dinv, T* __restrict__ p,
                                                  T* __restrict__ xzero, double* __restrict__ part) {
  cg_start_body<T, S>(nchunks, r, dinv, p, xzero, blockIdx.x, part + (int64_t)blockIdx.x * 2 * S);
}

template <typename T, int S>
__global__ __launch_bounds__(64 * kProdWaves) void k_cg_spmv_dot(int n, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, const T* __restrict__ vals,
                                                     const T* __restrict__ p, T* __restrict__ q, const Ctl* c,
                                                     double* __restrict__ part) {
  if (c->n_active == 0) return;
  spmv_dot_body<T, S, kProdWaves>(n, rp, ci, vals, p, q, blockIdx.x, part + (int64_t)blockIdx.x * S);
}

template <typename T, int S>
__global__ __launch_bounds__(256) void k_cg_update(int64_t nchunks, T* __restrict__ x, const T* __restrict__ p,
                                                   const T* __restrict__ q, T* __restrict__ r,
                                                   const T* __restrict__ dinv, const Ctl* c,
                                                   double* __restrict__ part) {
  if (c->n_active == 0) return;
  update_body<T, S>(nchunks, x, p, q, r, dinv, c, blockIdx.x, part + (int64_t)blockIdx.x * 2 * S);
}

template <typename T, int S>
__global__ __launch_bounds__(256) void k_cg_pupdate(int64_t nchunks, const T* __restrict__ r,
                                                    const T* __restrict__ dinv, T* __restrict__ p, const Ctl* c) {
  if (c->n_active == 0) return;
  pupdate_body<T, S>(nchunks, r, dinv, p, c, blockIdx.x);
}

// x += d for the samples still in refinement (FP64 += FP32 correction).
template <int S>
__global__ __launch_bounds__(256) void k_ir_update(int64_t total, double* __restrict__ x,
                                                   const float* __restrict__ d, const Ctl* c) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int e = (int)(i % S);
    if (c->oactive[e]) __builtin_nontemporal_store(__builtin_nontemporal_load(x + i) + (double)__builtin_nontemporal_load(d + i), x + i);
  }
}

// x = 0 for samples whose right-hand side is zero.
template <int S>
__global__ __launch_bounds__(256) void k_zero_where(int64_t total, double* __restrict__ x, const Ctl* c) {
  zero_where_body<S>(total, x, c, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

// ----------------------------------------------- one-sample (scalar) path ---

// r = b - A x with G lanes per row (scalar CRS), block partials |r|^2, |b|^2.
template <int G>
__global__ __launch_bounds__(256) void k_residual_scalar(int n, const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci,
                                                         const double* __restrict__ vals,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ b, double* __restrict__ rout,
                                                         double* __restrict__ part) {
  const int g = threadIdx.x % G;
  double acc[2][1] = {{0.0}, {0.0}};
  const int64_t row = (int64_t)blockIdx.x * (kBlock / G) + threadIdx.x / G;
  double s = 0.0;
  if (row < n)
    for (int64_t k = rp[row] + g; k < rp[row + 1]; k += G) s += __builtin_nontemporal_load(vals + k) * x[ci[k]];
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (row < n && g == 0) {
    const double r = b[row] - s;
    if (rout) rout[row] = r;
    acc[0][0] = r * r;
    acc[1][0] = b[row] * b[row];
  }
  block_partials<1, 1, 2, kBlock / 64>(acc, part + (int64_t)blockIdx.x * 2);
}

// q = A p with G lanes per row, block partials p.q.
template <int G>
__global__ __launch_bounds__(256) void k_cg_spmv_dot_scalar(int n, const int32_t* __restrict__ rp,
                                                            const int32_t* __restrict__ ci,
                                                            const double* __restrict__ vals,
                                                            const double* __restrict__ p, double* __restrict__ q,
                                                            const Ctl* c, double* __restrict__ part) {
  if (c->n_active == 0) return;
  const int g = threadIdx.x % G;
  double acc[1][1] = {{0.0}};
  const int64_t row = (int64_t)blockIdx.x * (kBlock / G) + threadIdx.x / G;
  double s = 0.0;
  if (row < n)
    for (int64_t k = rp[row] + g; k < rp[row + 1]; k += G) s += __builtin_nontemporal_load(vals + k) * p[ci[k]];
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (row < n && g == 0) {
    q[row] = s;
    acc[0][0] = p[row] * s;
  }
  block_partials<1, 1, 1, kBlock / 64>(acc, part + (int64_t)blockIdx.x);
}

// G = 0: the same two kernels over row tiles read by the whole workgroup.
__global__ __launch_bounds__(kScThreads) void k_residual_scalar_tile(int n, const int32_t* __restrict__ rp,
                                                                    const int32_t* __restrict__ ci,
                                                                    const double* __restrict__ vals,
                                                                    const double* __restrict__ x,
                                                                    const double* __restrict__ b,
                                                                    double* __restrict__ rout,
                                                                    double* __restrict__ part) {
  __shared__ ScTileLds<double> t;
  const int64_t r0 = (int64_t)blockIdx.x * ScShape<double>::rows;
  bool has = false;
  const double s = sc_tile_row<double>(t, n, rp, ci, vals, x, r0, &has);
  double acc[2][1] = {{0.0}, {0.0}};
  if (has) {
    const int64_t row = r0 + threadIdx.x;
    const double r = b[row] - s;
    if (rout) rout[row] = r;
    acc[0][0] = r * r;
    acc[1][0] = b[row] * b[row];
  }
  block_partials<1, 1, 2, kScThreads / 64>(acc, part + (int64_t)blockIdx.x * 2);
}

__global__ __launch_bounds__(kScThreads) void k_cg_spmv_dot_scalar_tile(int n, const int32_t* __restrict__ rp,
                                                                       const int32_t* __restrict__ ci,
                                                                       const double* __restrict__ vals,
                                                                       const double* __restrict__ p,
                                                                       double* __restrict__ q, const Ctl* c,
                                                                       double* __restrict__ part) {
  if (c->n_active == 0) return;
  __shared__ ScTileLds<double> t;
  const int64_t r0 = (int64_t)blockIdx.x * ScShape<double>::rows;
  bool has = false;
  const double s = sc_tile_row<double>(t, n, rp, ci, vals, p, r0, &has);
  double acc[1][1] = {{0.0}};
  if (has) {
    const int64_t row = r0 + threadIdx.x;
    q[row] = s;
    acc[0][0] = p[row] * s;
  }
  block_partials<1, 1, 1, kScThreads / 64>(acc, part + (int64_t)blockIdx.x);
}

// rows per workgroup of the one-sample product kernels
template <int G>
constexpr int sc_rows_per_block() {
  return G == 0 ? ScShape<double>::rows : kBlock / G;
}

template <int G>
static void launch_residual_scalar(const ens_graph* g, const double* vals, const double* x, const double* b,
                                   double* rout, double* part, unsigned rb, hipStream_t st) {
  if constexpr (G == 0)
    hipLaunchKernelGGL(k_residual_scalar_tile, dim3(rb), dim3(kScThreads), 0, st, g->n, g->row_ptr, g->col_idx,
                       vals, x, b, rout, part);
  else
    hipLaunchKernelGGL(k_residual_scalar<G>, dim3(rb), dim3(kBlock), 0, st, g->n, g->row_ptr, g->col_idx, vals, x,
                       b, rout, part);
}

// ------------------------------------------------------------ host side ---

struct Work {
  Ctl* ctl;
  double* part;   // block partials, [blocks][2 s]
  double* part1;  // first-stage sums, [kRedBlocks][2 s]
  void* vec[5];
  // polls copy into a stack word instead of the device context's pinned one
  // (for the entry point that must not allocate, even the context)
  bool pageable_poll = false;
};

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Largest grid of any kernel that writes block partials for this problem.
static int64_t max_partial_blocks(int64_t n, int s) {
  if (s == 1) return (n * 32 + kBlock - 1) / kBlock + 1;  // up to 32 lanes per row
  // row kernels: 4 waves x 64/L rows, L = s/V >= s/2 (FP64 rows of the residual)
  const int64_t row_blocks = (n * s + 511) / 512 + 1;
  // streaming kernels: kU chunks of >= 2 samples per thread
  const int64_t vec_blocks = (n * s / 2 + kBlock * kU - 1) / (kBlock * kU) + 1;
  return row_blocks > vec_blocks ? row_blocks : vec_blocks;
}

static size_t ws_layout(int64_t n, int s, bool mixed, Work* w, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? base + off : nullptr;
    off += round256(bytes);
    return p;
  };
  Ctl* ctl = (Ctl*)take(sizeof(Ctl));
  double* part = (double*)take((size_t)max_partial_blocks(n, s) * 2 * s * sizeof(double));
  double* part1 = (double*)take((size_t)kRedBlocks * 2 * s * sizeof(double));
  const size_t vb = (size_t)n * s * (mixed ? sizeof(float) : sizeof(double));
  void* v[5];
  for (int i = 0; i < 5; ++i) v[i] = take(vb);
  if (w) {
    w->ctl = ctl;
    w->part = part;
    w->part1 = part1;
    for (int i = 0; i < 5; ++i) w->vec[i] = v[i];
  }
  return off;
}

static unsigned grid_for(int64_t items, int64_t per_block) {
  int64_t b = (items + per_block - 1) / per_block;
  return (unsigned)(b < 1 ? 1 : b);
}

// Sum `nrows` block partials of NQ*S doubles and run the finalize step.
// Small grids go straight to the one-block final stage.
template <int S, int NQ>
static void reduce(const Work& w, int64_t nrows, int op, int arg, int gate, hipStream_t st) {
  constexpr int P = NQ * S;
  if (nrows <= 512) {
    hipLaunchKernelGGL((k_reduce_final<S, NQ>), dim3(1), dim3(kBlock), 0, st, w.part, nrows, w.ctl, op, arg, gate);
    return;
  }
  int64_t r = nrows / 64;
  if (r > kRedBlocks) r = kRedBlocks;
  hipLaunchKernelGGL((k_reduce_stage1<P>), dim3((unsigned)r), dim3(kBlock), 0, st, w.part, nrows, w.part1, w.ctl,
                     gate);
  hipLaunchKernelGGL((k_reduce_final<S, NQ>), dim3(1), dim3(kBlock), 0, st, w.part1, r, w.ctl, op, arg, gate);
}

static ens_status poll_active(const Work& w, bool outer, hipStream_t st, int32_t* out) {
  Ctl* ctl = w.ctl;
  if (w.pageable_poll) {
    int32_t h = 0;
    ENS_HIP_TRY(hipMemcpyAsync(&h, outer ? &ctl->n_oactive : &ctl->n_active, sizeof(int32_t),
                               hipMemcpyDeviceToHost, st));
    ENS_HIP_TRY(hipStreamSynchronize(st));
    prof_collect();
    *out = h;
    return ENS_OK;
  }
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

// Launches of one CG iteration (A, reductions, B, reductions, C).
template <typename T, int S>
static void cg_iteration(const ens_graph* g, const T* vals, T* x, T* r, T* p, T* q, T* dinv, const Work& w, int k,
                         hipStream_t st) {
  using M = EnsMap<T, S>;
  using VM = VecMap<T, S>;
  const int64_t nchunks = (int64_t)g->n * S / VM::V;
  const unsigned sb = grid_for(g->n, kProdWaves * M::RPW);
  const unsigned vb = grid_for(nchunks, (int64_t)kBlock * kU);
  const int kid = sizeof(T) == 8 ? ENS_K_SPMV_F64 : ENS_K_SPMV_F32;
  const double wv = sizeof(T);
  const double spmv_bytes = (double)g->nnz * (S * wv + 4.0) + 4.0 * (g->n + 1) + 2.0 * g->n * S * wv;
  prof_begin(kid, st);
  hipLaunchKernelGGL((k_cg_spmv_dot<T, S>), dim3(sb), dim3(64 * kProdWaves), 0, st, g->n, g->row_ptr, g->col_idx, vals, p, q,
                     w.ctl, w.part);
  prof_end(kid, st, spmv_bytes);
  reduce<S, 1>(w, sb, OP_ALPHA, 0, 1, st);
  hipLaunchKernelGGL((k_cg_update<T, S>), dim3(vb), dim3(kBlock), 0, st, nchunks, x, p, q, r, dinv, w.ctl, w.part);
  reduce<S, 2>(w, vb, OP_UPDATE, k, 1, st);
  hipLaunchKernelGGL((k_cg_pupdate<T, S>), dim3(vb), dim3(kBlock), 0, st, nchunks, r, dinv, p, w.ctl);
}

// CG loop on already-initialised state; x is the solution (FP64 CG) or
// the correction d (refinement inner solve).  pause_at > 0: return after
// the first poll that finds 1..pause_at samples still iterating, with
// *paused_after = the iterations launched so far (left at -1 otherwise).
template <typename T, int S>
static ens_status cg_loop(const ens_graph* g, const T* vals, T* x, T* r, T* p, T* q, T* dinv, Work& w,
                          int max_iter, int check_every, hipStream_t st, int pause_at = 0,
                          int* paused_after = nullptr) {
  for (int k0 = 0; k0 < max_iter; k0 += check_every) {
    const int k1 = k0 + check_every < max_iter ? k0 + check_every : max_iter;
    for (int k = k0 + 1; k <= k1; ++k) cg_iteration<T, S>(g, vals, x, r, p, q, dinv, w, k, st);
    ENS_LAUNCH_CHECK();
    int32_t act = 0;
    ens_status s2 = poll_active(w, false, st, &act);
    if (s2 != ENS_OK) return s2;
    if (act == 0) break;
    if (pause_at > 0 && act <= pause_at && k1 < max_iter) {
      *paused_after = k1;
      return ENS_OK;
    }
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
    stats[e].compacted = h.compacted[e];
    stats[e].rel_res = h.rel_res[e];
    if (h.status[e] != ENS_SAMPLE_CONVERGED) rc = ENS_W_NOT_CONVERGED;
  }
  return rc;
}

// FP64 residual r = b - A x (stored as TR when rout is given) and the
// finalize step `op` on its norms.
template <int S, typename TR>
static void residual(const ens_graph* g, const double* vals, const double* x, const double* b, TR* rout,
                     const Work& w, int op, int arg, hipStream_t st, bool initial = false) {
  using M = EnsMap<double, S>;
  const unsigned sb = grid_for(g->n, kProdWaves * M::RPW);
  if (initial) {
    const int64_t total = (int64_t)g->n * S;
    const unsigned xb = grid_for(total / 2, 256 * 4);
    hipLaunchKernelGGL(k_x_nonzero, dim3(xb < 2048 ? xb : 2048), dim3(256), 0, st, total, x, w.ctl);
  }
  hipLaunchKernelGGL((k_residual<S, TR>), dim3(sb), dim3(64 * kProdWaves), 0, st, g->n, g->row_ptr, g->col_idx, vals, x, b,
                     rout, w.part, initial ? (const Ctl*)w.ctl : (const Ctl*)nullptr);
  reduce<S, 2>(w, sb, op, arg, 0, st);
}

template <typename T, int S>
static void cg_start(int64_t n, const T* r, const T* dinv, T* p, T* xzero, const Work& w, hipStream_t st) {
  const int64_t nchunks = n * S / VecMap<T, S>::V;
  const unsigned vb = grid_for(nchunks, (int64_t)kBlock * kU);
  hipLaunchKernelGGL((k_cg_start<T, S>), dim3(vb), dim3(kBlock), 0, st, nchunks, r, dinv, p, xzero, w.part);
  reduce<S, 2>(w, vb, OP_RHO, 0, 0, st);
}

// ------------------------------------------------------------ compaction --

// Columns of an ensemble picked for the compacted one: j -> sample col[j].
struct ColPick {
  int32_t col[kMaxS / 2];
};

// dst[r][j] = src[r][col[j]] for rows r < rows, j < H.
template <int S, int H>
__global__ __launch_bounds__(256) void k_gather_cols(int64_t rows, const double* __restrict__ src,
                                                     double* __restrict__ dst, ColPick pick) {
  __shared__ int32_t s_col[H];
  if (threadIdx.x < H) s_col[threadIdx.x] = pick.col[threadIdx.x];
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * H) return;
  const int64_t r = t / H;
  const int j = (int)(t % H);
  dst[t] = src[r * S + s_col[j]];
}

// dst[r][col[j]] = src[r][j] for j < m (the samples that moved).
template <int S, int H>
__global__ __launch_bounds__(256) void k_scatter_cols(int64_t rows, const double* __restrict__ src,
                                                      double* __restrict__ dst, ColPick pick, int m) {
  __shared__ int32_t s_col[H];
  if (threadIdx.x < H) s_col[threadIdx.x] = pick.col[threadIdx.x];
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * H) return;
  const int64_t r = t / H;
  const int j = (int)(t % H);
  if (j < m) dst[r * S + s_col[j]] = src[t];
}

// The CG state of the picked samples into the compacted control block; the
// columns after the m moving samples are padding and never iterate.
template <int H>
__global__ void k_ctl_compact(const Ctl* __restrict__ src, Ctl* __restrict__ dst, ColPick pick, int m) {
  const int j = threadIdx.x;
  if (j == 0) {
    dst->rtol = src->rtol;
    dst->inner_rtol = src->inner_rtol;
    dst->max_iter = src->max_iter;
    dst->inner_max_iter = src->inner_max_iter;
    dst->max_outer = src->max_outer;
    dst->mixed = src->mixed;
    dst->coupled = src->coupled;
    dst->xnz = src->xnz;
    dst->n_active = m;
    dst->n_oactive = 0;
  }
  if (j < kMaxS) {
    const bool live = j < H && j < m;
    const int e = j < H ? pick.col[j] : 0;
    dst->rho[j] = src->rho[e];
    dst->alpha[j] = src->alpha[e];
    dst->beta[j] = src->beta[e];
    dst->tol2[j] = src->tol2[e];
    dst->bnorm2[j] = src->bnorm2[e];
    dst->rel_res[j] = src->rel_res[e];
    dst->orr_prev[j] = src->orr_prev[e];
    dst->active[j] = live ? src->active[e] : 0;
    dst->oactive[j] = 0;
    dst->iters[j] = src->iters[e];
    dst->oiters[j] = src->oiters[e];
    dst->kiter[j] = src->kiter[e];
    dst->status[j] = src->status[e];
    dst->zero_b[j] = src->zero_b[e];
    dst->compacted[j] = live;
  }
}

// The moved samples' CG state back into the full control block.
template <int H>
__global__ void k_ctl_expand(const Ctl* __restrict__ src, Ctl* __restrict__ dst, ColPick pick, int m) {
  const int j = threadIdx.x;
  if (j < H && j < m) {
    const int e = pick.col[j];
    dst->rho[e] = src->rho[j];
    dst->rel_res[e] = src->rel_res[j];
    dst->active[e] = src->active[j];
    dst->iters[e] = src->iters[j];
    dst->kiter[e] = src->kiter[j];
    dst->status[e] = src->status[j];
    dst->compacted[e] = 1;
  }
  __syncthreads();
  if (j == 0) {
    int na = 0;
    for (int q = 0; q < kMaxS; ++q) na += dst->active[q];
    dst->n_active = na;
  }
}

// Bytes of the compacted ensemble: its control block, matrix values and
// five vectors (x, r, p, q, D^-1), for an s-sample solve (0 if s < 8).
static size_t compact_bytes(int64_t n, int64_t nnz, int s) {
  if (s < 8) return 0;
  const size_t h = (size_t)s / 2;
  return round256(sizeof(Ctl)) + round256((size_t)nnz * h * sizeof(double)) +
         5 * round256((size_t)n * h * sizeof(double));
}

// Finish the samples still iterating in an ensemble of H = S/2: gather the
// values, vectors and CG state of the active samples (padded with finished
// ones, which stay inactive), run the loop there, scatter x and the state
// back.
template <int S, int H>
static ens_status cg_compacted(const ens_graph* g, const double* vals, double* x, const double* r, const double* p,
                               const double* dinv, Work& w, int max_iter, int check_every, char* base,
                               hipStream_t st) {
  int32_t act[kMaxS];
  ENS_HIP_TRY(hipMemcpyAsync(act, w.ctl->active, sizeof(int32_t) * S, hipMemcpyDeviceToHost, st));
  ENS_HIP_TRY(hipStreamSynchronize(st));
  ColPick pick{};
  int m = 0;
  for (int e = 0; e < S && m < H; ++e)
    if (act[e]) pick.col[m++] = e;
  int k = m;
  for (int e = 0; e < S && k < H; ++e)
    if (!act[e]) pick.col[k++] = e;
  const int64_t n = g->n, nnz = g->nnz;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* q = base + off;
    off += round256(bytes);
    return q;
  };
  Ctl* cc = (Ctl*)take(sizeof(Ctl));
  double* vc = (double*)take((size_t)nnz * H * sizeof(double));
  double* xc = (double*)take((size_t)n * H * sizeof(double));
  double* rc = (double*)take((size_t)n * H * sizeof(double));
  double* pc = (double*)take((size_t)n * H * sizeof(double));
  double* qc = (double*)take((size_t)n * H * sizeof(double));
  double* dc = (double*)take((size_t)n * H * sizeof(double));
  const unsigned gv = grid_for(nnz * H, 256), gn = grid_for(n * H, 256);
  hipLaunchKernelGGL((k_gather_cols<S, H>), dim3(gv), dim3(256), 0, st, nnz, vals, vc, pick);
  hipLaunchKernelGGL((k_gather_cols<S, H>), dim3(gn), dim3(256), 0, st, n, x, xc, pick);
  hipLaunchKernelGGL((k_gather_cols<S, H>), dim3(gn), dim3(256), 0, st, n, r, rc, pick);
  hipLaunchKernelGGL((k_gather_cols<S, H>), dim3(gn), dim3(256), 0, st, n, p, pc, pick);
  hipLaunchKernelGGL((k_gather_cols<S, H>), dim3(gn), dim3(256), 0, st, n, dinv, dc, pick);
  hipLaunchKernelGGL((k_ctl_compact<H>), dim3(1), dim3(64), 0, st, w.ctl, cc, pick, m);
  ENS_LAUNCH_CHECK();
  Work cw = w;
  cw.ctl = cc;
  ens_status rc2 = cg_loop<double, H>(g, vc, xc, rc, pc, qc, dc, cw, max_iter, check_every, st);
  if (rc2 != ENS_OK) return rc2;
  hipLaunchKernelGGL((k_scatter_cols<S, H>), dim3(gn), dim3(256), 0, st, n, xc, x, pick, m);
  hipLaunchKernelGGL((k_ctl_expand<H>), dim3(1), dim3(64), 0, st, cc, w.ctl, pick, m);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

template <int S>
static ens_status cg_fp64(const ens_graph* g, const double* vals, const double* b, double* x,
                          const ens_cg_opts& o, Work& w, hipStream_t st, char* compact_base = nullptr) {
  double* r = (double*)w.vec[0];
  double* p = (double*)w.vec[1];
  double* q = (double*)w.vec[2];
  double* dinv = (double*)w.vec[3];
  const int64_t n = g->n;
  const int64_t total = n * S;
  hipLaunchKernelGGL((k_diag_inv<double, S>), dim3(grid_for(total, 256)), dim3(256), 0, st, g->n, g->row_ptr,
                     g->col_idx, vals, dinv);
  residual<S, double>(g, vals, x, b, r, w, OP_START, 0, st, true);
  hipLaunchKernelGGL(k_zero_where<S>, dim3(grid_for(total, 256 * 8)), dim3(kBlock), 0, st, total, x, w.ctl);
  cg_start<double, S>(n, r, dinv, p, (double*)nullptr, w, st);
  ENS_LAUNCH_CHECK();
  int paused = -1;
  const int pause_at = (compact_base && S >= 8) ? S / 2 : 0;
  ens_status rc = cg_loop<double, S>(g, vals, x, r, p, q, dinv, w, o.max_iter, o.check_every, st, pause_at, &paused);
  if (rc != ENS_OK) return rc;
  if constexpr (S >= 8) {
    if (paused >= 0) {
      rc = cg_compacted<S, S / 2>(g, vals, x, r, p, dinv, w, o.max_iter - paused, o.check_every, compact_base, st);
      if (rc != ENS_OK) return rc;
    }
  }
  residual<S, double>(g, vals, x, b, (double*)nullptr, w, OP_TRUE, 0, st);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

template <int S>
static ens_status cg_mixed(const ens_graph* g, const double* vals, const float* vals32, const double* b, double* x,
                           const ens_cg_opts& o, Work& w, hipStream_t st) {
  float* r = (float*)w.vec[0];
  float* p = (float*)w.vec[1];
  float* q = (float*)w.vec[2];
  float* dinv = (float*)w.vec[3];
  float* d = (float*)w.vec[4];
  const int64_t n = g->n;
  const int64_t total = n * S;
  hipLaunchKernelGGL((k_diag_inv<float, S>), dim3(grid_for(total, 256)), dim3(256), 0, st, g->n, g->row_ptr,
                     g->col_idx, vals32, dinv);
  ENS_LAUNCH_CHECK();
  for (int outer = 0;; ++outer) {
    residual<S, float>(g, vals, x, b, r, w, OP_OUTER, outer, st, outer == 0);
    if (outer == 0)
      hipLaunchKernelGGL(k_zero_where<S>, dim3(grid_for(total, 256 * 8)), dim3(kBlock), 0, st, total, x, w.ctl);
    ENS_LAUNCH_CHECK();
    int32_t act = 0;
    ens_status rc = poll_active(w, true, st, &act);
    if (rc != ENS_OK) return rc;
    if (act == 0) break;
    cg_start<float, S>(n, r, dinv, p, d, w, st);
    ENS_LAUNCH_CHECK();
    rc = cg_loop<float, S>(g, vals32, d, r, p, q, dinv, w, o.inner_max_iter, o.check_every, st);
    if (rc != ENS_OK) return rc;
    hipLaunchKernelGGL(k_ir_update<S>, dim3(grid_for(total, 256 * 8)), dim3(kBlock), 0, st, total, x, d, w.ctl);
    ENS_LAUNCH_CHECK();
  }
  return ENS_OK;
}

// One-sample Jacobi-CG in three phases so that several independent solves
// can be interleaved on their own streams: set-up (control block, D^-1,
// r = b - A x, first direction), iterations k0+1..k1, true residual.
template <int G>
static void scalar_setup(const ens_graph* g, const double* vals, const double* b, double* x, const ens_cg_opts& o,
                         const Work& w, hipStream_t st) {
  double* r = (double*)w.vec[0];
  double* p = (double*)w.vec[1];
  double* dinv = (double*)w.vec[3];
  const int64_t n = g->n;
  const unsigned rb = grid_for(n, sc_rows_per_block<G>());
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, st, w.ctl, o.rtol, o.inner_rtol, o.max_iter,
                     o.inner_max_iter, o.max_outer, 0, 0);
  hipLaunchKernelGGL((k_diag_inv<double, 1>), dim3(grid_for(n, 256)), dim3(256), 0, st, g->n, g->row_ptr,
                     g->col_idx, vals, dinv);
  launch_residual_scalar<G>(g, vals, x, b, r, w.part, rb, st);
  reduce<1, 2>(w, rb, OP_START, 0, 0, st);
  hipLaunchKernelGGL(k_zero_where<1>, dim3(grid_for(n, 256 * 8)), dim3(kBlock), 0, st, n, x, w.ctl);
  cg_start<double, 1>(n, r, dinv, p, (double*)nullptr, w, st);
}

template <int G>
static void scalar_iters(const ens_graph* g, const double* vals, double* x, const Work& w, int k0, int k1,
                         hipStream_t st) {
  double* r = (double*)w.vec[0];
  double* p = (double*)w.vec[1];
  double* q = (double*)w.vec[2];
  double* dinv = (double*)w.vec[3];
  const int64_t n = g->n;
  const unsigned rb = grid_for(n, sc_rows_per_block<G>());
  const unsigned vb = grid_for(n, (int64_t)kBlock * kU);
  for (int k = k0 + 1; k <= k1; ++k) {
    prof_begin(ENS_K_SCALAR_SPMV, st);
    if constexpr (G == 0)
      hipLaunchKernelGGL(k_cg_spmv_dot_scalar_tile, dim3(rb), dim3(kScThreads), 0, st, g->n, g->row_ptr, g->col_idx,
                         vals, p, q, w.ctl, w.part);
    else
      hipLaunchKernelGGL(k_cg_spmv_dot_scalar<G>, dim3(rb), dim3(kBlock), 0, st, g->n, g->row_ptr, g->col_idx, vals,
                         p, q, w.ctl, w.part);
    prof_end(ENS_K_SCALAR_SPMV, st, (double)g->nnz * 12.0 + 4.0 * (n + 1) + 16.0 * n);
    reduce<1, 1>(w, rb, OP_ALPHA, 0, 1, st);
    hipLaunchKernelGGL((k_cg_update<double, 1>), dim3(vb), dim3(kBlock), 0, st, n, x, p, q, r, dinv, w.ctl, w.part);
    reduce<1, 2>(w, vb, OP_UPDATE, k, 1, st);
    hipLaunchKernelGGL((k_cg_pupdate<double, 1>), dim3(vb), dim3(kBlock), 0, st, n, r, dinv, p, w.ctl);
  }
}

template <int G>
static void scalar_finish(const ens_graph* g, const double* vals, const double* b, const double* x, const Work& w,
                          hipStream_t st) {
  const unsigned rb = grid_for(g->n, sc_rows_per_block<G>());
  launch_residual_scalar<G>(g, vals, x, b, (double*)nullptr, w.part, rb, st);
  reduce<1, 2>(w, rb, OP_TRUE, 0, 0, st);
}

template <int G>
static ens_status cg_scalar_one(const ens_graph* g, const double* vals, const double* b, double* x,
                                const ens_cg_opts& o, Work& w, hipStream_t st) {
  scalar_setup<G>(g, vals, b, x, o, w, st);
  ENS_LAUNCH_CHECK();
  for (int k0 = 0; k0 < o.max_iter; k0 += o.check_every) {
    const int k1 = k0 + o.check_every < o.max_iter ? k0 + o.check_every : o.max_iter;
    scalar_iters<G>(g, vals, x, w, k0, k1, st);
    ENS_LAUNCH_CHECK();
    int32_t act = 0;
    ens_status rc = poll_active(w, false, st, &act);
    if (rc != ENS_OK) return rc;
    if (act == 0) break;
  }
  scalar_finish<G>(g, vals, b, x, w, st);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

// Up to `ns` one-sample solves at a time, each on its own stream with its
// own workspace slice; the host launches a chunk of iterations for every
// unfinished solve, then polls all of them once.
template <int G>
static ens_status cg_scalar_concurrent(const ens_graph* g, int s, const double* values, const double* b, double* x,
                                       const ens_cg_opts& o, int ns, char* ws, size_t slice, ens_cg_stat* stats,
                                       hipStream_t user) {
  DeviceCtx* cx = device_ctx();
  if (!cx || !ensure_side_streams(cx, ns)) {
    set_error("could not create the side streams");
    return ENS_E_HIP;
  }
  const int64_t n = g->n, nnz = g->nnz;
  std::vector<Work> w(ns);
  for (int i = 0; i < ns; ++i) ws_layout(n, 1, false, &w[i], ws + (size_t)i * slice);
  ENS_HIP_TRY(hipEventRecord(cx->ev_in, user));
  for (int i = 0; i < ns; ++i) ENS_HIP_TRY(hipStreamWaitEvent(cx->side[i], cx->ev_in, 0));
  ens_status agg = ENS_OK;
  for (int e0 = 0; e0 < s; e0 += ns) {
    const int m = s - e0 < ns ? s - e0 : ns;
    std::vector<int> active;
    for (int i = 0; i < m; ++i) {
      const int e = e0 + i;
      scalar_setup<G>(g, values + (int64_t)e * nnz, b + (int64_t)e * n, x + (int64_t)e * n, o, w[i], cx->side[i]);
      active.push_back(i);
    }
    ENS_LAUNCH_CHECK();
    for (int k0 = 0; k0 < o.max_iter && !active.empty(); k0 += o.check_every) {
      const int k1 = k0 + o.check_every < o.max_iter ? k0 + o.check_every : o.max_iter;
      for (int i : active) {
        const int e = e0 + i;
        scalar_iters<G>(g, values + (int64_t)e * nnz, x + (int64_t)e * n, w[i], k0, k1, cx->side[i]);
        ENS_HIP_TRY(hipMemcpyAsync(cx->host_flag + i, &w[i].ctl->n_active, sizeof(int32_t), hipMemcpyDeviceToHost,
                                   cx->side[i]));
      }
      ENS_LAUNCH_CHECK();
      for (int i : active) ENS_HIP_TRY(hipStreamSynchronize(cx->side[i]));
      prof_collect();
      std::vector<int> still;
      for (int i : active)
        if (cx->host_flag[i] != 0) still.push_back(i);
      active.swap(still);
    }
    for (int i = 0; i < m; ++i) {
      const int e = e0 + i;
      scalar_finish<G>(g, values + (int64_t)e * nnz, b + (int64_t)e * n, x + (int64_t)e * n, w[i], cx->side[i]);
    }
    ENS_LAUNCH_CHECK();
    for (int i = 0; i < m; ++i) {
      ens_status st = read_stats(w[i].ctl, 1, &stats[e0 + i], cx->side[i]);
      if (st == ENS_W_NOT_CONVERGED) agg = st;
      else if (st != ENS_OK) return st;
    }
  }
  for (int i = 0; i < ns; ++i) {
    ENS_HIP_TRY(hipEventRecord(cx->side_ev[i], cx->side[i]));
    ENS_HIP_TRY(hipStreamWaitEvent(user, cx->side_ev[i], 0));
  }
  return agg;
}

template <typename T, int S>
__global__ __launch_bounds__(256) void k_mg_update_r(int64_t nchunks, T* __restrict__ x, const T* __restrict__ p,
                                                     const T* __restrict__ q, T* __restrict__ r, const Ctl* c,
                                                     double* __restrict__ part) {
  if (c->n_active == 0) return;
  update_r_body<T, S>(nchunks, x, p, q, r, c, blockIdx.x, part + (int64_t)blockIdx.x * 2 * S);
}

template <typename T, int S>
__global__ __launch_bounds__(256) void k_mg_rz(int64_t nchunks, const T* __restrict__ r, const T* __restrict__ z,
                                               T* __restrict__ pz, const Ctl* c, int gate, double* __restrict__ part) {
  if (gate && c->n_active == 0) return;
  rz_body<T, S>(nchunks, r, z, pz, blockIdx.x, part + (int64_t)blockIdx.x * 2 * S);
}

template <typename T, int S>
__global__ __launch_bounds__(256) void k_mg_pz(int64_t nchunks, const T* __restrict__ z, T* __restrict__ p,
                                               const Ctl* c) {
  if (c->n_active == 0) return;
  pupdate_z_body<T, S>(nchunks, z, p, c, blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill_zero(int64_t count, T* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) v[i] = (T)0;
}

// Iterations k0+1..k1 of CG with z = M r in precision T: q = A p and alpha;
// the update of x and r with the convergence test; the cycle; r.z and beta;
// the new direction.  x is the solution (FP64 solve) or the correction d
// (FP32 inner solve of the refinement).
template <typename T, int S>
static void mg_iterations(const ens_graph* g, const T* vals, const MgPlan& plan, T* x, T* r, T* p, T* q, T* z,
                          const Work& w, int k0, int k1, hipStream_t st) {
  const int64_t n = g->n;
  const int64_t nchunks = n * S / VecMap<T, S>::V;
  const unsigned sb = grid_for(n, kProdWaves * EnsMap<T, S>::RPW);
  const unsigned db = grid_for(n, 4 * EnsMap<T, S>::RPW);  // row tiles of the cycle's passes
  const unsigned vb = grid_for(nchunks, (int64_t)kBlock * kU);
  const int kid = sizeof(T) == 8 ? ENS_K_SPMV_F64 : ENS_K_SPMV_F32;
  const double spmv_bytes = (double)g->nnz * (S * (double)sizeof(T) + 4.0) + 4.0 * (n + 1) + 2.0 * n * S * sizeof(T);
  for (int k = k0 + 1; k <= k1; ++k) {
    prof_begin(kid, st);
    hipLaunchKernelGGL((k_cg_spmv_dot<T, S>), dim3(sb), dim3(64 * kProdWaves), 0, st, g->n, g->row_ptr, g->col_idx, vals, p, q,
                       w.ctl, w.part);
    prof_end(kid, st, spmv_bytes);
    reduce<S, 1>(w, sb, OP_ALPHA, 0, 1, st);
    hipLaunchKernelGGL((k_mg_update_r<T, S>), dim3(vb), dim3(kBlock), 0, st, nchunks, x, p, q, r, w.ctl, w.part);
    reduce<S, 2>(w, vb, OP_UPDATE_R, k, 1, st);
    // the cycle's last fine-level pass also writes the r . z partials, one
    // row per row tile of that pass (db rows)
    mg_vcycle<T, S>(plan, r, z, w.ctl, st, w.part);
    reduce<S, 1>(w, db, OP_BETA, 0, 1, st);
    hipLaunchKernelGGL((k_mg_pz<T, S>), dim3(vb), dim3(kBlock), 0, st, nchunks, z, p, w.ctl);
  }
}

// z = M r, p = z and rho = r.z for the active samples.
template <typename T, int S>
static void mg_start(int64_t n, const MgPlan& plan, T* r, T* z, T* p, const Work& w, hipStream_t st) {
  const int64_t nchunks = n * S / VecMap<T, S>::V;
  const unsigned vb = grid_for(nchunks, (int64_t)kBlock * kU);
  mg_vcycle<T, S>(plan, r, z, w.ctl, st);
  hipLaunchKernelGGL((k_mg_rz<T, S>), dim3(vb), dim3(kBlock), 0, st, nchunks, r, z, p, w.ctl, 0, w.part);
  reduce<S, 2>(w, vb, OP_RHO, 0, 0, st);
}

// FP64 CG with z = M r from the FP64 multigrid cycle.
template <int S>
static ens_status cg_mg(const ens_graph* g, const double* vals, const double* b, double* x, const ens_cg_opts& o,
                        const MgPlan& plan, Work& w, hipStream_t st) {
  double* r = (double*)w.vec[0];
  double* p = (double*)w.vec[1];
  double* q = (double*)w.vec[2];
  double* z = (double*)w.vec[3];
  const int64_t n = g->n;
  const int64_t total = n * S;
  residual<S, double>(g, vals, x, b, r, w, OP_START, 0, st, true);
  hipLaunchKernelGGL(k_zero_where<S>, dim3(grid_for(total, 256 * 8)), dim3(kBlock), 0, st, total, x, w.ctl);
  mg_start<double, S>(n, plan, r, z, p, w, st);
  ENS_LAUNCH_CHECK();
  for (int k0 = 0; k0 < o.max_iter; k0 += o.check_every) {
    const int k1 = k0 + o.check_every < o.max_iter ? k0 + o.check_every : o.max_iter;
    mg_iterations<double, S>(g, vals, plan, x, r, p, q, z, w, k0, k1, st);
    ENS_LAUNCH_CHECK();
    int32_t act = 0;
    ens_status rc = poll_active(w, false, st, &act);
    if (rc != ENS_OK) return rc;
    if (act == 0) break;
  }
  residual<S, double>(g, vals, x, b, (double*)nullptr, w, OP_TRUE, 0, st);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

// FP32-in-FP64 refinement whose FP32 inner CG is preconditioned by the FP32
// multigrid cycle: FP64 residual r = b - A x rounded to FP32, inner solve
// A32 d = r32 to the inner tolerance, x += d in FP64.
template <int S>
static ens_status cg_mixed_mg(const ens_graph* g, const double* vals, const float* vals32, const double* b, double* x,
                              const ens_cg_opts& o, const MgPlan& plan, Work& w, hipStream_t st) {
  float* r = (float*)w.vec[0];
  float* p = (float*)w.vec[1];
  float* q = (float*)w.vec[2];
  float* z = (float*)w.vec[3];
  float* d = (float*)w.vec[4];
  const int64_t n = g->n;
  const int64_t total = n * S;
  for (int outer = 0;; ++outer) {
    residual<S, float>(g, vals, x, b, r, w, OP_OUTER, outer, st, outer == 0);
    if (outer == 0)
      hipLaunchKernelGGL(k_zero_where<S>, dim3(grid_for(total, 256 * 8)), dim3(kBlock), 0, st, total, x, w.ctl);
    ENS_LAUNCH_CHECK();
    int32_t act = 0;
    ens_status rc = poll_active(w, true, st, &act);
    if (rc != ENS_OK) return rc;
    if (act == 0) break;
    hipLaunchKernelGGL(k_fill_zero<float>, dim3(grid_for(total, 256)), dim3(256), 0, st, total, d);
    mg_start<float, S>(n, plan, r, z, p, w, st);
    ENS_LAUNCH_CHECK();
    for (int k0 = 0; k0 < o.inner_max_iter; k0 += o.check_every) {
      const int k1 = k0 + o.check_every < o.inner_max_iter ? k0 + o.check_every : o.inner_max_iter;
      mg_iterations<float, S>(g, vals32, plan, d, r, p, q, z, w, k0, k1, st);
      ENS_LAUNCH_CHECK();
      rc = poll_active(w, false, st, &act);
      if (rc != ENS_OK) return rc;
      if (act == 0) break;
    }
    hipLaunchKernelGGL(k_ir_update<S>, dim3(grid_for(total, 256 * 8)), dim3(kBlock), 0, st, total, x, d, w.ctl);
    ENS_LAUNCH_CHECK();
  }
  return ENS_OK;
}

ens_status check_graph(const ens_graph* g);

static ens_cg_opts normalized(const ens_cg_opts* in) {
  ens_cg_opts o = *in;
  if (o.max_iter <= 0) o.max_iter = 10000;
  if (o.inner_max_iter <= 0) o.inner_max_iter = 10000;
  if (o.max_outer <= 0) o.max_outer = 10;
  if (o.check_every <= 0) o.check_every = 16;
  if (!(o.inner_rtol > 0.0)) o.inner_rtol = 1e-5;
  return o;
}

// ens_cg on a given workspace; pageable_poll: polls without the device
// context (ens_cg_noalloc).
static ens_status cg_run(const ens_graph* graph, int32_t s, const double* values, const float* values32,
                         const double* b, double* x, const ens_cg_opts* opts, void* workspace, size_t ws_bytes,
                         ens_cg_stat* stats, hipStream_t stream, bool pageable_poll) {
  ens_status st = check_graph(graph);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK(opts && stats, "null options or stats");
  ENS_ARG_CHECK(values && b && x && workspace, "null device pointer");
  ENS_ARG_CHECK(aligned16(values) && aligned16(b) && aligned16(x), "buffers must be 16-byte aligned");
  ENS_ARG_CHECK(((uintptr_t)workspace & 255u) == 0, "workspace must be 256-byte aligned");
  ENS_ARG_CHECK(opts->rtol >= 0.0, "rtol must be >= 0");
  ENS_ARG_CHECK(!opts->mixed || (values32 && aligned16(values32)), "mixed mode needs values32");
  if (opts->mixed && opts->coupled) {
    set_error("coupled CG is implemented for FP64 (mixed = 0) only");
    return ENS_E_UNSUPPORTED;
  }
  ENS_ARG_CHECK(!opts->compact || (!opts->mixed && !opts->coupled),
                "compaction is for the FP64 per-sample CG (mixed and coupled 0)");
  if (!supported_s(s)) {
    set_error("ensemble size %d not compiled in", s);
    return ENS_E_UNSUPPORTED;
  }
  const bool mixed = opts->mixed != 0;
  const size_t base_need = ws_layout(graph->n, s, mixed, nullptr, nullptr);
  const size_t cbytes = opts->compact ? compact_bytes(graph->n, graph->nnz, s) : 0;
  const size_t need = base_need + cbytes;
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
  w.pageable_poll = pageable_poll;
  ens_cg_opts o = normalized(opts);
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, stream, w.ctl, o.rtol, o.inner_rtol, o.max_iter,
                     o.inner_max_iter, o.max_outer, (int)mixed, o.coupled ? 1 : 0);
  ENS_LAUNCH_CHECK();
  switch (s) {
#define ENS_CG_CASE(SS)                                                                                      \
  case SS:                                                                                                   \
    st = mixed ? cg_mixed<SS>(graph, values, values32, b, x, o, w, stream)                                  \
               : cg_fp64<SS>(graph, values, b, x, o, w, stream, cbytes ? (char*)workspace + base_need : nullptr); \
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

// Workspace bytes of ens_cg for these options (graph and s checked).
static size_t cg_ws_need(const ens_graph* graph, int s, const ens_cg_opts& o) {
  return ws_layout(graph->n, s, o.mixed != 0, nullptr, nullptr) +
         (o.compact && !o.mixed && !o.coupled ? compact_bytes(graph->n, graph->nnz, s) : 0);
}

// Workspace of ens_cg_noalloc: a file-scope device array, one copy per GPU,
// held until the process ends and shared by every call on that GPU.  In host
// code the name is a host-side stand-in, never a device address: kernels
// and copies get the address hipGetSymbolAddress returns, resolved once per
// device with that device current.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_ptr;  // by device id

static ens_status scratch_ptr(void** out) {
  int dev = 0;
  ENS_HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
      return ENS_E_HIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ENS_OK;
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
  *bytes = ws_layout(graph->n, s, opts->mixed != 0, nullptr, nullptr) +
           (opts->compact && !opts->mixed && !opts->coupled ? compact_bytes(graph->n, graph->nnz, s) : 0);
  return ENS_OK;
}

ens_status ens_cg(const ens_graph* graph, int32_t s, const double* values, const float* values32, const double* b,
                  double* x, const ens_cg_opts* opts, void* workspace, size_t ws_bytes, ens_cg_stat* stats,
                  hipStream_t stream) {
  return cg_run(graph, s, values, values32, b, x, opts, workspace, ws_bytes, stats, stream, false);
}

ens_status ens_cg_noalloc(const ens_graph* graph, int32_t s, const double* values, const float* values32,
                          const double* b, double* x, const ens_cg_opts* opts, ens_cg_stat* stats,
                          hipStream_t stream) {
  // size check first: it needs no device and allocates nothing
  ens_status st = check_graph(graph);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK(opts, "null options");
  if (!supported_s(s)) {
    set_error("ensemble size %d not compiled in", s);
    return ENS_E_UNSUPPORTED;
  }
  const size_t need = cg_ws_need(graph, s, *opts);
  if (need > kScratchBytes) {
    set_error("ens_cg_noalloc needs %zu bytes of workspace; its scratch array holds %zu (use ens_cg with a "
              "caller workspace)", need, kScratchBytes);
    return ENS_E_NOMEM;
  }
  void* ws = nullptr;
  st = scratch_ptr(&ws);
  if (st != ENS_OK) return st;
  ProfPause no_events;
  return cg_run(graph, s, values, values32, b, x, opts, ws, kScratchBytes, stats, stream, true);
}

ens_status ens_cg_mg(const ens_graph* graph, int32_t s, const double* values, const float* values32, const double* b,
                     double* x, const ens_cg_opts* opts, const ens_mg* mg, void* workspace, size_t ws_bytes,
                     ens_cg_stat* stats, hipStream_t stream) {
  ens_status st = check_graph(graph);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK(opts && stats && mg && mg->buffer, "null options, stats or hierarchy");
  ENS_ARG_CHECK(values && b && x && workspace, "null device pointer");
  ENS_ARG_CHECK(aligned16(values) && aligned16(b) && aligned16(x), "buffers must be 16-byte aligned");
  ENS_ARG_CHECK(((uintptr_t)workspace & 255u) == 0, "workspace must be 256-byte aligned");
  ENS_ARG_CHECK(opts->rtol >= 0.0, "rtol must be >= 0");
  ENS_ARG_CHECK(!opts->coupled, "the multigrid solve uses per-sample scalars");
  ENS_ARG_CHECK(!opts->compact, "the multigrid solve does not compact (compact must be 0)");
  ENS_ARG_CHECK((opts->mixed != 0) == (mg->fp32 != 0), "mixed mode needs an FP32 cycle, FP64 CG an FP64 one");
  ENS_ARG_CHECK(!opts->mixed || (values32 && aligned16(values32)), "mixed mode needs values32");
  ENS_ARG_CHECK(mg->s == s, "hierarchy built for another ensemble size");
  const int64_t nn = (int64_t)(mg->N + 1) * (mg->N + 1) * (mg->N + 1);
  ENS_ARG_CHECK(graph->n == nn, "graph is not the hierarchy's fine mesh");
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
  if (mg_stage(mg) < 2) {
    set_error("multigrid hierarchy not set up: call ens_mg_build and ens_mg_setup first");
    return ENS_E_ARG;
  }
  if (mg_nonsym(mg)) {
    set_error("multigrid hierarchy set up for a nonsymmetric operator: CG needs a symmetric preconditioner");
    return ENS_E_ARG;
  }
  MgPlan plan;
  if (!mg_plan(mg->N, mg->M, s, mg->fp32 != 0, (char*)mg->buffer, &plan)) {
    set_error("multigrid hierarchy of N=%d is not supported", mg->N);
    return ENS_E_UNSUPPORTED;
  }
  if (mg->bytes < plan.bytes) {
    set_error("multigrid buffer of %zu bytes is smaller than the %zu required", mg->bytes, plan.bytes);
    return ENS_E_NOMEM;
  }
  mg_attach_fine(&plan, graph->row_ptr, graph->col_idx, values, mixed ? values32 : nullptr);
  Work w;
  ws_layout(graph->n, s, mixed, &w, (char*)workspace);
  ens_cg_opts o = normalized(opts);
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, stream, w.ctl, o.rtol, o.inner_rtol, o.max_iter,
                     o.inner_max_iter, o.max_outer, (int)mixed, 0);
  ENS_LAUNCH_CHECK();
  switch (s) {
#define ENS_MG_CASE(SS)                                                                      \
  case SS:                                                                                   \
    st = mixed ? cg_mixed_mg<SS>(graph, values, values32, b, x, o, plan, w, stream)          \
               : cg_mg<SS>(graph, values, b, x, o, plan, w, stream);                         \
    break;
    ENS_MG_CASE(4)
    ENS_MG_CASE(8)
    ENS_MG_CASE(16)
    ENS_MG_CASE(32)
#undef ENS_MG_CASE
  }
  if (st != ENS_OK) return st;
  return read_stats(w.ctl, s, stats, stream);
}

ens_status ens_scalar_cg_concurrent_workspace_bytes(const ens_graph* graph, int32_t streams, size_t* bytes) {
  ens_status st = check_graph(graph);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK(bytes && streams >= 1 && streams <= kMaxSideStreams, "streams must be in 1..32");
  *bytes = (size_t)streams * ws_layout(graph->n, 1, false, nullptr, nullptr);
  return ENS_OK;
}

ens_status ens_scalar_cg_concurrent(const ens_graph* graph, int32_t s, const double* values, const double* b,
                                    double* x, const ens_cg_opts* opts, int32_t lanes_per_row, int32_t streams,
                                    void* workspace, size_t ws_bytes, ens_cg_stat* stats, hipStream_t stream) {
  ens_status st = check_graph(graph);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK(opts && stats && s >= 1, "bad arguments");
  ENS_ARG_CHECK(streams >= 1 && streams <= kMaxSideStreams, "streams must be in 1..32");
  ENS_ARG_CHECK(!opts->mixed && !opts->coupled, "the scalar baseline is per-sample FP64");
  ENS_ARG_CHECK(!opts->compact, "the scalar baseline does not compact (compact must be 0)");
  ENS_ARG_CHECK(values && b && x && workspace, "null device pointer");
  ENS_ARG_CHECK(((uintptr_t)workspace & 255u) == 0, "workspace must be 256-byte aligned");
  if (graph->n == 0) {
    for (int e = 0; e < s; ++e) stats[e] = ens_cg_stat{0, 0, ENS_SAMPLE_CONVERGED, 0, 0.0};
    return ENS_OK;
  }
  const size_t slice = ws_layout(graph->n, 1, false, nullptr, nullptr);
  const int ns = streams < s ? streams : s;
  if (ws_bytes < (size_t)ns * slice) {
    set_error("workspace of %zu bytes is smaller than the %zu required", ws_bytes, (size_t)ns * slice);
    return ENS_E_NOMEM;
  }
  ens_cg_opts o = normalized(opts);
  ENS_ARG_CHECK(lanes_per_row >= 0, "lanes_per_row must be 0 (row tiles) or 4, 8, 16, 32");
  switch (lanes_per_row) {
    case 0: return cg_scalar_concurrent<0>(graph, s, values, b, x, o, ns, (char*)workspace, slice, stats, stream);
    case 4: return cg_scalar_concurrent<4>(graph, s, values, b, x, o, ns, (char*)workspace, slice, stats, stream);
    case 8: return cg_scalar_concurrent<8>(graph, s, values, b, x, o, ns, (char*)workspace, slice, stats, stream);
    case 16: return cg_scalar_concurrent<16>(graph, s, values, b, x, o, ns, (char*)workspace, slice, stats, stream);
    case 32: return cg_scalar_concurrent<32>(graph, s, values, b, x, o, ns, (char*)workspace, slice, stats, stream);
    default: set_error("lanes_per_row %d not supported", lanes_per_row); return ENS_E_ARG;
  }
}

ens_status ens_scalar_cg(const ens_graph* graph, int32_t s, const double* values, const double* b, double* x,
                         const ens_cg_opts* opts, int32_t lanes_per_row, void* workspace, size_t ws_bytes,
                         ens_cg_stat* stats, hipStream_t stream) {
  ens_status st = check_graph(graph);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK(opts && stats && s >= 1, "bad arguments");
  ENS_ARG_CHECK(!opts->mixed, "the scalar baseline is FP64 only");
  ENS_ARG_CHECK(!opts->coupled, "the scalar baseline solves samples independently (coupled must be 0)");
  ENS_ARG_CHECK(!opts->compact, "the scalar baseline does not compact (compact must be 0)");
  ENS_ARG_CHECK(values && b && x && workspace, "null device pointer");
  ENS_ARG_CHECK(((uintptr_t)workspace & 255u) == 0, "workspace must be 256-byte aligned");
  const size_t need = ws_layout(graph->n, 1, false, nullptr, nullptr);
  if (ws_bytes < need) {
    set_error("workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    return ENS_E_NOMEM;
  }
  ENS_ARG_CHECK(lanes_per_row >= 0, "lanes_per_row must be 0 (row tiles) or 4, 8, 16, 32");
  const int G = lanes_per_row;
  Work w;
  ws_layout(graph->n, 1, false, &w, (char*)workspace);
  ens_cg_opts o = normalized(opts);
  ens_status agg = ENS_OK;
  for (int e = 0; e < s; ++e) {
    const double* ve = values + (int64_t)e * graph->nnz;
    const double* be = b + (int64_t)e * graph->n;
    double* xe = x + (int64_t)e * graph->n;
    switch (G) {
      case 0: st = cg_scalar_one<0>(graph, ve, be, xe, o, w, stream); break;
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
