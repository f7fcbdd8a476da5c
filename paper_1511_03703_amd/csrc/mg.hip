// Multigrid V-cycle for the ensemble Q1 hierarchy (Sec. 3.5, Alg. vcycle):
// setup of the coarse levels and the kernels of one cycle.  Every sample
// has its own hierarchy (the matrices, bounds and coarse inverses are
// per sample; graphs and transfers are shared), so the ensemble cycle is the
// stacked per-sample preconditioner M_c = sum_i M_i (x) e_i e_i^T.
//
// The cycle runs in FP64, or in FP32 on FP32 copies of every level's
// matrix (the preconditioner of the refinement's FP32 inner solve); the
// bounds, the Chebyshev constants and the coarse inverse stay FP64.
//
// One level of the cycle, rhs B, result OUT (x0 = 0), theta/delta of the
// per-sample Chebyshev interval [lmax/4, lmax]:
//   XA = d = D^-1 B / theta                          (elementwise)
//   d = c1 d + c2 D^-1 (B - A XA);  XB = XA + d        (row pass)
//   R = B - A XB                                       (row pass)
//   B' = P^T R on the coarse level; OUT' = cycle(B')
//   XB += P OUT'                                       (fine nodes)
//   d = D^-1 (B - A XB) / theta;  XA = XB + d          (row pass)
//   d = c1 d + c2 D^-1 (B - A XA);  OUT = XA + d       (row pass)
// with c1 = rho1 rho0, c2 = 2 rho1 / delta, rho0 = delta / theta,
// rho1 = 1 / (2 theta / delta - rho0).  The x vectors alternate between two
// buffers because every row pass gathers its input at neighbouring rows.
#include <string.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "cgcore.hpp"
#include "mg.hpp"

namespace ens {

// Hierarchies whose sample-independent part (ens_mg_build) or whole set-up
// (ens_mg_setup) is done, by buffer and shape: setting up an unbuilt buffer
// would read uninitialised graphs, so both calls refuse it.
struct MgRecord {
  const void* buffer;
  int N, M, s, fp32;
  double L;
  int stage;  // 1 built, 2 set up
  int adv;    // set up for the advection-diffusion operator (nonsymmetric)
};
static std::mutex g_mg_mu;
static std::vector<MgRecord> g_mg;

static void mg_mark(const ens_mg* mg, double L, int stage, int adv = 0) {
  std::lock_guard<std::mutex> lk(g_mg_mu);
  for (auto& r : g_mg)
    if (r.buffer == mg->buffer) {
      if (stage == 1) {
        r = MgRecord{mg->buffer, mg->N, mg->M, mg->s, mg->fp32, L, 1, 0};
      } else if (r.N == mg->N && r.M == mg->M && r.s == mg->s && r.fp32 == mg->fp32) {
        r.stage = stage;
        r.adv = adv;
      }
      return;
    }
  g_mg.push_back(MgRecord{mg->buffer, mg->N, mg->M, mg->s, mg->fp32, L, stage, adv});
}

static const MgRecord* mg_find(const ens_mg* mg) {
  for (const auto& r : g_mg)
    if (r.buffer == mg->buffer && r.N == mg->N && r.M == mg->M && r.s == mg->s && r.fp32 == mg->fp32) return &r;
  return nullptr;
}

// The stage reached by this buffer with this shape (0: none).
int mg_stage(const ens_mg* mg) {
  std::lock_guard<std::mutex> lk(g_mg_mu);
  const MgRecord* r = mg_find(mg);
  return r ? r->stage : 0;
}

// Whether the buffer is set up for a nonsymmetric (advection-diffusion)
// operator.
int mg_nonsym(const ens_mg* mg) {
  std::lock_guard<std::mutex> lk(g_mg_mu);
  const MgRecord* r = mg_find(mg);
  return r ? r->adv : 0;
}

// The correlation length the buffer was built for (0: not built).
static double mg_built_L(const ens_mg* mg) {
  std::lock_guard<std::mutex> lk(g_mg_mu);
  const MgRecord* r = mg_find(mg);
  return r ? r->L : 0.0;
}

constexpr int kMgPartRows = 8192;

static size_t r256m(size_t b) { return (b + 255) & ~(size_t)255; }

int mg_levels(int N, int* Ns) {
  int L = 0;
  Ns[L++] = N;
  while (L < kMgMaxLevels && Ns[L - 1] % 2 == 0 && Ns[L - 1] > 4) {
    Ns[L] = Ns[L - 1] / 2;
    ++L;
  }
  return L;
}

bool mg_plan(int N, int M, int S, int fp32, char* base, MgPlan* plan) {
  int Ns[kMgMaxLevels];
  plan->levels = mg_levels(N, Ns);
  plan->fp32 = fp32;
  const size_t tw = fp32 ? sizeof(float) : sizeof(double);
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += r256m(bytes);
    return p;
  };
  for (int k = 0; k < plan->levels; ++k) {
    MgLevel& l = plan->lv[k];
    l = MgLevel();
    l.N = Ns[k];
    l.n = (int64_t)(l.N + 1) * (l.N + 1) * (l.N + 1);
    l.nnz = (int64_t)(3 * l.N + 1) * (3 * l.N + 1) * (3 * l.N + 1);
    const size_t vb = (size_t)l.n * S * tw;
    if (k > 0) {
      size_t klb = 0;
      if (ens_kl_bytes(l.N, M, &klb) != ENS_OK) return false;
      l.own_rp = (int32_t*)take(sizeof(int32_t) * (l.n + 1));
      l.own_ci = (int32_t*)take(sizeof(int32_t) * l.nnz);
      l.own_vals = (double*)take(sizeof(double) * l.nnz * S);
      if (fp32) l.own_vals32 = (float*)take(sizeof(float) * l.nnz * S);
      l.kl = take(klb);
      l.rp = l.own_rp;
      l.ci = l.own_ci;
      l.vals = l.own_vals;
      l.vals32 = l.own_vals32;
      // FP64 load vector of the coarse assembly (scratch), then the cycle's rhs
      l.b = take((size_t)l.n * S * sizeof(double));
    }
    l.dinv = take(vb);
    l.lmax = (double*)take(sizeof(double) * S);
    l.xa = take(vb);
    l.xb = take(vb);
    l.r = take(vb);
    l.d = take(vb);
  }
  MgLevel& c = plan->lv[plan->levels - 1];
  c.m = (int64_t)(c.N - 1) * (c.N - 1) * (c.N - 1);
  if (c.m > kMgMaxCoarse) return false;
  c.ainv = (double*)take(sizeof(double) * S * (c.m > 0 ? c.m * c.m : 1));
  plan->part = (double*)take(sizeof(double) * kMgPartRows * S);
  // per-tile bound maxima of each level, formed by its assembly (the fine
  // level's only with ens_mg_assemble_setup)
  for (int k = 0; k < plan->levels; ++k)
    plan->lv[k].tpart = (double*)take(sizeof(double) * (size_t)asm_tiles(plan->lv[k].N, S) * S);
  plan->bytes = off;
  return true;
}

void mg_attach_fine(MgPlan* plan, const int32_t* rp, const int32_t* ci, const double* vals, const float* vals32) {
  plan->lv[0].rp = rp;
  plan->lv[0].ci = ci;
  plan->lv[0].vals = vals;
  plan->lv[0].vals32 = vals32;
}

// --------------------------------------------------------------- kernels ---

__device__ inline bool mg_idle(const Ctl* gate) { return gate && gate->n_active == 0; }

// Chebyshev constants of sample e's interval [lmax/4, lmax].
struct ChebK {
  double inv_theta, c1, c2;
};
__device__ inline ChebK cheb_consts(double lmax) {
  const double hi = lmax, lo = lmax / kMgRatio;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
  const double sigma = theta / delta;
  const double rho0 = 1.0 / sigma, rho1 = 1.0 / (2.0 * sigma - rho0);
  return ChebK{1.0 / theta, rho1 * rho0, 2.0 * rho1 / delta};
}

// One pass over the rows of the matrix the cycle runs on (FP64, or the FP32
// copy for an FP32 cycle) for D^-1 and the per-sample Gershgorin bound
// max_i sum_j |a_ij| / a_ii (row sums in ascending entry order, in FP64):
// block maxima over a grid-stride range of rows, then one block over the
// block maxima.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_mg_diag_bound(int64_t n, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci, const T* __restrict__ vals,
                                                       T* __restrict__ dinv, double* __restrict__ part) {
  constexpr int G = 256 / S;
  __shared__ double red[G][S];
  const int e = threadIdx.x % S, g = threadIdx.x / S;
  double m = 0.0;
  for (int64_t row = (int64_t)blockIdx.x * G + g; row < n; row += (int64_t)gridDim.x * G) {
    double s = 0.0, dg = 0.0;
    const int64_t k1 = rp[row + 1];
#pragma unroll 3
    for (int64_t k = rp[row]; k < k1; ++k) {
      const double v = (double)vals[k * S + e];
      s += fabs(v);
      if (ci[k] == row) dg = v;
    }
    dinv[row * S + e] = sizeof(T) == 8 ? (T)(1.0 / dg) : (T)1 / (T)dg;
    const double q = s / dg;
    m = q > m ? q : m;
  }
  red[g][e] = m;
  __syncthreads();
  if (threadIdx.x < S) {
    double t = red[0][e];
    for (int j = 1; j < G; ++j) t = red[j][e] > t ? red[j][e] : t;
    part[(int64_t)blockIdx.x * S + e] = t;
  }
}

// First stage of a long maximum: workgroup b takes the b-th contiguous
// range of rows and writes its per-sample maximum to out[b][S].
template <int S>
__global__ __launch_bounds__(1024) void k_mg_max_stage(const double* __restrict__ part, int64_t rows,
                                                       double* __restrict__ out) {
  constexpr int G = 1024 / S;
  __shared__ double red[G][S];
  const int e = threadIdx.x % S, g = threadIdx.x / S;
  const int64_t r0 = rows * blockIdx.x / gridDim.x, r1 = rows * (blockIdx.x + 1) / gridDim.x;
  double t = 0.0;
  for (int64_t r = r0 + g; r < r1; r += G) {
    const double v = part[r * S + e];
    t = v > t ? v : t;
  }
  red[g][e] = t;
  __syncthreads();
  if (threadIdx.x < S) {
    double u = red[0][e];
    for (int j = 1; j < G; ++j) u = red[j][e] > u ? red[j][e] : u;
    out[(int64_t)blockIdx.x * S + e] = u;
  }
}

// out[e] = max over `rows` partial rows: G = 1024/S threads per sample stride
// the rows, then combine in LDS (max is exact in any order).
template <int S>
__global__ __launch_bounds__(1024) void k_mg_max(const double* __restrict__ part, int rows, double* __restrict__ out) {
  constexpr int G = 1024 / S;
  __shared__ double red[G][S];
  const int e = threadIdx.x % S, g = threadIdx.x / S;
  double t = 0.0;
  for (int r = g; r < rows; r += G) {
    const double v = part[(int64_t)r * S + e];
    t = v > t ? v : t;
  }
  red[g][e] = t;
  __syncthreads();
  if (threadIdx.x < S) {
    double u = red[0][e];
    for (int j = 1; j < G; ++j) u = red[j][e] > u ? red[j][e] : u;
    out[e] = u;
  }
}

// Dense inverse of sample e's interior block of the coarsest matrix, by
// Gauss-Jordan elimination in place without pivoting: the block's symmetric
// part is positive definite (the diffusion block; with advection the
// interior block of C is skew-symmetric and adds nothing to it), so the
// diagonal pivots are positive.  One workgroup per sample.
template <int S>
__global__ __launch_bounds__(256) void k_mg_inverse(int N, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci, const double* __restrict__ vals,
                                                    int64_t m, double* __restrict__ ainv) {
  __shared__ double f[kMgMaxCoarse];
  const int e = blockIdx.x;
  double* A = ainv + (int64_t)e * m * m;
  const int I = N - 1;  // interior nodes per axis
  for (int64_t t = threadIdx.x; t < m * m; t += blockDim.x) A[t] = 0.0;
  __syncthreads();
  for (int64_t a = threadIdx.x; a < m; a += blockDim.x) {
    const int i = 1 + (int)(a % I), j = 1 + (int)((a / I) % I), k = 1 + (int)(a / ((int64_t)I * I));
    const int64_t row = i + (int64_t)(N + 1) * (j + (int64_t)(N + 1) * k);
    for (int64_t q = rp[row]; q < rp[row + 1]; ++q) {
      const int64_t col = ci[q];
      const int ci_ = (int)(col % (N + 1)), cj = (int)((col / (N + 1)) % (N + 1)), ck = (int)(col / ((int64_t)(N + 1) * (N + 1)));
      if (ci_ == 0 || cj == 0 || ck == 0 || ci_ == N || cj == N || ck == N) continue;
      const int64_t b = (ci_ - 1) + (int64_t)I * ((cj - 1) + (int64_t)I * (ck - 1));
      A[a * m + b] = vals[q * S + e];
    }
  }
  __syncthreads();
  for (int64_t p = 0; p < m; ++p) {
    const double piv = A[p * m + p];
    __syncthreads();
    for (int64_t j = threadIdx.x; j < m; j += blockDim.x) A[p * m + j] = (j == p ? 1.0 : A[p * m + j]) / piv;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) f[i] = A[i * m + p];
    __syncthreads();
    for (int64_t t = threadIdx.x; t < m * m; t += blockDim.x) {
      const int64_t i = t / m, j = t % m;
      if (i == p) continue;
      A[t] = (j == p ? 0.0 : A[t]) - f[i] * A[p * m + j];
    }
    __syncthreads();
  }
}

// d = D^-1 B / theta, the first Chebyshev step from x = 0, whose iterate
// x = 0 + d is d itself (the next step reads it as its x).
template <typename T, int S>
__global__ __launch_bounds__(256) void k_mg_cheb0(int64_t nchunks, const T* __restrict__ b,
                                                  const T* __restrict__ dinv, const double* __restrict__ lmax,
                                                  T* __restrict__ d, const Ctl* gate) {
  if (mg_idle(gate)) return;
  using VM = VecMap<T, S>;
  using vt = typename VM::vt;
  const int sub = (threadIdx.x & 63) % VM::L;
  vt it;
#pragma unroll
  for (int v = 0; v < VM::V; ++v) it[v] = (T)cheb_consts(lmax[VM::sample(sub, v)]).inv_theta;
  const int64_t base = (int64_t)blockIdx.x * kBlock * kU + threadIdx.x;
  vt bv[kU], dv[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int64_t i = base + u * kBlock;
    if (i < nchunks) {
      bv[u] = load_stream((const vt*)b + i);
      dv[u] = load_stream((const vt*)dinv + i);
    }
  }
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int64_t i = base + u * kBlock;
    if (i < nchunks) {
      store_stream((vt*)d + i, dv[u] * bv[u] * it);
    }
  }
}

enum MgRowMode { MG_RES = 0, MG_CHEB1 = 1, MG_CHEB2 = 2 };

// Row passes of the cycle (one row tile of 4 wavefronts per block):
//   MG_RES:   r = B - A x
//   MG_CHEB1: d = D^-1 (B - A x) / theta;           xout = x + d
//   MG_CHEB2: d' = c1 d + c2 D^-1 (B - A x);         xout = x + d'
// MG_CHEB2 is the last step of the order-2 smoother, so d' is not stored
// (nothing reads it: the next smoothing sweep starts a new direction).
// DOT (the cycle's very last pass, on the finest level, inside CG): the
// block's per-sample partials of B . xout, i.e. r . z with z = M r, go to
// dot[blockIdx.x][S], so CG needs no separate pass over r and z.
template <typename T, int S, int MODE, bool DOT = false>
__global__ __launch_bounds__(256) void k_mg_row(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                const T* __restrict__ vals, const T* __restrict__ x,
                                                const T* __restrict__ b, const T* __restrict__ dinv,
                                                const double* __restrict__ lmax, T* __restrict__ d,
                                                T* __restrict__ out, const Ctl* gate, double* __restrict__ dot) {
  static_assert(!DOT || MODE == MG_CHEB2, "the dot is formed in the smoother's last step");
  if (mg_idle(gate)) return;
  using M = EnsMap<T, S>;
  using vt = typename M::vt;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane % M::L;
  const int64_t row = ((int64_t)blockIdx.x * 4 + wave) * M::RPW + lane / M::L;
  constexpr int R = 4 * M::RPW;
  __shared__ RowTileLds<R> tile;
  const bool staged = stage_row_tile(tile, n, rp, ci, (int64_t)blockIdx.x * R);
  double acc[1][M::V];
#pragma unroll
  for (int v = 0; v < M::V; ++v) acc[0][v] = 0.0;
  if (row < n) {
    const vt ax =
        tile_row_product<T, S>(tile, staged, (int)(row - (int64_t)blockIdx.x * R), ci, vals, x, sub);
    const int64_t i = row * M::L + sub;
    const vt bv = load_stream((const vt*)b + i);
    const vt res = bv - ax;
    if (MODE == MG_RES) {
      store_stream((vt*)out + i, res);
      return;
    }
    vt k1, k2;
#pragma unroll
    for (int v = 0; v < M::V; ++v) {
      const ChebK c = cheb_consts(lmax[sub * M::V + v]);
      k1[v] = (T)(MODE == MG_CHEB1 ? 0.0 : c.c1);
      k2[v] = (T)(MODE == MG_CHEB1 ? c.inv_theta : c.c2);
    }
    const vt dv = load_stream((const vt*)dinv + i) * res;
    vt dn;
    if (MODE == MG_CHEB1) dn = k2 * dv;
    else dn = k1 * load_stream((const vt*)d + i) + k2 * dv;
    if (MODE == MG_CHEB1) store_stream((vt*)d + i, dn);
    const vt xn = ((const vt*)x)[i] + dn;
    store_stream((vt*)out + i, xn);
    if (DOT) {
#pragma unroll
      for (int v = 0; v < M::V; ++v) acc[0][v] = (double)bv[v] * (double)xn[v];
    }
  }
  if (DOT) block_partials<S, M::V, 1, 4>(acc, dot + (int64_t)blockIdx.x * S);
}

// Coarse interior node c collects the residual of the fine interior nodes
// around fine node 2c (weight 1 on the axis, 1/2 one step off), in a fixed
// order; coarse boundary nodes get 0.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_mg_restrict(int Nc, const T* __restrict__ rf, T* __restrict__ bc,
                                                     const Ctl* gate) {
  if (mg_idle(gate)) return;
  using VM = VecMap<T, S>;
  using vt = typename VM::vt;
  const int Nf = 2 * Nc;
  const int64_t nc = (int64_t)(Nc + 1) * (Nc + 1) * (Nc + 1);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * VM::L) return;
  const int64_t node = t / VM::L;
  const int sub = (int)(t % VM::L);
  const int I = (int)(node % (Nc + 1)), J = (int)((node / (Nc + 1)) % (Nc + 1)), K = (int)(node / ((int64_t)(Nc + 1) * (Nc + 1)));
  vt acc = (vt)0;
  if (I > 0 && J > 0 && K > 0 && I < Nc && J < Nc && K < Nc) {
    for (int dk = -1; dk <= 1; ++dk)
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
          const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
          if (i <= 0 || j <= 0 || k <= 0 || i >= Nf || j >= Nf || k >= Nf) continue;
          const T w = (T)((di ? 0.5 : 1.0) * (dj ? 0.5 : 1.0) * (dk ? 0.5 : 1.0));
          const int64_t f = i + (int64_t)(Nf + 1) * (j + (int64_t)(Nf + 1) * k);
          acc += w * ((const vt*)rf)[f * VM::L + sub];
        }
  }
  ((vt*)bc)[t] = acc;
}

// Fine interior node: xf += sum of its interior coarse parents with the
// trilinear weights.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_mg_prolong(int Nc, const T* __restrict__ xc, T* __restrict__ xf,
                                                    const Ctl* gate) {
  if (mg_idle(gate)) return;
  using VM = VecMap<T, S>;
  using vt = typename VM::vt;
  const int Nf = 2 * Nc;
  const int64_t nf = (int64_t)(Nf + 1) * (Nf + 1) * (Nf + 1);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nf * VM::L) return;
  const int64_t node = t / VM::L;
  const int sub = (int)(t % VM::L);
  const int i = (int)(node % (Nf + 1)), j = (int)((node / (Nf + 1)) % (Nf + 1)), k = (int)(node / ((int64_t)(Nf + 1) * (Nf + 1)));
  if (i == 0 || j == 0 || k == 0 || i == Nf || j == Nf || k == Nf) return;
  int Ii[2], Jj[2], Kk[2];
  double wi[2], wj[2], wk[2];
  auto parents = [](int q, int* P, double* w) -> int {
    if (q % 2 == 0) {
      P[0] = q / 2;
      w[0] = 1.0;
      return 1;
    }
    P[0] = (q - 1) / 2;
    w[0] = 0.5;
    P[1] = (q + 1) / 2;
    w[1] = 0.5;
    return 2;
  };
  const int ni = parents(i, Ii, wi), nj = parents(j, Jj, wj), nk = parents(k, Kk, wk);
  vt acc = (vt)0;
  for (int c = 0; c < nk; ++c)
    for (int bq = 0; bq < nj; ++bq)
      for (int a = 0; a < ni; ++a) {
        const int I = Ii[a], J = Jj[bq], K = Kk[c];
        if (I == 0 || J == 0 || K == 0 || I == Nc || J == Nc || K == Nc) continue;
        const int64_t cn = I + (int64_t)(Nc + 1) * (J + (int64_t)(Nc + 1) * K);
        acc += (T)(wi[a] * wj[bq] * wk[c]) * ((const vt*)xc)[cn * VM::L + sub];
      }
  store_stream((vt*)xf + t, load_stream((const vt*)xf + t) + acc);
}

// Coarsest level: boundary rows are identities (x = B), interior rows take
// the per-sample dense inverse.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_mg_coarse(int Nc, int64_t m, const double* __restrict__ ainv,
                                                   const T* __restrict__ b, T* __restrict__ x, const Ctl* gate) {
  if (mg_idle(gate)) return;
  const int64_t n = (int64_t)(Nc + 1) * (Nc + 1) * (Nc + 1);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * S) return;
  const int64_t node = t / S;
  const int e = (int)(t % S);
  const int i = (int)(node % (Nc + 1)), j = (int)((node / (Nc + 1)) % (Nc + 1)), k = (int)(node / ((int64_t)(Nc + 1) * (Nc + 1)));
  if (i == 0 || j == 0 || k == 0 || i == Nc || j == Nc || k == Nc) {
    x[t] = b[t];
    return;
  }
  const int I = Nc - 1;
  const int64_t a = (i - 1) + (int64_t)I * ((j - 1) + (int64_t)I * (k - 1));
  const double* row = ainv + ((int64_t)e * m + a) * m;
  double acc = 0.0;
  for (int64_t c = 0; c < m; ++c) {
    const int ii = 1 + (int)(c % I), jj = 1 + (int)((c / I) % I), kk = 1 + (int)(c / ((int64_t)I * I));
    const int64_t cn = ii + (int64_t)(Nc + 1) * (jj + (int64_t)(Nc + 1) * kk);
    acc += row[c] * (double)b[cn * S + e];
  }
  x[t] = (T)acc;
}

// Galerkin coarse operator of Alg. vcycle, A_c = P^T A_f P with R = P^T, P
// the trilinear interpolation of k_mg_prolong.  Lane e of a group of S
// lanes forms the 27 entries of one coarse row for sample e:
//   (P^T A P)_{IJ} = sum_i P_{iI} sum_j A_ij P_{jJ}.
// For an interior coarse node I the fine children are i = 2I + o,
// o in {-1,0,1}^3 (all interior, weight prod (o ? 1/2 : 1)); row i holds the
// 27 neighbours j = i + d, and a fine node j = 2I + t, t = o + d, has the
// coarse parents I + t/2 (t even, weight 1) or I + (t-1)/2 and I + (t+1)/2
// (t odd, 1/2 each).  With o, d and t known at compile time every term goes
// to a fixed one of 27 register accumulators, indexed by the parent's offset
// from I, and every weight product is a power of two, so each term
// A_ij * w is exact and only the additions round; they run in the order
// children (z, y, x ascending), row entries ascending, parents (z, y, x,
// ascending).  Terms through a coarse boundary parent land in that
// parent's accumulator and are dropped at the store: boundary columns of
// interior rows are stored zeros and boundary rows identity rows, as on
// the assembled levels (P has no boundary columns).  Interior rows of
// every level hold the full 3x3x3 neighbour block in ascending order.
// Workgroups of consecutive rows are dealt to the 8 XCDs in contiguous
// ranges, so the fine rows that neighbouring coarse rows share are read
// through one L2.
__device__ inline int64_t xcd_contiguous_block(int64_t b, int64_t nb) {
  const int64_t per = nb / 8, rem = nb % 8, x = b % 8, k = b / 8;
  return x * per + (x < rem ? x : rem) + k;
}

// An empty asm that reads and writes every accumulator: a point every term
// so far must have reached.
template <int T>
__device__ __forceinline__ void acc_fence(double (&acc)[27]) {
  if constexpr (T < 27) {
    asm volatile("" : "+v"(acc[T]));
    acc_fence<T + 1>(acc);
  }
}

// The terms of fine child i = 2I + (OX, OY, OZ) (row `a`, this lane's
// sample) in entry order, then the fence: the compiler otherwise orders the
// work by accumulator and keeps all 729 loaded values of a row live.
template <int C, int S>
__device__ __forceinline__ void galerkin_children(double (&acc)[27], int I, int J, int K, int64_t pf,
                                                  const int32_t* __restrict__ rpf, const double* __restrict__ vf,
                                                  int e) {
  if constexpr (C < 27) {
    constexpr int OX = C % 3 - 1, OY = (C / 3) % 3 - 1, OZ = C / 9 - 1;
    constexpr double wi = (OX ? 0.5 : 1.0) * (OY ? 0.5 : 1.0) * (OZ ? 0.5 : 1.0);
    const int64_t i = (2 * I + OX) + pf * ((2 * J + OY) + pf * (2 * K + OZ));
    const double* a = vf + (int64_t)rpf[i] * S + e;
    double av[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) av[q] = a[q * S];
#pragma unroll
    for (int q = 0; q < 27; ++q) {
      const int dx = q % 3 - 1, dy = (q / 3) % 3 - 1, dz = q / 9 - 1;
      const int tz = OZ + dz, ty = OY + dy, tx = OX + dx;
      // parents per axis: count, first offset from I; weight
      const int nz = (tz & 1) ? 2 : 1, ny = (ty & 1) ? 2 : 1, nx = (tx & 1) ? 2 : 1;
      const int fz = (tz & 1) ? (tz - 1) / 2 : tz / 2, fy = (ty & 1) ? (ty - 1) / 2 : ty / 2,
                fx = (tx & 1) ? (tx - 1) / 2 : tx / 2;
      const double wt = wi * ((nz == 2 ? 0.5 : 1.0) * (ny == 2 ? 0.5 : 1.0) * (nx == 2 ? 0.5 : 1.0));
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int p = 0; p < 2; ++p) {
            if (c >= nz || b >= ny || p >= nx) continue;
            acc[(fz + c + 1) * 9 + (fy + b + 1) * 3 + (fx + p + 1)] += av[q] * wt;
          }
    }
    acc_fence<0>(acc);
    galerkin_children<C + 1, S>(acc, I, J, K, pf, rpf, vf, e);
  }
}

template <int S>
__global__ __launch_bounds__(256) void k_mg_galerkin(int Nc, const int32_t* __restrict__ rpf,
                                                     const double* __restrict__ vf, const int32_t* __restrict__ rpc,
                                                     const int32_t* __restrict__ cic, double* __restrict__ vc,
                                                     float* __restrict__ vc32) {
  constexpr int G = 256 / S;
  const int e = threadIdx.x % S;
  const int64_t nc = (int64_t)(Nc + 1) * (Nc + 1) * (Nc + 1);
  const int64_t row = xcd_contiguous_block(blockIdx.x, gridDim.x) * G + threadIdx.x / S;
  if (row >= nc) return;
  const int I = (int)(row % (Nc + 1)), J = (int)((row / (Nc + 1)) % (Nc + 1)),
            K = (int)(row / ((int64_t)(Nc + 1) * (Nc + 1)));
  const int64_t q0 = rpc[row];
  if (I == 0 || J == 0 || K == 0 || I == Nc || J == Nc || K == Nc) {
    const int64_t q1 = rpc[row + 1];
    for (int64_t q = q0; q < q1; ++q) {
      const double v = cic[q] == row ? 1.0 : 0.0;
      vc[q * S + e] = v;
      if (vc32) vc32[q * S + e] = (float)v;
    }
    return;
  }
  double acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = 0.0;
  galerkin_children<0, S>(acc, I, J, K, (int64_t)2 * Nc + 1, rpf, vf, e);
#pragma unroll
  for (int q = 0; q < 27; ++q) {
    const int dx = q % 3 - 1, dy = (q / 3) % 3 - 1, dz = q / 9 - 1;
    const bool bnd = I + dx == 0 || I + dx == Nc || J + dy == 0 || J + dy == Nc || K + dz == 0 || K + dz == Nc;
    const double v = bnd ? 0.0 : acc[q];
    vc[(q0 + q) * S + e] = v;
    if (vc32) vc32[(q0 + q) * S + e] = (float)v;
  }
}

// ------------------------------------------------------------ host side ---

static unsigned blocks_for(int64_t items, int64_t per) {
  const int64_t b = (items + per - 1) / per;
  return (unsigned)(b < 1 ? 1 : b);
}

template <typename T, int S>
static void cycle(const MgPlan& P, int k, const T* B, T* OUT, const Ctl* gate, hipStream_t st,
                  double* dot = nullptr) {
  using EM = EnsMap<T, S>;
  using VM = VecMap<T, S>;
  const MgLevel& l = P.lv[k];
  const T* vals = sizeof(T) == 4 ? (const T*)l.vals32 : (const T*)l.vals;
  const T* dinv = (const T*)l.dinv;
  T *xa = (T*)l.xa, *xb = (T*)l.xb, *r = (T*)l.r, *d = (T*)l.d;
  if (k == P.levels - 1) {
    hipLaunchKernelGGL((k_mg_coarse<T, S>), dim3(blocks_for(l.n * S, 256)), dim3(256), 0, st, l.N, l.m, l.ainv, B,
                       OUT, gate);
    return;
  }
  const MgLevel& c = P.lv[k + 1];
  T* cb = (T*)c.b;
  T* cx = (T*)c.xb;
  const int64_t nchunks = l.n * S / VM::V;
  const unsigned rb = blocks_for(l.n, 4 * EM::RPW);
  // algorithmic bytes of the fine row passes: the matrix and the gathered
  // x once, plus (vectors read + written) x n x S x sizeof(T)
  const double mat = (double)l.nnz * (S * (double)sizeof(T) + 4.0) + 4.0 * (l.n + 1);
  const double vec = (double)l.n * S * sizeof(T);
  const bool fine = k == 0;
  hipLaunchKernelGGL((k_mg_cheb0<T, S>), dim3(blocks_for(nchunks, (int64_t)kBlock * kU)), dim3(kBlock), 0, st,
                     nchunks, B, dinv, l.lmax, d, gate);
  if (fine) prof_begin(ENS_K_MG_ROW, st);
  hipLaunchKernelGGL((k_mg_row<T, S, MG_CHEB2>), dim3(rb), dim3(256), 0, st, (int)l.n, l.rp, l.ci, vals, d, B, dinv,
                     l.lmax, d, xb, gate, (double*)nullptr);
  if (fine) prof_end(ENS_K_MG_ROW, st, mat + 4.0 * vec);  // x is d: one vector read less
  if (fine) prof_begin(ENS_K_MG_ROW, st);
  hipLaunchKernelGGL((k_mg_row<T, S, MG_RES>), dim3(rb), dim3(256), 0, st, (int)l.n, l.rp, l.ci, vals, xb, B, dinv,
                     l.lmax, d, r, gate, (double*)nullptr);
  if (fine) prof_end(ENS_K_MG_ROW, st, mat + 3.0 * vec);
  hipLaunchKernelGGL((k_mg_restrict<T, S>), dim3(blocks_for(c.n * VM::L, 256)), dim3(256), 0, st, c.N, r, cb, gate);
  cycle<T, S>(P, k + 1, cb, cx, gate, st);
  hipLaunchKernelGGL((k_mg_prolong<T, S>), dim3(blocks_for(l.n * VM::L, 256)), dim3(256), 0, st, c.N, cx, xb, gate);
  if (fine) prof_begin(ENS_K_MG_ROW, st);
  hipLaunchKernelGGL((k_mg_row<T, S, MG_CHEB1>), dim3(rb), dim3(256), 0, st, (int)l.n, l.rp, l.ci, vals, xb, B, dinv,
                     l.lmax, d, xa, gate, (double*)nullptr);
  if (fine) prof_end(ENS_K_MG_ROW, st, mat + 5.0 * vec);
  if (fine) prof_begin(ENS_K_MG_ROW, st);
  if (dot && fine)
    hipLaunchKernelGGL((k_mg_row<T, S, MG_CHEB2, true>), dim3(rb), dim3(256), 0, st, (int)l.n, l.rp, l.ci, vals, xa,
                       B, dinv, l.lmax, d, OUT, gate, dot);
  else
    hipLaunchKernelGGL((k_mg_row<T, S, MG_CHEB2>), dim3(rb), dim3(256), 0, st, (int)l.n, l.rp, l.ci, vals, xa, B,
                       dinv, l.lmax, d, OUT, gate, (double*)nullptr);
  if (fine) prof_end(ENS_K_MG_ROW, st, mat + 5.0 * vec);
}

template <typename T, int S>
void mg_vcycle(const MgPlan& plan, const T* r, T* z, const Ctl* gate, hipStream_t st, double* dot) {
  cycle<T, S>(plan, 0, r, z, gate, st, dot);
}

#define ENS_MG_INST(T, S) \
  template void mg_vcycle<T, S>(const MgPlan&, const T*, T*, const Ctl*, hipStream_t, double*);
ENS_MG_INST(double, 4)
ENS_MG_INST(double, 8)
ENS_MG_INST(double, 16)
ENS_MG_INST(double, 32)
ENS_MG_INST(float, 4)
ENS_MG_INST(float, 8)
ENS_MG_INST(float, 16)
ENS_MG_INST(float, 32)
#undef ENS_MG_INST

static ens_status build(const MgPlan& P, int M, double L, hipStream_t st) {
  for (int k = 1; k < P.levels; ++k) {
    const MgLevel& l = P.lv[k];
    ens_status rc = ens_graph_build(l.N, l.own_rp, l.own_ci, st);
    if (rc == ENS_OK) rc = ens_kl_build(l.N, M, L, l.kl, st);
    if (rc != ENS_OK) return rc;
  }
  return ENS_OK;
}

// Level bound from the per-tile maxima its assembly wrote: the maximum in
// two stages (exact in any order).
template <int S>
static void tile_bound(const MgPlan& P, const MgLevel& l, hipStream_t st) {
  const int64_t rows = asm_tiles(l.N, S);
  int64_t g1 = rows / 256;
  if (g1 < 1) g1 = 1;
  if (g1 > 256) g1 = 256;
  hipLaunchKernelGGL(k_mg_max_stage<S>, dim3((unsigned)g1), dim3(1024), 0, st, l.tpart, rows, P.part);
  hipLaunchKernelGGL(k_mg_max<S>, dim3(1), dim3(1024), 0, st, P.part, (int)g1, l.lmax);
}

// D^-1 and the bound of a level by a pass over the matrix the cycle runs
// on there (the FP32 copy for an FP32 cycle).
template <int S>
static void row_bound(const MgPlan& P, const MgLevel& l, hipStream_t st) {
  const unsigned gb = blocks_for(l.n, 256 / S) < (unsigned)kMgPartRows ? blocks_for(l.n, 256 / S) : kMgPartRows;
  if (P.fp32)
    hipLaunchKernelGGL((k_mg_diag_bound<float, S>), dim3(gb), dim3(256), 0, st, l.n, l.rp, l.ci, l.vals32,
                       (float*)l.dinv, P.part);
  else
    hipLaunchKernelGGL((k_mg_diag_bound<double, S>), dim3(gb), dim3(256), 0, st, l.n, l.rp, l.ci, l.vals,
                       (double*)l.dinv, P.part);
  hipLaunchKernelGGL(k_mg_max<S>, dim3(1), dim3(1024), 0, st, P.part, (int)gb, l.lmax);
}

template <int S>
static void coarsest_inverse(const MgPlan& P, hipStream_t st) {
  const MgLevel& c = P.lv[P.levels - 1];
  if (c.m > 0)
    hipLaunchKernelGGL(k_mg_inverse<S>, dim3(S), dim3(256), 0, st, c.N, c.rp, c.ci, c.vals, c.m, c.ainv);
}

// fine_done: the fine level's D^-1 and per-tile bound maxima were formed by
// its assembly (ens_mg_assemble_setup); only their maximum is taken here.
// adv (nullable): {alpha, vx, vy, vz} of the advection-diffusion operator
// every coarse level is rediscretized with.
template <int S>
static ens_status setup(const MgPlan& P, const ens_problem& prob, const double* xi, hipStream_t st,
                        bool fine_done = false, const double* adv = nullptr) {
  for (int k = 0; k < P.levels; ++k) {
    const MgLevel& l = P.lv[k];
    if (k > 0) {
      // the coarse operator, with its D^-1 and per-tile bounds formed by the
      // assembly
      ens_graph g{(int32_t)l.n, l.nnz, l.own_rp, l.own_ci};
      const double *sq = nullptr, *phi = nullptr;
      const int32_t* tr = nullptr;
      kl_parts(l.kl, prob.M, &sq, &tr, &phi);
      ens_status rc = assemble_launch(l.N, &g, sq, tr, phi, &prob, S, xi, l.own_vals, l.own_vals32, (double*)l.b,
                                      P.fp32 ? 1 : 2, l.dinv, l.tpart, st, adv);
      if (rc != ENS_OK) return rc;
    }
    if (k > 0 || fine_done) tile_bound<S>(P, l, st);
    else row_bound<S>(P, l, st);
  }
  coarsest_inverse<S>(P, st);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

// Coarse levels as Galerkin products P^T A P of the level above, formed in
// FP64 from its FP64 matrix (an FP32 cycle's copy rounded from them), D^-1
// and bounds by a pass over each coarse level's cycle matrix, the coarsest
// inverse.  fine_done: the fine level's D^-1 and per-tile maxima came from
// its assembly.  The fine FP64 matrix must be attached.
template <int S>
static ens_status setup_galerkin(const MgPlan& P, hipStream_t st, bool fine_done) {
  for (int k = 0; k < P.levels; ++k) {
    const MgLevel& l = P.lv[k];
    if (k > 0) {
      const MgLevel& f = P.lv[k - 1];
      hipLaunchKernelGGL(k_mg_galerkin<S>, dim3(blocks_for(l.n, 256 / S)), dim3(256), 0, st, l.N, f.rp, f.vals,
                         l.rp, l.ci, l.own_vals, P.fp32 ? l.own_vals32 : nullptr);
    }
    if (k == 0 && fine_done) tile_bound<S>(P, l, st);
    else row_bound<S>(P, l, st);
  }
  coarsest_inverse<S>(P, st);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

}  // namespace ens

using namespace ens;

extern "C" {

ens_status ens_mg_bytes(int32_t N, int32_t M, int32_t s, int32_t fp32, size_t* bytes) {
  ENS_ARG_CHECK(bytes && N >= 1 && M >= 0, "bad multigrid arguments");
  if (!supported_s(s)) {
    set_error("ensemble size %d not compiled in", s);
    return ENS_E_UNSUPPORTED;
  }
  MgPlan plan;
  if (!mg_plan(N, M, s, fp32 != 0, nullptr, &plan)) {
    set_error("coarsest multigrid level of N=%d has more than %lld interior unknowns", N, (long long)kMgMaxCoarse);
    return ENS_E_UNSUPPORTED;
  }
  *bytes = plan.bytes;
  return ENS_OK;
}

ens_status ens_mg_build(const ens_mg* mg, double L, hipStream_t stream) {
  ENS_ARG_CHECK(mg && mg->buffer, "null multigrid argument");
  ENS_ARG_CHECK(((uintptr_t)mg->buffer & 255u) == 0, "multigrid buffer must be 256-byte aligned");
  ENS_ARG_CHECK(L > 0.0, "correlation length must be positive");
  size_t need = 0;
  ens_status rc = ens_mg_bytes(mg->N, mg->M, mg->s, mg->fp32, &need);
  if (rc != ENS_OK) return rc;
  if (mg->bytes < need) {
    set_error("multigrid buffer of %zu bytes is smaller than the %zu required", mg->bytes, need);
    return ENS_E_NOMEM;
  }
  MgPlan plan;
  mg_plan(mg->N, mg->M, mg->s, mg->fp32 != 0, (char*)mg->buffer, &plan);
  rc = build(plan, mg->M, L, stream);
  if (rc == ENS_OK) ENS_LAUNCH_CHECK();
  if (rc == ENS_OK) mg_mark(mg, L, 1);
  return rc;
}

ens_status ens_mg_setup(const ens_mg* mg, const ens_graph* graph, const double* values, const float* values32,
                        const ens_problem* problem, const double* xi, hipStream_t stream) {
  ENS_ARG_CHECK(mg && graph && values && problem && xi && mg->buffer, "null multigrid argument");
  ENS_ARG_CHECK(((uintptr_t)mg->buffer & 255u) == 0, "multigrid buffer must be 256-byte aligned");
  ENS_ARG_CHECK(aligned16(values), "values must be 16-byte aligned");
  ENS_ARG_CHECK(!mg->fp32 || (values32 && aligned16(values32)), "an FP32 cycle needs the FP32 fine matrix");
  ENS_ARG_CHECK(problem->M == mg->M, "problem->M differs from the hierarchy's M");
  const int64_t n = (int64_t)(mg->N + 1) * (mg->N + 1) * (mg->N + 1);
  ENS_ARG_CHECK(graph->n == n && graph->row_ptr && graph->col_idx, "graph is not the N^3 mesh's graph");
  MgPlan plan;
  size_t need = 0;
  ens_status rc = ens_mg_bytes(mg->N, mg->M, mg->s, mg->fp32, &need);
  if (rc != ENS_OK) return rc;
  if (mg->bytes < need) {
    set_error("multigrid buffer of %zu bytes is smaller than the %zu required", mg->bytes, need);
    return ENS_E_NOMEM;
  }
  const double Lb = mg_built_L(mg);
  if (Lb <= 0.0) {
    set_error("multigrid buffer not built: call ens_mg_build first");
    return ENS_E_ARG;
  }
  ENS_ARG_CHECK(problem->L == Lb, "problem->L differs from the correlation length the hierarchy was built for");
  mg_plan(mg->N, mg->M, mg->s, mg->fp32 != 0, (char*)mg->buffer, &plan);
  mg_attach_fine(&plan, graph->row_ptr, graph->col_idx, values, mg->fp32 ? values32 : nullptr);
  switch (mg->s) {
    case 4: rc = setup<4>(plan, *problem, xi, stream); break;
    case 8: rc = setup<8>(plan, *problem, xi, stream); break;
    case 16: rc = setup<16>(plan, *problem, xi, stream); break;
    default: rc = setup<32>(plan, *problem, xi, stream); break;
  }
  if (rc == ENS_OK) mg_mark(mg, Lb, 2);
  return rc;
}

static ens_status assemble_setup(const ens_mg* mg, const ens_graph* graph, const void* kl,
                                 const ens_problem* problem, const double* adv, const double* xi, double* values,
                                 float* values32, double* rhs, hipStream_t stream, bool galerkin = false) {
  ENS_ARG_CHECK(mg && graph && kl && problem && xi && rhs && mg->buffer, "null argument");
  ENS_ARG_CHECK(values || mg->fp32, "an FP64 hierarchy needs the FP64 fine matrix");
  ENS_ARG_CHECK(values || !galerkin, "Galerkin coarse levels need the FP64 fine matrix");
  ENS_ARG_CHECK(((uintptr_t)mg->buffer & 255u) == 0, "multigrid buffer must be 256-byte aligned");
  ENS_ARG_CHECK((!values || aligned16(values)) && aligned16(rhs), "values and rhs must be 16-byte aligned");
  ENS_ARG_CHECK(!mg->fp32 || (values32 && aligned16(values32)), "an FP32 cycle needs the FP32 fine matrix");
  ENS_ARG_CHECK(problem->M == mg->M && problem->M >= 0 && problem->M <= 16, "problem->M differs or is out of range");
  int64_t n = 0, nnz = 0;
  ens_status rc = ens_mesh_sizes(mg->N, &n, &nnz, nullptr);
  if (rc != ENS_OK) return rc;
  ENS_ARG_CHECK(graph->n == n && graph->nnz == nnz && graph->row_ptr && graph->col_idx,
                "graph is not the N^3 mesh's graph");
  size_t need = 0;
  rc = ens_mg_bytes(mg->N, mg->M, mg->s, mg->fp32, &need);
  if (rc != ENS_OK) return rc;
  if (mg->bytes < need) {
    set_error("multigrid buffer of %zu bytes is smaller than the %zu required", mg->bytes, need);
    return ENS_E_NOMEM;
  }
  const double Lb = mg_built_L(mg);
  if (Lb <= 0.0) {
    set_error("multigrid buffer not built: call ens_mg_build first");
    return ENS_E_ARG;
  }
  ENS_ARG_CHECK(problem->L == Lb, "problem->L differs from the correlation length the hierarchy was built for");
  MgPlan plan;
  mg_plan(mg->N, mg->M, mg->s, mg->fp32 != 0, (char*)mg->buffer, &plan);
  // a one-level hierarchy inverts the fine matrix itself, in FP64
  ENS_ARG_CHECK(values || plan.levels > 1, "a one-level hierarchy needs the FP64 fine matrix");
  mg_attach_fine(&plan, graph->row_ptr, graph->col_idx, values, mg->fp32 ? values32 : nullptr);
  const double *sq = nullptr, *phi = nullptr;
  const int32_t* tr = nullptr;
  kl_parts(kl, problem->M, &sq, &tr, &phi);
  rc = assemble_launch(mg->N, graph, sq, tr, phi, problem, mg->s, xi, values, values32, rhs, mg->fp32 ? 1 : 2,
                       plan.lv[0].dinv, plan.lv[0].tpart, stream, adv);
  if (rc != ENS_OK) return rc;
  if (galerkin) switch (mg->s) {
      case 4: rc = setup_galerkin<4>(plan, stream, true); break;
      case 8: rc = setup_galerkin<8>(plan, stream, true); break;
      case 16: rc = setup_galerkin<16>(plan, stream, true); break;
      default: rc = setup_galerkin<32>(plan, stream, true); break;
    }
  else switch (mg->s) {
      case 4: rc = setup<4>(plan, *problem, xi, stream, true, adv); break;
      case 8: rc = setup<8>(plan, *problem, xi, stream, true, adv); break;
      case 16: rc = setup<16>(plan, *problem, xi, stream, true, adv); break;
      default: rc = setup<32>(plan, *problem, xi, stream, true, adv); break;
    }
  if (rc == ENS_OK) mg_mark(mg, Lb, 2, adv && adv[0] != 0.0 ? 1 : 0);
  return rc;
}

ens_status ens_mg_assemble_setup(const ens_mg* mg, const ens_graph* graph, const void* kl,
                                 const ens_problem* problem, const double* xi, double* values, float* values32,
                                 double* rhs, hipStream_t stream) {
  return assemble_setup(mg, graph, kl, problem, nullptr, xi, values, values32, rhs, stream);
}

ens_status ens_mg_assemble_setup_galerkin(const ens_mg* mg, const ens_graph* graph, const void* kl,
                                          const ens_problem* problem, const double* xi, double* values,
                                          float* values32, double* rhs, hipStream_t stream) {
  return assemble_setup(mg, graph, kl, problem, nullptr, xi, values, values32, rhs, stream, true);
}

ens_status ens_mg_setup_galerkin(const ens_mg* mg, const ens_graph* graph, const double* values,
                                 const float* values32, hipStream_t stream) {
  ENS_ARG_CHECK(mg && graph && values && mg->buffer, "null multigrid argument");
  ENS_ARG_CHECK(((uintptr_t)mg->buffer & 255u) == 0, "multigrid buffer must be 256-byte aligned");
  ENS_ARG_CHECK(aligned16(values), "values must be 16-byte aligned");
  ENS_ARG_CHECK(!mg->fp32 || (values32 && aligned16(values32)), "an FP32 cycle needs the FP32 fine matrix");
  int64_t n = 0, nnz = 0;
  ens_status rc = ens_mesh_sizes(mg->N, &n, &nnz, nullptr);
  if (rc != ENS_OK) return rc;
  ENS_ARG_CHECK(graph->n == n && graph->nnz == nnz && graph->row_ptr && graph->col_idx,
                "graph is not the N^3 mesh's graph");
  size_t need = 0;
  rc = ens_mg_bytes(mg->N, mg->M, mg->s, mg->fp32, &need);
  if (rc != ENS_OK) return rc;
  if (mg->bytes < need) {
    set_error("multigrid buffer of %zu bytes is smaller than the %zu required", mg->bytes, need);
    return ENS_E_NOMEM;
  }
  const double Lb = mg_built_L(mg);
  if (Lb <= 0.0) {
    set_error("multigrid buffer not built: call ens_mg_build first");
    return ENS_E_ARG;
  }
  MgPlan plan;
  mg_plan(mg->N, mg->M, mg->s, mg->fp32 != 0, (char*)mg->buffer, &plan);
  mg_attach_fine(&plan, graph->row_ptr, graph->col_idx, values, mg->fp32 ? values32 : nullptr);
  switch (mg->s) {
    case 4: rc = setup_galerkin<4>(plan, stream, false); break;
    case 8: rc = setup_galerkin<8>(plan, stream, false); break;
    case 16: rc = setup_galerkin<16>(plan, stream, false); break;
    default: rc = setup_galerkin<32>(plan, stream, false); break;
  }
  if (rc == ENS_OK) mg_mark(mg, Lb, 2);
  return rc;
}

ens_status ens_mg_assemble_setup_adv(const ens_mg* mg, const ens_graph* graph, const void* kl,
                                     const ens_nl_problem* problem, const double* xi, double* values,
                                     float* values32, double* rhs, hipStream_t stream) {
  ENS_ARG_CHECK(problem, "null problem");
  ENS_ARG_CHECK(std::isfinite(problem->alpha) && std::isfinite(problem->vx) && std::isfinite(problem->vy) &&
                    std::isfinite(problem->vz),
                "alpha and v must be finite");
  const ens_problem lin{problem->M, problem->L, problem->kappa0, problem->sigma, problem->f};
  const double adv[4] = {problem->alpha, problem->vx, problem->vy, problem->vz};
  return assemble_setup(mg, graph, kl, &lin, adv, xi, values, values32, rhs, stream);
}

ens_status ens_mg_level_values(const ens_mg* mg, int32_t level, int32_t* N, const double** values,
                               const float** values32) {
  ENS_ARG_CHECK(mg && mg->buffer && N && values && values32, "null argument");
  MgPlan plan;
  if (!mg_plan(mg->N, mg->M, mg->s, mg->fp32 != 0, (char*)mg->buffer, &plan)) {
    set_error("coarsest multigrid level of N=%d has more than %lld interior unknowns", mg->N, (long long)kMgMaxCoarse);
    return ENS_E_UNSUPPORTED;
  }
  ENS_ARG_CHECK(level >= 1 && level < plan.levels, "level is not a coarse level of this hierarchy");
  *N = plan.lv[level].N;
  *values = plan.lv[level].own_vals;
  *values32 = plan.lv[level].own_vals32;
  return ENS_OK;
}

ens_status ens_mg_release(const ens_mg* mg) {
  ENS_ARG_CHECK(mg, "null multigrid argument");
  std::lock_guard<std::mutex> lk(g_mg_mu);
  for (size_t i = 0; i < g_mg.size(); ++i)
    if (g_mg[i].buffer == mg->buffer) {
      g_mg.erase(g_mg.begin() + (long)i);
      break;
    }
  return ENS_OK;
}

}  // extern "C"
