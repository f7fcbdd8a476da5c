// Learned initial guess, reduced-basis part: a POD basis built by the
// method of snapshots from solutions the ensemble solver produced.
//
//   snapshots S [n][m] (one column per solved sample)
//   G = S^T S [m][m]                         (FP64, split-K tiled GEMM)
//   top-r eigenpairs of G by block subspace iteration with a seeded start
//   block, Gram-Schmidt (twice), and a final Rayleigh-Ritz step whose k x k
//   eigenproblem is solved by cyclic Jacobi in one workgroup
//   Phi = S V_r diag(lambda_r)^(-1/2) [n][r], each column's largest-magnitude
//   entry made positive
//   coefficients C = X^T Phi and reconstruction x0 = Phi c in the ensemble
//   layout [n][s].
// Everything is FP64 except the network outputs c (FP32).
#include "common.hpp"

namespace ens {

// C[M][N] (= or +=) op(A)[M][K] op(B)[K][N], FP64.  op(A)[i][k] is A[i*lda+k]
// (TA = 0) or A[k*lda+i] (TA = 1); likewise op(B)[k][j] is B[k*ldb+j]
// (TB = 0) or B[j*ldb+k] (TB = 1).  Block tile 64 x 64, 16 x 16 threads with
// 4 x 4 outputs each, K staged through LDS in slices of 16.  blockIdx.z
// selects a K range [z*kchunk, (z+1)*kchunk) and writes its partial product
// to C + z*cstride (split-K; summed by k_sum_slices).
template <int TA, int TB>
__global__ __launch_bounds__(256) void k_dgemm(int64_t M, int64_t N, int64_t K, const double* __restrict__ A,
                                               int64_t lda, const double* __restrict__ B, int64_t ldb,
                                               double* __restrict__ C, int64_t ldc, int64_t kchunk,
                                               int64_t cstride) {
  __shared__ double As[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = kb + kchunk < K ? kb + kchunk : K;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int64_t k0 = kb; k0 < ke; k0 += 16) {
    // each of the 256 threads loads 4 elements of each 16 x 64 slice
    for (int t = threadIdx.x; t < 16 * 64; t += 256) {
      const int kk = TA ? t / 64 : t % 16;
      const int ii = TA ? t % 64 : t / 16;
      const int64_t gi = i0 + ii, gk = k0 + kk;
      As[kk][ii] = (gi < M && gk < ke) ? (TA ? A[gk * lda + gi] : A[gi * lda + gk]) : 0.0;
      const int kk2 = TB ? t % 16 : t / 64;
      const int jj = TB ? t / 16 : t % 64;
      const int64_t gj = j0 + jj, gk2 = k0 + kk2;
      Bs[kk2][jj] = (gj < N && gk2 < ke) ? (TB ? B[gj * ldb + gk2] : B[gk2 * ldb + gj]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][ty + 16 * q];
        b[q] = Bs[kk][tx + 16 * q];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
    }
    __syncthreads();
  }
  double* Cz = C + (int64_t)blockIdx.z * cstride;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = i0 + ty + 16 * p, j = j0 + tx + 16 * q;
      if (i < M && j < N) Cz[i * ldc + j] = acc[p][q];
    }
}

// out[i] = sum_z parts[z*stride + i], z ascending.
__global__ void k_sum_slices(int64_t count, int nz, const double* __restrict__ parts, int64_t stride,
                             double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double s = 0.0;
  for (int z = 0; z < nz; ++z) s += parts[(int64_t)z * stride + i];
  out[i] = s;
}

// Orthonormalise the k columns of Y [m][k] (row-major) in place, one
// workgroup: classical Gram-Schmidt applied twice per column (CGS2), the k
// projections of a pass computed by the wavefronts in parallel and applied
// in ascending column order.  A column whose norm falls below 1e-14 of the
// first column's is reported through *rank_deficient.
__global__ __launch_bounds__(1024) void k_orth(int m, int k, double* __restrict__ Y, int* __restrict__ rank_def) {
  __shared__ double d[256];
  __shared__ double red[16];
  __shared__ double s_norm;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = blockDim.x >> 6;
  double first = 0.0;
  for (int j = 0; j < k; ++j) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = wave; i < j; i += nw) {
        double sum = 0.0;
        for (int r = lane; r < m; r += 64) sum += Y[(int64_t)r * k + i] * Y[(int64_t)r * k + j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
        if (lane == 0) d[i] = sum;
      }
      __syncthreads();
      for (int r = t; r < m; r += blockDim.x) {
        double v = Y[(int64_t)r * k + j];
        for (int i = 0; i < j; ++i) v -= d[i] * Y[(int64_t)r * k + i];
        Y[(int64_t)r * k + j] = v;
      }
      __syncthreads();
    }
    double sum = 0.0;
    for (int r = t; r < m; r += blockDim.x) sum += Y[(int64_t)r * k + j] * Y[(int64_t)r * k + j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    if (lane == 0) red[wave] = sum;
    __syncthreads();
    if (t == 0) {
      double tot = 0.0;
      for (int w = 0; w < nw; ++w) tot += red[w];
      s_norm = sqrt(tot);
    }
    __syncthreads();
    const double nrm = s_norm;
    if (j == 0) first = nrm;
    if (t == 0 && (!(nrm > 1e-300) || nrm < 1e-14 * first)) *rank_def = 1;
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int r = t; r < m; r += blockDim.x) Y[(int64_t)r * k + j] *= inv;
    __syncthreads();
  }
}

// Cyclic Jacobi on a symmetric k x k matrix H (row-major, in place), one
// workgroup; the rotation angles are computed by thread 0 and applied to
// rows/columns in parallel.  On exit the diagonal of H holds the
// eigenvalues and U [k][k] the eigenvectors (columns).
__global__ __launch_bounds__(256) void k_jacobi(int k, double* __restrict__ H, double* __restrict__ U, int sweeps) {
  __shared__ double s_c, s_s;
  __shared__ int s_skip;
  const int t = threadIdx.x;
  for (int i = t; i < k * k; i += blockDim.x) U[i] = (i / k == i % k) ? 1.0 : 0.0;
  __syncthreads();
  for (int sw = 0; sw < sweeps; ++sw) {
    for (int p = 0; p < k - 1; ++p)
      for (int q = p + 1; q < k; ++q) {
        if (t == 0) {
          const double apq = H[p * k + q], app = H[p * k + p], aqq = H[q * k + q];
          if (fabs(apq) <= 1e-300 || fabs(apq) <= 1e-18 * sqrt(fabs(app * aqq))) {
            s_skip = 1;
          } else {
            const double tau = (aqq - app) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            s_c = 1.0 / sqrt(1.0 + tt * tt);
            s_s = tt * s_c;
            s_skip = 0;
          }
        }
        __syncthreads();
        if (!s_skip) {
          const double c = s_c, s = s_s;
          // rows p, q of H
          for (int j = t; j < k; j += blockDim.x) {
            const double hp = H[p * k + j], hq = H[q * k + j];
            H[p * k + j] = c * hp - s * hq;
            H[q * k + j] = s * hp + c * hq;
          }
          __syncthreads();
          // columns p, q of H and of U
          for (int i = t; i < k; i += blockDim.x) {
            const double hp = H[i * k + p], hq = H[i * k + q];
            H[i * k + p] = c * hp - s * hq;
            H[i * k + q] = s * hp + c * hq;
            const double up = U[i * k + p], uq = U[i * k + q];
            U[i * k + p] = c * up - s * uq;
            U[i * k + q] = s * up + c * uq;
          }
        }
        __syncthreads();
      }
  }
}

// Sort the Jacobi result by eigenvalue descending; V[m][r] = Q U[:, top r],
// lambda[r].
__global__ void k_ritz_select(int m, int k, int r, const double* __restrict__ H, const double* __restrict__ U,
                              const double* __restrict__ Q, double* __restrict__ V, double* __restrict__ lambda) {
  __shared__ int order[256];
  if (threadIdx.x == 0) {
    for (int i = 0; i < k; ++i) order[i] = i;
    for (int i = 0; i < k; ++i)  // selection sort, k <= 256
      for (int j = i + 1; j < k; ++j)
        if (H[order[j] * k + order[j]] > H[order[i] * k + order[i]]) {
          const int tmp = order[i];
          order[i] = order[j];
          order[j] = tmp;
        }
    for (int j = 0; j < r; ++j) lambda[j] = H[order[j] * k + order[j]];
  }
  __syncthreads();
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (int64_t)m * r;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / r;
    const int j = (int)(t % r), c = order[j];
    double s = 0.0;
    for (int l = 0; l < k; ++l) s += Q[i * k + l] * U[l * k + c];
    V[t] = s;
  }
}

// Phi columns scaled by lambda^(-1/2) (in place on the S V product).
__global__ void k_scale_cols(int64_t n, int r, double* __restrict__ P, const double* __restrict__ lambda) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * r) return;
  P[t] *= 1.0 / sqrt(lambda[t % r]);
}

// Sign rule: the largest-magnitude entry of every column is positive (ties:
// the lowest row).  One workgroup per column.
__global__ __launch_bounds__(256) void k_sign_cols(int64_t n, int r, double* __restrict__ P) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int j = blockIdx.x;
  double best = -1.0;
  int64_t besti = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double a = fabs(P[i * r + j]);
    if (a > best) {
      best = a;
      besti = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = besti;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double o = bv[threadIdx.x + s];
      const int64_t oi = bi[threadIdx.x + s];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const bool flip = P[bi[0] * r + j] < 0.0;
  __syncthreads();
  if (flip)
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) P[i * r + j] = -P[i * r + j];
}

// S[i][col0 + e] = x[i][e]
__global__ void k_collect(int64_t n, int s, const double* __restrict__ x, double* __restrict__ S, int m, int col0) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * s) return;
  const int64_t i = t / s;
  const int e = (int)(t % s);
  S[i * m + col0 + e] = x[t];
}

// x0[i][e] = sum_j Phi[i][j] (mu[j] + sd[j] c[e][j])   (c FP32; mu, sd nullable)
__global__ __launch_bounds__(256) void k_reconstruct(int64_t n, int r, int s, const double* __restrict__ Phi,
                                                     const float* __restrict__ c, const double* __restrict__ mu,
                                                     const double* __restrict__ sd, double* __restrict__ x0) {
  // the de-standardised coefficients chat[e][j] = mu_j + sd_j c[e][j] of all
  // samples, staged once per block
  extern __shared__ double chat[];
  for (int t = threadIdx.x; t < s * r; t += blockDim.x) {
    const int j = t % r;
    double cj = (double)c[t];
    if (sd) cj *= sd[j];
    if (mu) cj += mu[j];
    chat[t] = cj;
  }
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * s) return;
  const int64_t i = t / s;
  const int e = (int)(t % s);
  const double* prow = Phi + i * r;
  const double* ce = chat + (int64_t)e * r;
  double acc = 0.0;
  for (int j = 0; j < r; ++j) acc += prow[j] * ce[j];
  x0[t] = acc;
}

// Per-column mean and standard deviation of C [m][r] (one thread per
// column, rows in order) and the standardised targets T = (C - mu) / sd.
// Mean and standard deviation of each coefficient over the m snapshots
// (one lane per coefficient, one workgroup), the scale of each coefficient
// its own deviation or (common) the largest of them, and the network
// targets T = (C - mu) / scale.  With one common scale the targets keep the
// coefficients' relative sizes, so the network's squared error is the
// squared error of the lifted guess in the orthonormal basis.
__global__ void k_standardize(int m, int r, int common, const double* __restrict__ C, double* __restrict__ mu,
                              double* __restrict__ sd, float* __restrict__ T) {
  __shared__ double s_dev[1024];
  const int j = threadIdx.x;
  double mean = 0.0, dev = 0.0;
  if (j < r) {
    double s1 = 0.0;
    for (int i = 0; i < m; ++i) s1 += C[(int64_t)i * r + j];
    mean = s1 / m;
    double s2 = 0.0;
    for (int i = 0; i < m; ++i) {
      const double d = C[(int64_t)i * r + j] - mean;
      s2 += d * d;
    }
    dev = sqrt(s2 / m);
  }
  s_dev[j] = dev;
  __syncthreads();
  if (common) {
    double mx = 0.0;
    for (int k = 0; k < r; ++k) mx = s_dev[k] > mx ? s_dev[k] : mx;
    dev = mx;
  }
  if (!(dev > 0.0)) dev = 1.0;
  if (j >= r) return;
  mu[j] = mean;
  sd[j] = dev;
  for (int i = 0; i < m; ++i) T[(int64_t)i * r + j] = (float)((C[(int64_t)i * r + j] - mean) / dev);
}

// ------------------------------------------------------------ host side ---

template <int TA, int TB>
static void dgemm(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* B, int64_t ldb,
                  double* C, int64_t ldc, int splits, double* scratch, hipStream_t st) {
  if (splits <= 1) {
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), 1);
    hipLaunchKernelGGL((k_dgemm<TA, TB>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, K, (int64_t)0);
    return;
  }
  // the split path writes C densely (leading dimension N); callers pass ldc == N
  int64_t kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + 15) / 16 * 16;
  const int nz = (int)((K + kchunk - 1) / kchunk);
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)nz);
  hipLaunchKernelGGL((k_dgemm<TA, TB>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, scratch, N, kchunk,
                     M * N);
  hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)((M * N + 255) / 256)), dim3(256), 0, st, M * N, nz, scratch,
                     M * N, C);
  (void)ldc;
}

static int gram_splits(int64_t n) {
  int64_t s = n / 4096;
  if (s < 1) s = 1;
  if (s > 32) s = 32;
  return (int)s;
}

}  // namespace ens

using namespace ens;

extern "C" {

ens_status ens_pod_collect(const double* x, int64_t n, int32_t s, double* S, int32_t m, int32_t col0,
                           hipStream_t stream) {
  ENS_ARG_CHECK(x && S && n >= 0 && s >= 1 && m >= 1 && col0 >= 0 && col0 + s <= m, "bad collect arguments");
  if (n == 0) return ENS_OK;
  hipLaunchKernelGGL(k_collect, dim3((unsigned)((n * s + 255) / 256)), dim3(256), 0, stream, n, s, x, S, m, col0);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

ens_status ens_pod_gram_workspace_bytes(int64_t n, int32_t m, size_t* bytes) {
  ENS_ARG_CHECK(bytes && n >= 1 && m >= 1, "bad sizes");
  *bytes = (size_t)gram_splits(n) * m * m * sizeof(double);
  return ENS_OK;
}

ens_status ens_pod_gram(const double* S, int64_t n, int32_t m, double* G, void* workspace, size_t ws_bytes,
                        hipStream_t stream) {
  ENS_ARG_CHECK(S && G && n >= 1 && m >= 1, "bad Gram arguments");
  const int sp = gram_splits(n);
  ENS_ARG_CHECK(sp == 1 || workspace, "null workspace");
  if (sp > 1 && ws_bytes < (size_t)sp * m * m * sizeof(double)) {
    set_error("Gram workspace too small");
    return ENS_E_NOMEM;
  }
  // G = S^T S: op(A) = S^T (TA = 1, lda = m), op(B) = S (TB = 0, ldb = m), K = n
  dgemm<1, 0>(m, m, n, S, m, S, m, G, m, sp, (double*)workspace, stream);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

ens_status ens_pod_eig_workspace_bytes(int32_t m, int32_t k, size_t* bytes) {
  ENS_ARG_CHECK(bytes && m >= 1 && k >= 1, "bad sizes");
  *bytes = (size_t)(3 * (size_t)m * k + 3 * (size_t)k * k + 64) * sizeof(double);
  return ENS_OK;
}

ens_status ens_pod_eig(const double* G, int32_t m, int32_t k, int32_t r, const double* start, int32_t iters,
                       double* V, double* lambda, void* workspace, size_t ws_bytes, hipStream_t stream) {
  ENS_ARG_CHECK(G && start && V && lambda && workspace, "null pointer");
  ENS_ARG_CHECK(m >= 1 && k >= 1 && k <= 256 && k <= m && r >= 1 && r <= k && iters >= 0, "bad sizes");
  size_t need = 0;
  ens_pod_eig_workspace_bytes(m, k, &need);
  if (ws_bytes < need) {
    set_error("eigen workspace too small");
    return ENS_E_NOMEM;
  }
  double* Y = (double*)workspace;
  double* Q = Y + (size_t)m * k;
  double* T = Q + (size_t)m * k;
  double* H = T + (size_t)m * k;
  double* U = H + (size_t)k * k;
  int* flag = (int*)(U + 2 * (size_t)k * k);
  ENS_HIP_TRY(hipMemcpyAsync(Y, start, (size_t)m * k * sizeof(double), hipMemcpyDeviceToDevice, stream));
  ENS_HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), stream));
  // power steps: Y <- G orth(Y)
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(k_orth, dim3(1), dim3(1024), 0, stream, m, k, Y, flag);
    ENS_HIP_TRY(hipMemcpyAsync(Q, Y, (size_t)m * k * sizeof(double), hipMemcpyDeviceToDevice, stream));
    dgemm<0, 0>(m, k, m, G, m, Q, k, Y, k, 1, nullptr, stream);
  }
  // Rayleigh-Ritz on span(Y)
  hipLaunchKernelGGL(k_orth, dim3(1), dim3(1024), 0, stream, m, k, Y, flag);
  dgemm<0, 0>(m, k, m, G, m, Y, k, T, k, 1, nullptr, stream);   // T = G Q
  dgemm<1, 0>(k, k, m, Y, k, T, k, H, k, 1, nullptr, stream);   // H = Q^T G Q
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(256), 0, stream, k, H, U, 12);
  hipLaunchKernelGGL(k_ritz_select, dim3(64), dim3(256), 0, stream, m, k, r, H, U, Y, V, lambda);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

ens_status ens_pod_basis(const double* S, int64_t n, int32_t m, const double* V, const double* lambda, int32_t r,
                         double* Phi, hipStream_t stream) {
  ENS_ARG_CHECK(S && V && lambda && Phi && n >= 1 && m >= 1 && r >= 1 && r <= m, "bad basis arguments");
  dgemm<0, 0>(n, r, m, S, m, V, r, Phi, r, 1, nullptr, stream);  // Phi = S V
  hipLaunchKernelGGL(k_scale_cols, dim3((unsigned)((n * r + 255) / 256)), dim3(256), 0, stream, n, r, Phi, lambda);
  hipLaunchKernelGGL(k_sign_cols, dim3((unsigned)r), dim3(256), 0, stream, n, r, Phi);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

ens_status ens_pod_project_workspace_bytes(int64_t n, int32_t r, int32_t s, size_t* bytes) {
  ENS_ARG_CHECK(bytes && n >= 1 && r >= 1 && s >= 1, "bad sizes");
  *bytes = (size_t)gram_splits(n) * r * s * sizeof(double);
  return ENS_OK;
}

ens_status ens_pod_project(const double* Phi, const double* X, int64_t n, int32_t r, int32_t s, double* C,
                           void* workspace, size_t ws_bytes, hipStream_t stream) {
  ENS_ARG_CHECK(Phi && X && C && n >= 1 && r >= 1 && s >= 1, "bad projection arguments");
  const int sp = gram_splits(n);
  ENS_ARG_CHECK(sp == 1 || workspace, "null workspace");
  if (sp > 1 && ws_bytes < (size_t)sp * r * s * sizeof(double)) {
    set_error("projection workspace too small");
    return ENS_E_NOMEM;
  }
  // C[e][j] = sum_i X[i][e] Phi[i][j]: op(A) = X^T (TA = 1, lda = s), op(B) = Phi
  dgemm<1, 0>(s, r, n, X, s, Phi, r, C, r, sp, (double*)workspace, stream);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

ens_status ens_pod_reconstruct(const double* Phi, int64_t n, int32_t r, const float* c, const double* mu,
                               const double* sd, int32_t s, double* x0, hipStream_t stream) {
  ENS_ARG_CHECK(Phi && c && x0 && n >= 1 && r >= 1 && s >= 1, "bad reconstruction arguments");
  ENS_ARG_CHECK((int64_t)s * r <= 8192, "s * r must not exceed 8192 (coefficients staged in 64 KB of LDS)");
  hipLaunchKernelGGL(k_reconstruct, dim3((unsigned)((n * s + 255) / 256)), dim3(256),
                     (size_t)s * r * sizeof(double), stream, n, r, s, Phi, c, mu, sd, x0);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

ens_status ens_pod_standardize(const double* C, int32_t m, int32_t r, int32_t common, double* mu, double* sd,
                               float* T, hipStream_t stream) {
  ENS_ARG_CHECK(C && mu && sd && T && m >= 1 && r >= 1 && r <= 1024, "bad standardize arguments");
  hipLaunchKernelGGL(k_standardize, dim3(1), dim3((unsigned)((r + 63) / 64 * 64)), 0, stream, m, r, common, C, mu,
                     sd, T);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

}  // extern "C"
