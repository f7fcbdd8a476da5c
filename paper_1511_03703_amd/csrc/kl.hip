// Karhunen-Loeve table of the diffusion coefficient, built on the GPU.
//
// Sec. 4 models kappa(x,y) = kappa0 + sigma sum_i kappa_i(x) y_i with kappa_i
// the eigenfunctions of the exponential covariance exp(-|x-x'|_1 / L), which
// are tensor products of sines and cosines.  We take kappa_i = sqrt(lambda_i)
// phi_i of the unit-variance kernel.  Because the 1-norm separates, the 3D
// eigenpairs are products of the 1D eigenpairs of exp(-|t-t'|/L) on [0,1].
// Centring t at 1/2 (half-width a = 1/2, c = 1/L), the 1D modes are
//   even: cos(w t) with c cos(w a) - w sin(w a) = 0, w in ((m-1)pi/a, (m-1/2)pi/a)
//   odd:  sin(w t) with w cos(w a) + c sin(w a) = 0, w in ((m-1/2)pi/a, m pi/a)
// with lambda = 2c / (w^2 + c^2); the root equations are written without
// poles and solved by safeguarded Newton iteration.  3D modes are ranked by
// lambda descending, ties broken by ascending (ix, iy, iz); each 3D lambda
// multiplies its 1D factors in ascending index order so permuted triples tie
// exactly.
#include "common.hpp"

namespace ens {

constexpr int kMaxM = 16;

struct KLView {
  double* sqrt_lam3;
  double* lam3;
  double* omega;
  double* lam1;
  double* norm1;
  int32_t* parity;
  int32_t* triple;
  double* phi;  // [M][2N]
};

__host__ __device__ inline size_t kl_phi_offset(int M) {
  size_t off = (size_t)M * 5 * sizeof(double) + (size_t)M * 4 * sizeof(int32_t);
  return (off + 15) & ~(size_t)15;
}

__host__ __device__ inline KLView kl_view(void* base, int M) {
  char* p = (char*)base;
  KLView v;
  v.sqrt_lam3 = (double*)p;
  v.lam3 = v.sqrt_lam3 + M;
  v.omega = v.lam3 + M;
  v.lam1 = v.omega + M;
  v.norm1 = v.lam1 + M;
  v.parity = (int32_t*)(v.norm1 + M);
  v.triple = v.parity + M;
  v.phi = (double*)(p + kl_phi_offset(M));
  return v;
}

// residual of the pole-free root equations and its derivative
__device__ inline void kl_eq(int odd, double w, double a, double c, double* g, double* dg) {
  double sn, cs;
  sincos(w * a, &sn, &cs);
  if (!odd) {  // c cos(wa) - w sin(wa)
    *g = c * cs - w * sn;
    *dg = -c * a * sn - sn - w * a * cs;
  } else {     // w cos(wa) + c sin(wa)
    *g = w * cs + c * sn;
    *dg = cs - w * a * sn + c * a * cs;
  }
}

__global__ void k_kl_modes(int M, double L, KLView v) {
  __shared__ double lam1[kMaxM];
  const double a = 0.5, c = 1.0 / L, pi = 3.14159265358979323846;
  int t = threadIdx.x;
  if (t < M) {
    int m = t / 2 + 1;
    int odd = t & 1;
    double lo = odd ? (m - 0.5) * pi / a : (m - 1) * pi / a;
    double hi = odd ? m * pi / a : (m - 0.5) * pi / a;
    double glo, ghi, d;
    kl_eq(odd, lo, a, c, &glo, &d);
    kl_eq(odd, hi, a, c, &ghi, &d);
    double w = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
      double g, dg;
      kl_eq(odd, w, a, c, &g, &dg);
      if (g == 0.0) break;
      // keep the bracket
      if ((g < 0.0) == (glo < 0.0)) lo = w; else hi = w;
      double wn = w - g / dg;
      if (!(wn > lo && wn < hi)) wn = 0.5 * (lo + hi);
      if (fabs(wn - w) <= 2e-16 * w) { w = wn; break; }
      w = wn;
    }
    double l1 = 2.0 * c / (w * w + c * c);
    double s2 = sin(2.0 * w * a) / (2.0 * w);
    v.omega[t] = w;
    v.lam1[t] = l1;
    v.norm1[t] = 1.0 / sqrt(odd ? a - s2 : a + s2);
    v.parity[t] = odd;
    lam1[t] = l1;
  }
  __syncthreads();
  // rank every triple (i,j,k) in [0,M)^3 by counting the triples before it
  int total = M * M * M;
  for (int q = t; q < total; q += blockDim.x) {
    int i = q / (M * M), j = (q / M) % M, k = q % M;
    int s0 = i, s1 = j, s2 = k, tmp;
    if (s1 < s0) { tmp = s0; s0 = s1; s1 = tmp; }
    if (s2 < s1) { tmp = s1; s1 = s2; s2 = tmp; }
    if (s1 < s0) { tmp = s0; s0 = s1; s1 = tmp; }
    double lq = (lam1[s0] * lam1[s1]) * lam1[s2];
    int rank = 0;
    for (int p = 0; p < total && rank < M; ++p) {
      int pi_ = p / (M * M), pj = (p / M) % M, pk = p % M;
      int u0 = pi_, u1 = pj, u2 = pk;
      if (u1 < u0) { tmp = u0; u0 = u1; u1 = tmp; }
      if (u2 < u1) { tmp = u1; u1 = u2; u2 = tmp; }
      if (u1 < u0) { tmp = u0; u0 = u1; u1 = tmp; }
      double lp = (lam1[u0] * lam1[u1]) * lam1[u2];
      if (lp > lq || (lp == lq && p < q)) ++rank;
    }
    if (rank < M) {
      v.triple[3 * rank + 0] = i;
      v.triple[3 * rank + 1] = j;
      v.triple[3 * rank + 2] = k;
      v.lam3[rank] = lq;
      v.sqrt_lam3[rank] = sqrt(lq);
    }
  }
}

// phi of 1D mode k at abscissa (e + g_q)/N, stored at [k][2e + q]
__global__ void k_kl_tables(int N, int M, KLView v) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  int per = 2 * N;
  if (idx >= M * per) return;
  int k = idx / per, pos = idx % per;
  int e = pos >> 1, q = pos & 1;
  const double r = 0.57735026918962576451;  // 1/sqrt(3)
  double g = q ? 0.5 * (1.0 + r) : 0.5 * (1.0 - r);
  double x = ((double)e + g) / (double)N;
  double t = x - 0.5;
  double w = v.omega[k];
  v.phi[idx] = v.norm1[k] * (v.parity[k] ? sin(w * t) : cos(w * t));
}

}  // namespace ens

using namespace ens;

extern "C" {

ens_status ens_kl_bytes(int32_t N, int32_t M, size_t* bytes) {
  ENS_ARG_CHECK(N >= 1 && bytes, "bad arguments");
  if (M < 0 || M > kMaxM) {
    set_error("M=%d outside the compiled range [0, %d]", M, kMaxM);
    return ENS_E_UNSUPPORTED;
  }
  *bytes = kl_phi_offset(M) + (size_t)M * 2 * N * sizeof(double) + 16;
  return ENS_OK;
}

ens_status ens_kl_build(int32_t N, int32_t M, double L, void* kl, hipStream_t stream) {
  size_t bytes = 0;
  ens_status st = ens_kl_bytes(N, M, &bytes);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK(kl && aligned16(kl), "kl table must be a 16-byte aligned device pointer");
  ENS_ARG_CHECK(L > 0.0, "correlation length must be positive");
  if (M == 0) return ENS_OK;
  KLView v = kl_view(kl, M);
  hipLaunchKernelGGL(k_kl_modes, dim3(1), dim3(256), 0, stream, M, L, v);
  ENS_LAUNCH_CHECK();
  int total = M * 2 * N;
  hipLaunchKernelGGL(k_kl_tables, dim3((total + 255) / 256), dim3(256), 0, stream, N, M, v);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

}  // extern "C"
