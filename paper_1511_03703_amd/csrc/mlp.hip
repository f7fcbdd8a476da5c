// Learned initial guess, network part: a 10 -> 256 -> 256 -> 32 MLP with
// GELU activations that maps the KL inputs y of a sample to the
// coefficients of a POD basis; its prediction only seeds CG.
//
// All matrix products run on gfx950 matrix cores (v_mfma_f32_16x16x32_bf16):
// BF16 operands, FP32 accumulation.  Bias, GELU, loss and Adam are FP32 on
// FP32 master weights.  Every product is written as one "NT" form,
//     C[m][n] = sum_k A[m][k] B[n][k]      (both operands K-contiguous),
// so each lane loads its 8-element MFMA fragment with one 16-byte load.  The
// backward products need transposed operands; the epilogues that produce
// activations and gradients therefore also write transposed BF16 copies.
//
// GELU is the exact form 0.5 z (1 + erf(z / sqrt 2)), derivative
// Phi(z) + z phi(z).
#include "common.hpp"

namespace ens {

constexpr int kIn = 10, kInPad = 32, kHid = 256, kOut = 32;
constexpr int64_t kOffW1 = 0, kOffB1 = kOffW1 + kHid * kIn, kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kHid * kHid,
                  kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kOut * kHid, kParams = kOffB3 + kOut;

typedef uint16_t bf16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round-to-nearest-even FP32 -> BF16 (bit pattern)
__device__ inline bf16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (bf16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ inline float from_bf16(bf16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

enum { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_BIAS = 2, EPI_DGELU = 3 };

struct Epi {
  const float* bias;  // [N]
  float* f32;         // [M][ld_f32]: result (STORE/BIAS), pre-activation (BIAS_GELU), dz (DGELU)
  int ld_f32;
  bf16_t* bf;         // [M][ld_bf]: activation / dz in BF16 (may be null)
  int ld_bf;
  bf16_t* bft;        // [N][ld_bft]: transposed BF16 copy (may be null)
  int ld_bft;
  const float* z;     // [M][ld_z]: pre-activation for DGELU
  int ld_z;
};

// One block = 4 waves = a 64 x 64 tile of C; each wave a 32 x 32 sub-tile
// of 2 x 2 MFMA 16 x 16 blocks.  K must be a multiple of 32; rows of A or B
// beyond M or N read as zero and outputs beyond M or N are not written.
// MFMA 16x16x32 fragments: lane l holds A[l%16][8(l/16) .. 8(l/16)+7] and
// B[8(l/16) .. +7][l%16]; the 16 x 16 result leaves D[4(l/16)+t][l%16],
// t = 0..3, in lane l.
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_nt(int M, int N, int K, const bf16_t* __restrict__ A, int lda,
                                                 const bf16_t* __restrict__ B, int ldb, Epi ep) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int n0 = blockIdx.x * 64 + (wave & 1) * 32;
  const int r = lane & 15, kq = (lane >> 4) * 8;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4)0.0f;
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int row = m0 + 16 * i + r;
      a[i] = row < M ? *(const bf16x8*)(A + (int64_t)row * lda + k0 + kq) : (bf16x8)0.0f;
      const int col = n0 + 16 * i + r;
      b[i] = col < N ? *(const bf16x8*)(B + (int64_t)col * ldb + k0 + kq) : (bf16x8)0.0f;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = m0 + 16 * i + 4 * (lane >> 4) + t;
        const int n = n0 + 16 * j + (lane & 15);
        if (m >= M || n >= N) continue;
        float v = acc[i][j][t];
        if (EPI == EPI_STORE) {
          ep.f32[(int64_t)m * ep.ld_f32 + n] = v;
        } else if (EPI == EPI_BIAS) {
          ep.f32[(int64_t)m * ep.ld_f32 + n] = v + ep.bias[n];
        } else if (EPI == EPI_BIAS_GELU) {
          const float z = v + ep.bias[n];
          ep.f32[(int64_t)m * ep.ld_f32 + n] = z;
          const bf16_t h = to_bf16(gelu(z));
          if (ep.bf) ep.bf[(int64_t)m * ep.ld_bf + n] = h;
          if (ep.bft) ep.bft[(int64_t)n * ep.ld_bft + m] = h;
        } else {  // EPI_DGELU
          const float dz = v * gelu_grad(ep.z[(int64_t)m * ep.ld_z + n]);
          ep.f32[(int64_t)m * ep.ld_f32 + n] = dz;
          const bf16_t h = to_bf16(dz);
          if (ep.bf) ep.bf[(int64_t)m * ep.ld_bf + n] = h;
          if (ep.bft) ep.bft[(int64_t)n * ep.ld_bft + m] = h;
        }
      }
}

// Input rows: X[b] = xi[idx ? idx[b] : b] padded with zeros to 32 columns,
// in BF16, plain and transposed; targets gathered likewise (FP32).
__global__ void k_mlp_input(int B, const float* __restrict__ xi, const float* __restrict__ tgt,
                            const int32_t* __restrict__ idx, bf16_t* __restrict__ xb, bf16_t* __restrict__ xbt,
                            float* __restrict__ tb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * kInPad) return;
  const int b = t / kInPad, k = t % kInPad;
  const int src = idx ? idx[b] : b;
  const bf16_t v = k < kIn ? to_bf16(xi[(int64_t)src * kIn + k]) : (bf16_t)0;
  xb[(int64_t)b * kInPad + k] = v;
  xbt[(int64_t)k * B + b] = v;
  if (tgt) tb[(int64_t)b * kOut + k] = tgt[(int64_t)src * kOut + k];  // kOut == kInPad
}

// BF16 copies of the weights: W1 [256][32] (K padded), W2 and W2^T, W3 and W3^T.
__global__ void k_mlp_weights(const float* __restrict__ p, bf16_t* __restrict__ w1, bf16_t* __restrict__ w2,
                              bf16_t* __restrict__ w2t, bf16_t* __restrict__ w3, bf16_t* __restrict__ w3t) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < kHid * kInPad) {
    const int n = t / kInPad, k = t % kInPad;
    w1[t] = k < kIn ? to_bf16(p[kOffW1 + n * kIn + k]) : (bf16_t)0;
  }
  if (t < kHid * kHid) {
    const int n = t / kHid, k = t % kHid;
    const bf16_t v = to_bf16(p[kOffW2 + t]);
    w2[t] = v;
    w2t[k * kHid + n] = v;
  }
  if (t < kOut * kHid) {
    const int n = t / kHid, k = t % kHid;
    const bf16_t v = to_bf16(p[kOffW3 + t]);
    w3[t] = v;
    w3t[k * kOut + n] = v;
  }
}

// dY = 2 (Y - T) / (B * 32), plain BF16 and transposed BF16 copies; one
// block accumulates the mean squared error in a fixed order.
__global__ __launch_bounds__(256) void k_mse(int B, const float* __restrict__ y, const float* __restrict__ t,
                                             float* __restrict__ dy, bf16_t* __restrict__ dyb,
                                             bf16_t* __restrict__ dybt, float* __restrict__ loss) {
  __shared__ double red[256];
  const int total = B * kOut;
  const float sc = 2.0f / (float)total;
  double acc = 0.0;
  for (int i = threadIdx.x; i < total; i += blockDim.x) {
    const float d = y[i] - t[i];
    acc += (double)d * (double)d;
    const float g = sc * d;
    dy[i] = g;
    const bf16_t h = to_bf16(g);
    dyb[i] = h;
    const int b = i / kOut, n = i % kOut;
    dybt[(int64_t)n * B + b] = h;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = (float)(red[0] / total);
}

// Column sums of an FP32 [M][N] matrix (bias gradients), fixed order.
// out[n] = sum over m of a[m][n]: a block of 256 threads covers 64 columns,
// four thread groups take interleaved rows with four running sums each, and
// the sixteen partial sums of a column are added in a fixed order.
__global__ __launch_bounds__(256) void k_colsum(int M, int N, const float* __restrict__ a, float* __restrict__ out) {
  __shared__ float part[4][64];
  const int col = blockIdx.x * 64 + (threadIdx.x & 63);
  const int g = threadIdx.x >> 6;
  float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
  if (col < N) {
    int m = g;
    for (; m + 12 < M; m += 16) {
      s0 += a[(int64_t)m * N + col];
      s1 += a[(int64_t)(m + 4) * N + col];
      s2 += a[(int64_t)(m + 8) * N + col];
      s3 += a[(int64_t)(m + 12) * N + col];
    }
    for (; m < M; m += 4) s0 += a[(int64_t)m * N + col];
  }
  part[g][threadIdx.x & 63] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (g == 0 && col < N) out[col] = (part[0][threadIdx.x] + part[1][threadIdx.x]) + (part[2][threadIdx.x] + part[3][threadIdx.x]);
}

// One Adam step (Kingma and Ba 2015, Algorithm 1) per element, FP32:
// moving averages of g and g^2, divided by the bias corrections c1 = 1 - b1^t
// and c2 = 1 - b2^t, eps added to the square root of the second moment.
// omb1 = 1 - b1 and omb2 = 1 - b2 come in as arguments, each the FP32
// rounding of the exact value (1.0f - 0.999f would carry the 1.3e-5 relative
// error of 0.999f into every second moment).
__global__ void k_adam(int64_t P, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float omb1, float omb2, float eps,
                       float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + omb1 * gi;
  const float vi = b2 * v[i] + omb2 * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Adam with beta = (0.9, 0.999), eps = 1e-8 at step t (1-based) over P
// elements; 1 - beta and the bias corrections 1 - beta^t are formed in FP64
// from the decimal betas and rounded once to FP32.
static void adam_launch(int64_t P, float* p, const float* g, float* m, float* v, int t, float lr,
                        hipStream_t stream) {
  const double b1 = 0.9, b2 = 0.999;
  double p1 = 1.0, p2 = 1.0;
  for (int k = 0; k < t; ++k) {
    p1 *= b1;
    p2 *= b2;
  }
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, stream, P, p, g, m, v, lr, (float)b1,
                     (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, (float)(1.0 - p1), (float)(1.0 - p2));
}

// ------------------------------------------------------------ host side ---

struct MlpWork {
  bf16_t *xb, *xbt, *h1b, *h1bt, *h2b, *h2bt, *dyb, *dybt, *dz2b, *dz2bt, *dz1bt;
  bf16_t *w1, *w2, *w2t, *w3, *w3t;
  float *tb, *z1, *z2, *y, *dy, *dz2, *dz1, *grad, *loss;
};

static size_t r256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t mlp_layout(int B, MlpWork* w, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? base + off : nullptr;
    off += r256(bytes);
    return p;
  };
  const size_t bh = sizeof(bf16_t), f = sizeof(float);
  MlpWork t;
  t.xb = (bf16_t*)take((size_t)B * kInPad * bh);
  t.xbt = (bf16_t*)take((size_t)B * kInPad * bh);
  t.h1b = (bf16_t*)take((size_t)B * kHid * bh);
  t.h1bt = (bf16_t*)take((size_t)B * kHid * bh);
  t.h2b = (bf16_t*)take((size_t)B * kHid * bh);
  t.h2bt = (bf16_t*)take((size_t)B * kHid * bh);
  t.dyb = (bf16_t*)take((size_t)B * kOut * bh);
  t.dybt = (bf16_t*)take((size_t)B * kOut * bh);
  t.dz2b = (bf16_t*)take((size_t)B * kHid * bh);
  t.dz2bt = (bf16_t*)take((size_t)B * kHid * bh);
  t.dz1bt = (bf16_t*)take((size_t)B * kHid * bh);
  t.w1 = (bf16_t*)take((size_t)kHid * kInPad * bh);
  t.w2 = (bf16_t*)take((size_t)kHid * kHid * bh);
  t.w2t = (bf16_t*)take((size_t)kHid * kHid * bh);
  t.w3 = (bf16_t*)take((size_t)kOut * kHid * bh);
  t.w3t = (bf16_t*)take((size_t)kOut * kHid * bh);
  t.tb = (float*)take((size_t)B * kOut * f);
  t.z1 = (float*)take((size_t)B * kHid * f);
  t.z2 = (float*)take((size_t)B * kHid * f);
  t.y = (float*)take((size_t)B * kOut * f);
  t.dy = (float*)take((size_t)B * kOut * f);
  t.dz2 = (float*)take((size_t)B * kHid * f);
  t.dz1 = (float*)take((size_t)B * kHid * f);
  t.grad = (float*)take((size_t)kParams * f);
  t.loss = (float*)take(64);
  if (w) *w = t;
  return off;
}

template <int EPI>
static void gemm(int M, int N, int K, const bf16_t* A, int lda, const bf16_t* B, int ldb, const Epi& ep,
                 hipStream_t st) {
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL((k_gemm_nt<EPI>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, ep);
}

static Epi epi(const float* bias, float* f32, int ld_f32, bf16_t* bf, int ld_bf, bf16_t* bft, int ld_bft,
               const float* z = nullptr, int ld_z = 0) {
  Epi e;
  e.bias = bias;
  e.f32 = f32;
  e.ld_f32 = ld_f32;
  e.bf = bf;
  e.ld_bf = ld_bf;
  e.bft = bft;
  e.ld_bft = ld_bft;
  e.z = z;
  e.ld_z = ld_z;
  return e;
}

// Forward on the batch already in w.xb / w.xbt; output Y (FP32) in w.y.
static void forward(const float* p, int B, const MlpWork& w, hipStream_t st) {
  gemm<EPI_BIAS_GELU>(B, kHid, kInPad, w.xb, kInPad, w.w1, kInPad,
                      epi(p + kOffB1, w.z1, kHid, w.h1b, kHid, w.h1bt, B), st);
  gemm<EPI_BIAS_GELU>(B, kHid, kHid, w.h1b, kHid, w.w2, kHid, epi(p + kOffB2, w.z2, kHid, w.h2b, kHid, w.h2bt, B),
                      st);
  gemm<EPI_BIAS>(B, kOut, kHid, w.h2b, kHid, w.w3, kHid, epi(p + kOffB3, w.y, kOut, nullptr, 0, nullptr, 0), st);
}

// Backward of the mean squared error against w.tb; gradients in w.grad.
static void backward(int B, const MlpWork& w, hipStream_t st) {
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, st, B, w.y, w.tb, w.dy, w.dyb, w.dybt, w.loss);
  float* g = w.grad;
  // dW3[n][k] = sum_b dY[b][n] H2[b][k]
  gemm<EPI_STORE>(kOut, kHid, B, w.dybt, B, w.h2bt, B, epi(nullptr, g + kOffW3, kHid, nullptr, 0, nullptr, 0), st);
  // dZ2 = (dY W3) * GELU'(Z2)
  gemm<EPI_DGELU>(B, kHid, kOut, w.dyb, kOut, w.w3t, kOut,
                  epi(nullptr, w.dz2, kHid, w.dz2b, kHid, w.dz2bt, B, w.z2, kHid), st);
  // dW2[n][k] = sum_b dZ2[b][n] H1[b][k]
  gemm<EPI_STORE>(kHid, kHid, B, w.dz2bt, B, w.h1bt, B, epi(nullptr, g + kOffW2, kHid, nullptr, 0, nullptr, 0), st);
  // dZ1 = (dZ2 W2) * GELU'(Z1)
  gemm<EPI_DGELU>(B, kHid, kHid, w.dz2b, kHid, w.w2t, kHid,
                  epi(nullptr, w.dz1, kHid, nullptr, 0, w.dz1bt, B, w.z1, kHid), st);
  // dW1[n][k] = sum_b dZ1[b][n] X[b][k], k < 10
  gemm<EPI_STORE>(kHid, kIn, B, w.dz1bt, B, w.xbt, B, epi(nullptr, g + kOffW1, kIn, nullptr, 0, nullptr, 0), st);
  hipLaunchKernelGGL(k_colsum, dim3((kHid + 63) / 64), dim3(256), 0, st, B, kHid, w.dz1, g + kOffB1);
  hipLaunchKernelGGL(k_colsum, dim3((kHid + 63) / 64), dim3(256), 0, st, B, kHid, w.dz2, g + kOffB2);
  hipLaunchKernelGGL(k_colsum, dim3((kOut + 63) / 64), dim3(256), 0, st, B, kOut, w.dy, g + kOffB3);
}

static void weights_bf16(const float* p, const MlpWork& w, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_weights, dim3((kHid * kHid + 255) / 256), dim3(256), 0, st, p, w.w1, w.w2, w.w2t, w.w3,
                     w.w3t);
}

static void load_batch(int B, const float* xi, const float* tgt, const int32_t* idx, const MlpWork& w,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_input, dim3((B * kInPad + 255) / 256), dim3(256), 0, st, B, xi, tgt, idx, w.xb, w.xbt,
                     w.tb);
}

static bool batch_ok(int B) { return B >= 32 && B <= 65536 && B % 32 == 0; }

}  // namespace ens

using namespace ens;

extern "C" {

int64_t ens_mlp_param_count(void) { return kParams; }

ens_status ens_mlp_workspace_bytes(int32_t batch, size_t* bytes) {
  ENS_ARG_CHECK(bytes && batch_ok(batch), "batch must be a multiple of 32 in [32, 65536]");
  *bytes = mlp_layout(batch, nullptr, nullptr);
  return ENS_OK;
}

ens_status ens_mlp_forward(const float* params, int32_t batch, const float* xi, float* out, void* workspace,
                           size_t ws_bytes, hipStream_t stream) {
  ENS_ARG_CHECK(params && xi && out && workspace, "null pointer");
  ENS_ARG_CHECK(batch_ok(batch), "batch must be a multiple of 32 in [32, 65536]");
  ENS_ARG_CHECK(((uintptr_t)workspace & 255u) == 0, "workspace must be 256-byte aligned");
  if (ws_bytes < mlp_layout(batch, nullptr, nullptr)) {
    set_error("MLP workspace too small");
    return ENS_E_NOMEM;
  }
  MlpWork w;
  mlp_layout(batch, &w, (char*)workspace);
  weights_bf16(params, w, stream);
  load_batch(batch, xi, nullptr, nullptr, w, stream);
  forward(params, batch, w, stream);
  ENS_HIP_TRY(hipMemcpyAsync(out, w.y, (size_t)batch * kOut * sizeof(float), hipMemcpyDeviceToDevice, stream));
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

ens_status ens_mlp_grad(const float* params, int32_t batch, const float* xi, const float* target, float* out,
                        float* grad, float* loss, void* workspace, size_t ws_bytes, hipStream_t stream) {
  ENS_ARG_CHECK(params && xi && target && grad && workspace, "null pointer");
  ENS_ARG_CHECK(batch_ok(batch), "batch must be a multiple of 32 in [32, 65536]");
  ENS_ARG_CHECK(((uintptr_t)workspace & 255u) == 0, "workspace must be 256-byte aligned");
  if (ws_bytes < mlp_layout(batch, nullptr, nullptr)) {
    set_error("MLP workspace too small");
    return ENS_E_NOMEM;
  }
  MlpWork w;
  mlp_layout(batch, &w, (char*)workspace);
  weights_bf16(params, w, stream);
  load_batch(batch, xi, target, nullptr, w, stream);
  forward(params, batch, w, stream);
  backward(batch, w, stream);
  if (out)
    ENS_HIP_TRY(hipMemcpyAsync(out, w.y, (size_t)batch * kOut * sizeof(float), hipMemcpyDeviceToDevice, stream));
  ENS_HIP_TRY(hipMemcpyAsync(grad, w.grad, (size_t)kParams * sizeof(float), hipMemcpyDeviceToDevice, stream));
  if (loss) ENS_HIP_TRY(hipMemcpyAsync(loss, w.loss, sizeof(float), hipMemcpyDeviceToDevice, stream));
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

ens_status ens_mlp_train(float* params, float* adam_m, float* adam_v, int32_t step0, const float* xi,
                         const float* target, int32_t count, int32_t batch, int32_t steps, const int32_t* batch_idx,
                         float lr, float* loss, void* workspace, size_t ws_bytes, hipStream_t stream) {
  ENS_ARG_CHECK(params && adam_m && adam_v && xi && target && batch_idx && workspace, "null pointer");
  ENS_ARG_CHECK(batch_ok(batch) && count >= 1 && steps >= 0 && step0 >= 0, "bad sizes");
  ENS_ARG_CHECK(((uintptr_t)workspace & 255u) == 0, "workspace must be 256-byte aligned");
  ENS_ARG_CHECK(lr > 0.0f, "learning rate must be positive");
  if (ws_bytes < mlp_layout(batch, nullptr, nullptr)) {
    set_error("MLP workspace too small");
    return ENS_E_NOMEM;
  }
  MlpWork w;
  mlp_layout(batch, &w, (char*)workspace);
  weights_bf16(params, w, stream);
  for (int s = 0; s < steps; ++s) {
    load_batch(batch, xi, target, batch_idx + (int64_t)s * batch, w, stream);
    forward(params, batch, w, stream);
    backward(batch, w, stream);
    if (loss) ENS_HIP_TRY(hipMemcpyAsync(loss + s, w.loss, sizeof(float), hipMemcpyDeviceToDevice, stream));
    adam_launch(kParams, params, w.grad, adam_m, adam_v, step0 + s + 1, lr, stream);
    weights_bf16(params, w, stream);
    ENS_LAUNCH_CHECK();
  }
  return ENS_OK;
}

ens_status ens_mlp_adam(float* params, const float* grad, float* adam_m, float* adam_v, int64_t count, int32_t step,
                        float lr, hipStream_t stream) {
  ENS_ARG_CHECK(params && grad && adam_m && adam_v, "null pointer");
  ENS_ARG_CHECK(count >= 0 && step >= 1, "count must be >= 0 and step >= 1");
  ENS_ARG_CHECK(lr > 0.0f, "learning rate must be positive");
  ENS_ARG_CHECK(count <= INT32_MAX, "count must fit in int32");
  if (count == 0) return ENS_OK;
  adam_launch(count, params, grad, adam_m, adam_v, step, lr, stream);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

}  // extern "C"
