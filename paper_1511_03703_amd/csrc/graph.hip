// Q1 mesh sizes and the CRS graph of its stiffness matrix, built on the GPU.
//
// Fig. "crs" of Sec. 2 defines the storage (row_map, col_entry); the graph is
// the sample-independent data the ensemble reads once for all s samples.
// Row i holds every node that shares a hexahedron with node i, ascending.
// On the structured mesh that set is the clipped 3x3x3 block of neighbours,
// so each row's start and columns follow in closed form without a scan:
// with c(t) = 1 + [t > 0] + [t < N] neighbours per axis and
// P(t) = sum_{t' < t} c(t') = max(3t - 1, 0) (t <= N), row (i,j,k) starts at
//   P(k) C^2 + c(k) P(j) C + c(k) c(j) P(i),     C = 3N + 1.
#include "common.hpp"

namespace ens {

__device__ inline int axis_count(int t, int N) { return 1 + (t > 0) + (t < N); }
__device__ inline int64_t axis_prefix(int t) { return t > 0 ? 3 * (int64_t)t - 1 : 0; }

__global__ __launch_bounds__(256) void k_graph(int N, int32_t* __restrict__ row_ptr,
                                                int32_t* __restrict__ col_idx) {
  const int64_t n1 = N + 1;
  const int64_t n = n1 * n1 * n1;
  const int64_t C = 3 * (int64_t)N + 1;
  int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  int i = (int)(id % n1), j = (int)((id / n1) % n1), k = (int)(id / (n1 * n1));
  int ck = axis_count(k, N), cj = axis_count(j, N);
  int64_t start = axis_prefix(k) * C * C + ck * axis_prefix(j) * C + (int64_t)ck * cj * axis_prefix(i);
  row_ptr[id] = (int32_t)start;
  if (id == n - 1) row_ptr[n] = (int32_t)(C * C * C);
  int64_t pos = start;
  for (int dz = -1; dz <= 1; ++dz) {
    int z = k + dz;
    if (z < 0 || z > N) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      int y = j + dy;
      if (y < 0 || y > N) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        int x = i + dx;
        if (x < 0 || x > N) continue;
        col_idx[pos++] = (int32_t)(x + n1 * (y + n1 * z));
      }
    }
  }
}

}  // namespace ens

using namespace ens;

extern "C" {

ens_status ens_mesh_sizes(int32_t N, int64_t* n, int64_t* nnz, int64_t* n_elem) {
  ENS_ARG_CHECK(N >= 1, "N must be >= 1");
  int64_t n1 = (int64_t)N + 1, c = 3 * (int64_t)N + 1;
  int64_t nn = n1 * n1 * n1, nz = c * c * c;
  if (nn > INT32_MAX || nz > INT32_MAX) {
    set_error("mesh N=%d exceeds the int32 index range", N);
    return ENS_E_RANGE;
  }
  if (n) *n = nn;
  if (nnz) *nnz = nz;
  if (n_elem) *n_elem = (int64_t)N * N * N;
  return ENS_OK;
}

ens_status ens_graph_build(int32_t N, int32_t* row_ptr, int32_t* col_idx, hipStream_t stream) {
  int64_t n = 0, nnz = 0;
  ens_status st = ens_mesh_sizes(N, &n, &nnz, nullptr);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK(row_ptr && col_idx, "null graph pointer");
  int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_graph, dim3((unsigned)blocks), dim3(256), 0, stream, N, row_ptr, col_idx);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

}  // extern "C"
