// Ensemble Q1 assembly of the stiffness matrix and load vector.
//
// Alg. "assembly" (Sec. 4) loops over cells and scatters each element matrix
// into the global matrix with atomic adds.  Here the loop is turned inside
// out: a lane owns one matrix row (one node) of one sample, visits the (up
// to 8) elements around the node in ascending element id and adds the
// element row K_e[a_i][.] into a 27-entry register row.  No atomics are
// needed, each entry is 0 + K_e1 + K_e2 + ... in ascending element order,
// and since every K_e is formed from a symmetric table with the same
// operations for (a,b) and (b,a) the assembled matrix is bitwise symmetric.
// The coefficient at each element's Gauss points is evaluated once per
// workgroup tile into LDS (k_assemble_tile).  The writes of a row are
// sample-contiguous ([nnz][s]).
//
// Element matrix on the uniform mesh (h = 1/N, 2x2x2 Gauss, weight h^3/8):
//   K_e[a][b] = sum_q kappa_q (h/8) G_q[a][b],
//   G_q[a][b] = grad_ref N_a(g_q) . grad_ref N_b(g_q)       (dimensionless)
// kappa_q = kappa0 + sigma sum_m sqrt(lambda_m) phi_m(x_q) y_m, with the 1D
// factors of phi_m read from the KL table.
#include "common.hpp"
#include "mg.hpp"

namespace ens {

constexpr int kAsmMaxM = 16;

// Q1 element tables at the 2 x 2 x 2 Gauss points (Sec. 4, Alg. assembly),
// fixed at compile time: with the element loops unrolled every entry the
// kernels read is a known constant, and since the reference coordinate of
// a Gauss point along each axis is (1 -+ 1/sqrt 3)/2 the tables hold only
// a few distinct values, which the compiler keeps in registers instead of
// loading (and spilling) a table per element.
struct Q1Tables {
  double G[8][8][8];   // [q][a][b]: grad N_a . grad N_b (reference), symmetric in (a,b)
  double N[8][8];      // [q][a]: N_a at Gauss point q
  double dN[8][8][3];  // [q][a][d]: reference derivative of N_a along axis d
  double NN[8][8][8];  // [q][a][b]: N_a N_b at Gauss point q
};

constexpr Q1Tables q1_tables() {
  Q1Tables t{};
  const double r = 0.57735026918962576451;
  const double g[2] = {0.5 * (1.0 - r), 0.5 * (1.0 + r)};
  for (int q = 0; q < 8; ++q) {
    const double s3[3] = {g[q & 1], g[(q >> 1) & 1], g[(q >> 2) & 1]};
    for (int a = 0; a < 8; ++a) {
      const int ax[3] = {a & 1, (a >> 1) & 1, (a >> 2) & 1};
      double l[3] = {0.0, 0.0, 0.0}, d[3] = {0.0, 0.0, 0.0};
      for (int k = 0; k < 3; ++k) {
        l[k] = ax[k] ? s3[k] : 1.0 - s3[k];
        d[k] = ax[k] ? 1.0 : -1.0;
      }
      t.N[q][a] = l[0] * l[1] * l[2];
      t.dN[q][a][0] = d[0] * l[1] * l[2];
      t.dN[q][a][1] = l[0] * d[1] * l[2];
      t.dN[q][a][2] = l[0] * l[1] * d[2];
    }
    for (int a = 0; a < 8; ++a)
      for (int b = a; b < 8; ++b) {
        double dot = 0.0;
        for (int k = 0; k < 3; ++k) dot += t.dN[q][a][k] * t.dN[q][b][k];
        t.G[q][a][b] = dot;
        t.G[q][b][a] = dot;
      }
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b) t.NN[q][a][b] = t.N[q][a] * t.N[q][b];
  }
  return t;
}

__device__ constexpr Q1Tables kQ1 = q1_tables();

// 1D factors of the Q1 shape functions at the two Gauss points of an axis:
// kL1[q][b] = l_b(g_q), l_0 = 1 - t, l_1 = t, g_q = (1 -+ 1/sqrt 3)/2 (the
// same values the tables above are products of).
__device__ constexpr double kL1[2][2] = {
    {1.0 - 0.5 * (1.0 - 0.57735026918962576451), 0.5 * (1.0 - 0.57735026918962576451)},
    {1.0 - 0.5 * (1.0 + 0.57735026918962576451), 0.5 * (1.0 + 0.57735026918962576451)}};

// Sum of the KL modes of sample e at the 8 Gauss points of element
// (ex, ey, ez): kq[q] = kappa0 + sum_m c_m X(qx) Y(qy) Z(qz).
__device__ inline void kl_points(const double* __restrict__ tab, const int32_t* __restrict__ kl_triple,
                                 const double* __restrict__ cm, int M, int64_t two_n, int ex, int ey, int ez,
                                 double kappa0, double (&kq)[8]) {
#pragma unroll
  for (int q = 0; q < 8; ++q) kq[q] = 0.0;
#pragma unroll 2
  for (int m = 0; m < M; ++m) {
    const double c = cm[m];
    const double* px = tab + kl_triple[3 * m + 0] * two_n + 2 * ex;
    const double* py = tab + kl_triple[3 * m + 1] * two_n + 2 * ey;
    const double* pz = tab + kl_triple[3 * m + 2] * two_n + 2 * ez;
    const double fx[2] = {px[0], px[1]}, fy[2] = {py[0], py[1]}, fz[2] = {pz[0], pz[1]};
    double yz[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) yz[t] = c * (fy[t & 1] * fz[t >> 1]);
#pragma unroll
    for (int q = 0; q < 8; ++q) kq[q] += fx[q & 1] * yz[q >> 1];
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) kq[q] = kappa0 + kq[q];
}

// Node tiles of the assemblies: a workgroup owns R = TX x TY x TZ nodes
// (one lane per row and sample); the elements touching the tile form an
// EX x EY x EZ block.
template <int Rv, int TYv>
struct AsmTile {
  static constexpr int R = Rv;
  static constexpr int TY = TYv, TZ = 4, TX = R / (TY * TZ);
  static constexpr int EX = TX + 1, EY = TY + 1, EZ = TZ + 1, NE = EX * EY * EZ;
  static_assert(TX * TY * TZ == R, "tile shape");
};

// LDS slot of Gauss point q of tile element le for sample sb: the 8 points
// of an element are stored in the order q ^ (le & 7), so that the lanes of a
// wavefront, which read the same q of consecutive elements, hit different
// banks without padding the rows.
template <int SB>
__device__ inline int kslot(int le, int q, int sb) {
  return ((le * 8 + (q ^ (le & 7))) * SB) + sb;
}

// LDS doubles of a tile's KL factors: for each of the M modes its 1D
// eigenfunction at the 2 Gauss abscissae of each element column along x,
// and the products Y(qy) Z(qz) for each (y, z) element pair of the tile's
// element block.
template <int EX, int EY, int EZ>
__host__ __device__ constexpr int tab_doubles(int M) { return M * (2 * EX + 4 * EY * EZ); }

// Phase 1 of the tiled assemblies: the coefficient at the 8 Gauss points of
// every element of the tile's EX x EY x EZ element block (origin ex0, ey0,
// ez0) for the SB samples e0.., times `scale`, into s_k[kslot(le, q, sb)].
// The sample-independent factors are staged in s_tab first (the x factors
// and the y-z products, read from the KL table once per workgroup), and
// each lane keeps the coefficients c_m = sigma sqrt(lambda_m) y_m of its one
// sample in registers (the NT lanes are a multiple of SB, so a lane's items
// all have the same sample).  An item is one element and sample, its PTS =
// 8 Gauss points (PTS = 4: half an element, the lanes then a multiple of
// 2 SB with a fixed z half each); whole elements read 3 instead of 4 LDS
// factor pairs per 8 points and mode, which made the linear assembly 3.6 %
// faster (5.10 -> 4.92 ms in alternating runs).  The sum follows kl_points
// operation by operation (the y-z product is formed once per tile instead
// of per sample: the same rounding), so the values are bitwise those of
// kl_points whatever PTS.  Ends with a barrier.
template <int NT, int SB, int EX, int EY, int EZ, bool SCALED, int PTS = 4>
__device__ inline void tile_coefficients(int N, const double* __restrict__ kl_sqrt_lam,
                                         const int32_t* __restrict__ kl_triple, const double* __restrict__ kl_phi,
                                         int M, double kappa0, double sigma, const double* __restrict__ xi, int e0,
                                         int ex0, int ey0, int ez0, double scale, double* s_tab, double* s_k) {
  static_assert(PTS == 4 || PTS == 8, "an item is half an element or a whole one");
  constexpr int HALVES = 8 / PTS;  // z halves of an element held by different lanes
  static_assert(NT % (HALVES * SB) == 0, "a lane's items must share one sample and z half");
  constexpr int NE = EX * EY * EZ;
  const int64_t two_n = 2 * (int64_t)N;
  double* s_x = s_tab;               // [M][EX][2]
  double* s_yz = s_tab + M * 2 * EX;  // [M][EY][EZ][4], index qy + 2 qz
  for (int t = threadIdx.x; t < M * 2 * EX; t += NT) {
    const int m = t / (2 * EX), l = (t / 2) % EX, q = t & 1;
    const int el = ex0 + l;
    s_x[t] = (el >= 0 && el < N) ? kl_phi[kl_triple[3 * m] * two_n + 2 * el + q] : 0.0;
  }
  for (int t = threadIdx.x; t < M * 4 * EY * EZ; t += NT) {
    const int m = t / (4 * EY * EZ), r = t % (4 * EY * EZ);
    const int ly = r / (4 * EZ), lz = (r / 4) % EZ, qy = r & 1, qz = (r >> 1) & 1;
    const int ey = ey0 + ly, ez = ez0 + lz;
    double v = 0.0;
    if (ey >= 0 && ey < N && ez >= 0 && ez < N)
      v = kl_phi[kl_triple[3 * m + 1] * two_n + 2 * ey + qy] * kl_phi[kl_triple[3 * m + 2] * two_n + 2 * ez + qz];
    s_yz[t] = v;
  }
  const int sb = threadIdx.x % SB, hz = HALVES == 2 ? (threadIdx.x / SB) & 1 : 0;
  double c[kAsmMaxM];
#pragma unroll
  for (int m = 0; m < kAsmMaxM; ++m) c[m] = m < M ? sigma * kl_sqrt_lam[m] * xi[(int64_t)(e0 + sb) * M + m] : 0.0;
  __syncthreads();
  // a lane's items are elements le0, le0 + D, le0 + 2 D, ... (D = NT / 2 SB):
  // their block coordinates advance by D's digits with carries instead of
  // being divided out per item
  constexpr int D = NT / (HALVES * SB);
  constexpr int DX = D % EX, DY = (D / EX) % EY, DZ = D / (EX * EY);
  int le = threadIdx.x / (HALVES * SB);
  int lx = le % EX, ly = (le / EX) % EY, lz = le / (EX * EY);
  for (; le < NE; le += D) {
    const int ex = ex0 + lx, ey = ey0 + ly, ez = ez0 + lz;
    if (ex >= 0 && ey >= 0 && ez >= 0 && ex < N && ey < N && ez < N) {
      double kq[PTS];  // Gauss points qx + 2 qy + 4 (hz or qz)
#pragma unroll
      for (int q = 0; q < PTS; ++q) kq[q] = 0.0;
      const double* px = s_x + lx * 2;
      const double* pyz = s_yz + (ly * EZ + lz) * 4 + 2 * hz;
      // every mode up to the largest M, each skipped by a uniform branch
      // when absent: the coefficients stay in fixed registers
#pragma unroll
      for (int m = 0; m < kAsmMaxM; ++m) {
        if (m < M) {
          const double fx[2] = {px[m * 2 * EX], px[m * 2 * EX + 1]};
          double yz[PTS / 2];
#pragma unroll
          for (int j = 0; j < PTS / 2; ++j) yz[j] = c[m] * pyz[m * 4 * EY * EZ + j];
#pragma unroll
          for (int q = 0; q < PTS; ++q) kq[q] += fx[q & 1] * yz[q >> 1];
        }
      }
#pragma unroll
      for (int q = 0; q < PTS; ++q) {
        const double k = kappa0 + kq[q];
        s_k[kslot<SB>(le, q + 4 * hz, sb)] = SCALED ? k * scale : k;
      }
    }
    lx += DX;
    ly += DY;
    lz += DZ;
    if (lx >= EX) {
      lx -= EX;
      ++ly;
    }
    if (ly >= EY) {
      ly -= EY;
      ++lz;
    }
  }
  __syncthreads();
}

// Workgroup index -> (tile, sample group, tile origin).  Workgroups are
// dealt to the 8 XCDs round-robin by index; the G sample groups of one tile
// take indices 8 apart (same XCD, dispatched together) so their partial
// writes of each row's sample ensemble meet in one L2.
template <int TX, int TY, int TZ, int G>
__device__ inline void tile_decode(int N, int64_t bid, int64_t* tile_id, int* sg, int* x0, int* y0, int* z0) {
  const int n1 = N + 1;
  const int ntx = (n1 + TX - 1) / TX, nty = (n1 + TY - 1) / TY, ntz = (n1 + TZ - 1) / TZ;
  const int64_t tiles = (int64_t)ntx * ntz * nty;
  int64_t tile;
  if (G > 1 && (bid / (8 * G)) < tiles / 8) {
    const int64_t blk = bid / (8 * G), rem = bid % (8 * G);
    *sg = (int)(rem / 8);
    tile = blk * 8 + rem % 8;
  } else {
    const int64_t rest = bid - (tiles / 8) * 8 * G;  // the last tiles % 8 tiles, plainly
    *sg = (int)(G > 1 ? rest % G : 0);
    tile = (G > 1 ? (tiles / 8) * 8 + rest / G : bid);
  }
  *tile_id = tile;
  *x0 = (int)(tile % ntx) * TX;
  tile /= ntx;
  *z0 = (int)(tile % ntz) * TZ;
  *y0 = (int)(tile / ntz) * TY;
}

// Ensemble assembly (Alg. "assembly" made atomic-free by row ownership): a
// workgroup owns a 4 x 2 x 4 block of nodes for all S samples (32 S lanes,
// one per row and sample, sample fastest).  It first evaluates the
// coefficient (times h/8) at the 8 Gauss points of each of the 5 x 3 x 5
// elements touching the block, once per element and sample, into LDS
// (153.6 KB for s = 32; the Gauss points of an element in a swizzled order
// instead of padded rows); then each (row, sample) lane gathers its (up to
// 8) elements from LDS in ascending element id and adds the element rows in
// that fixed order, so the sums are deterministic and the coefficient is
// evaluated 2.3 times per row instead of 8.  A wavefront holds whole sample
// ensembles of its rows, so every store of a matrix entry writes full
// 128-byte lines (s = 32: two FP64 lines, one FP32 line); split over
// workgroups of fewer samples, the partial lines of the FP32 copy alone took
// longer than the whole assembly does now.
// BND (fused multigrid set-up of this level): 0 none; 1 D^-1 in FP32 and
// the Gershgorin bound of the FP32 values; 2 D^-1 and the bound of the FP64
// values.  Each lane forms its row's sum_j |a_ij| / a_ii in ascending entry
// order in FP64 exactly as k_mg_diag_bound does, and the workgroup writes
// the maximum over its rows per sample to bpart[tile][s].
// ADV: the advection-diffusion operator D + alpha C instead (the linear part
// of the nonlinear problem's Jacobian, Eq. fenl_lin_sys with beta = 0):
// every element row also gets alpha (h^2/8) C_ab, C_ab = sum_q N_a (v.dN_b)
// one 8x8 table per launch.
// The body of k_assemble_tile for tile `bid`; xzero (nullable): a solution
// [n][s] whose rows of the tile are set to zero too.
template <int S, int BND, bool ADV>
__device__ __forceinline__ void assemble_tile_body(int N, const double* __restrict__ kl_sqrt_lam,
                                                   const int32_t* __restrict__ kl_triple,
                                                   const double* __restrict__ kl_phi, int M, double kappa0,
                                                   double sigma, double fsrc, double alpha, double vx, double vy,
                                                   double vz, const double* __restrict__ xi,
                                                   const int32_t* __restrict__ row_ptr, double* __restrict__ values,
                                                   float* __restrict__ values32, double* __restrict__ rhs,
                                                   void* __restrict__ dinv, double* __restrict__ bpart, int64_t bid,
                                                   double* __restrict__ xzero) {
  using T = AsmTile<32, 2>;
  constexpr int SB = S, NT = T::R * S;
  constexpr int TX = T::TX, TY = T::TY, EX = T::EX, EY = T::EY, NE = T::NE;
  constexpr int NTAB = tab_doubles<T::EX, T::EY, T::EZ>(kAsmMaxM);
  static_assert(NT <= NE * 8 * SB && NTAB >= 64, "tile shape");
  // [kappa at the Gauss points, [element][q][sample] | the tile's 1D KL
  // factors]; after the coefficients the factor area takes the advection
  // table, after the row pass the kappa area the per-row bounds
  __shared__ double s_buf[NE * 8 * SB + NTAB];
  double* s_k = s_buf;
  double* s_tab = s_buf + NE * 8 * SB;
  double* s_adv = s_tab;
  const int n1 = N + 1;
  int64_t tile_id;
  int sg, x0, y0, z0;
  tile_decode<TX, TY, T::TZ, 1>(N, bid, &tile_id, &sg, &x0, &y0, &z0);
  const int e0 = 0;
  const double h = 1.0 / (double)N;
  tile_coefficients<NT, SB, EX, EY, T::EZ, true, 8>(N, kl_sqrt_lam, kl_triple, kl_phi, M, kappa0, sigma, xi, e0,
                                                  x0 - 1, y0 - 1, z0 - 1, h * 0.125, s_tab, s_k);
  if (ADV) {
    if (threadIdx.x < 64) {
      const int a = threadIdx.x >> 3, b = threadIdx.x & 7;
      double c = 0.0;
      for (int q = 0; q < 8; ++q)
        c += kQ1.N[q][a] * (vx * kQ1.dN[q][b][0] + vy * kQ1.dN[q][b][1] + vz * kQ1.dN[q][b][2]);
      s_adv[threadIdx.x] = c;
    }
    __syncthreads();
  }

  const int r = threadIdx.x / SB, sb = threadIdx.x % SB;
  const int rx = r % TX, ry = (r / TX) % TY, rz = r / (TX * TY);
  const int ii = x0 + rx, jj = y0 + ry, kk = z0 + rz;
  const bool live = ii <= N && jj <= N && kk <= N;
  if (!BND && !live) return;
  double qrow = 0.0;  // this row's Gershgorin ratio (BND)
  const int e = e0 + sb;
  if (live) {
  const int64_t row = (int64_t)ii + n1 * ((int64_t)jj + (int64_t)n1 * kk);

  double acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = 0.0;
  int nelem = 0;
#pragma unroll
  for (int ez_off = -1; ez_off <= 0; ++ez_off)
#pragma unroll
    for (int ey_off = -1; ey_off <= 0; ++ey_off)
#pragma unroll
      for (int ex_off = -1; ex_off <= 0; ++ex_off) {
        const int ex = ii + ex_off, ey = jj + ey_off, ez = kk + ez_off;
        if (ex < 0 || ey < 0 || ez < 0 || ex >= N || ey >= N || ez >= N) continue;
        ++nelem;
        const int ai = (-ex_off) + 2 * (-ey_off) + 4 * (-ez_off);
        const int le = (rx + 1 + ex_off) + EX * ((ry + 1 + ey_off) + EY * (rz + 1 + ez_off));
        double kq[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) kq[q] = s_k[kslot<SB>(le, q, sb)];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          if (b == ai) continue;  // the diagonal follows from the row sum below
          const int dx = ex_off + (b & 1), dy = ey_off + ((b >> 1) & 1), dz = ez_off + ((b >> 2) & 1);
          const int slot27 = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
          double kab = 0.0;
#pragma unroll
          for (int q = 0; q < 8; ++q) kab += kq[q] * kQ1.G[q][ai][b];
          if (ADV) kab += h * h * 0.125 * alpha * s_adv[ai * 8 + b];
          acc[slot27] += kab;
        }
      }

  // every element row sums to zero (the shape functions sum to one, so
  // sum_b grad N_b = 0, and C_ab = sum_q N_a v . grad N_b too), hence so
  // does the assembled row before the boundary conditions: its diagonal is
  // minus the sum of its other entries (added in ascending neighbour order),
  // which saves the 8 diagonal element entries' Gauss sums
  {
    double off = 0.0;
#pragma unroll
    for (int t = 0; t < 27; ++t)
      if (t != 13) off += acc[t];
    acc[13] = -off;
  }
  const bool bnd_row = (ii == 0 || ii == N || jj == 0 || jj == N || kk == 0 || kk == N);
  const int64_t start = row_ptr[row];
  double sabs = 0.0, dg = 0.0;
  // with 32 samples a wavefront's store covers whole 128-byte lines (FP32
  // and FP64), which then go out non-temporally (measured 4.98 -> 4.87 ms at
  // 128^3); smaller ensembles write partial lines, whose pieces are better
  // merged in L2 by ordinary stores
  constexpr bool NT = S == 32;
  auto st = [](auto* p, auto v) {
    if (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
  };
  auto put = [&](int64_t k, int slot27, double v) {
    if (values) st(values + k, v);
    if (values32) st(values32 + k, (float)v);
    if (BND) {
      const double vc = BND == 1 ? (double)(float)v : v;  // the value the cycle runs on
      sabs += fabs(vc);
      if (slot27 == 13) dg = vc;
    }
  };
  if (ii >= 2 && jj >= 2 && kk >= 2 && ii <= N - 2 && jj <= N - 2 && kk <= N - 2) {
    // all 27 neighbours interior: entry t of the row is neighbour t
#pragma unroll
    for (int t = 0; t < 27; ++t) put((start + t) * S + e, t, acc[t]);
  } else {
    int pos = 0;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int x = ii + dx, yy = jj + dy, z = kk + dz;
          if (x < 0 || yy < 0 || z < 0 || x > N || yy > N || z > N) continue;
          const int slot27 = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
          double v = acc[slot27];
          const bool bnd_col = (x == 0 || x == N || yy == 0 || yy == N || z == 0 || z == N);
          if (bnd_row) v = (slot27 == 13) ? 1.0 : 0.0;
          else if (bnd_col) v = 0.0;
          put((start + pos) * S + e, slot27, v);
          ++pos;
        }
  }
  st(rhs + row * S + e, bnd_row ? 0.0 : (double)nelem * (fsrc * h * h * h * 0.125));
  if (xzero) st(xzero + row * S + e, 0.0);
  if (BND == 1) st((float*)dinv + row * S + e, 1.0f / (float)dg);
  if (BND == 2) st((double*)dinv + row * S + e, 1.0 / dg);
  if (BND) qrow = sabs / dg;
  }
  if (BND) {
    __syncthreads();  // every lane is done with s_k
    double* s_q = s_k;
    s_q[threadIdx.x] = qrow;
    __syncthreads();
    if (threadIdx.x < SB) {
      double m = 0.0;
      for (int rr = 0; rr < T::R; ++rr) {
        const double q = s_q[rr * SB + threadIdx.x];
        m = q > m ? q : m;
      }
      bpart[tile_id * S + threadIdx.x] = m;
    }
  }
}

template <int S, int BND, bool ADV>
__global__ __launch_bounds__(32 * S) void k_assemble_tile(int N, const double* __restrict__ kl_sqrt_lam,
                                                           const int32_t* __restrict__ kl_triple,
                                                           const double* __restrict__ kl_phi, int M, double kappa0,
                                                           double sigma, double fsrc, double alpha, double vx,
                                                           double vy, double vz, const double* __restrict__ xi,
                                                           const int32_t* __restrict__ row_ptr,
                                                           double* __restrict__ values, float* __restrict__ values32,
                                                           double* __restrict__ rhs, void* __restrict__ dinv,
                                                           double* __restrict__ bpart) {
  assemble_tile_body<S, BND, ADV>(N, kl_sqrt_lam, kl_triple, kl_phi, M, kappa0, sigma, fsrc, alpha, vx, vy, vz, xi,
                                  row_ptr, values, values32, rhs, dinv, bpart, blockIdx.x, nullptr);
}

// The assemblies of every group of a batch in one launch: workgroup b takes
// tile b - tile0 of group blk_grp[b] (FP64 values and load vector, the
// solution set to zero).
template <int S>
__global__ __launch_bounds__(32 * S) void kb_assemble(const AsmGroupDev* __restrict__ groups,
                                                       const int32_t* __restrict__ blk_grp, int M, double kappa0,
                                                       double sigma, double fsrc) {
  const AsmGroupDev& g = groups[blk_grp[blockIdx.x]];
  assemble_tile_body<S, 0, false>(g.N, g.sq, g.tr, g.phi, M, kappa0, sigma, fsrc, 0.0, 0.0, 0.0, 0.0, g.xi, g.rp,
                                  g.values, nullptr, g.rhs, nullptr, nullptr, (int64_t)blockIdx.x - g.tile0, g.x);
}

// Residual and Jacobian of the nonlinear problem (Sec. 4, Eq.
// diffusion_sys, Eq. fenl_lin_sys, Alg. "assembly" with alpha, beta != 0),
// row-owned like k_assemble_tile (same tiling, the coefficient kept in LDS
// per patch element): lane e of a row's group gathers the element
// solution u_e of its sample for each element around the node (ascending
// element id) and forms the element's Jacobian row a
//   J_ab = D_ab + alpha (h^2/8) C_ab + 2 beta (h^3/8) sum_q u_q N_a N_b,
//   D_ab = (h/8) sum_q kappa_q G_q[a][b],   C_ab = sum_q N_a (v.dN_b)
// (C does not depend on the element: one 8x8 table per launch), with u_q
// the interpolated solution at Gauss point q.  Since the diffusion and
// advection terms are linear in u and the reaction term quadratic, the
// element residual is
//   F_a = sum_b (D_ab + alpha (h^2/8) C_ab + beta (h^3/8) sum_q u_q N_a N_b) u_b
//         - (h^3/8) f sum_q N_a,
// so no gradient of u_h is formed; the reaction sums sum_q u_q N_a N_b are
// contracted from the nodal values directly (the triple products of the
// shape functions factor over the axes), so u_h at the Gauss points is not
// formed either.  Boundary rows: F = u and identity rows;
// boundary columns of interior rows stored as zeros; load (optional) = the
// source part of F.
template <int S, int SB, bool JAC>
__global__ __launch_bounds__(32 * SB) void k_nl_assemble(int N, const double* __restrict__ kl_sqrt_lam,
                                                         const int32_t* __restrict__ kl_triple,
                                                         const double* __restrict__ kl_phi, int M, double kappa0,
                                                         double sigma, double fsrc, double alpha, double beta,
                                                         double vx, double vy, double vz, const double* __restrict__ xi,
                                                         const int32_t* __restrict__ row_ptr,
                                                         const double* __restrict__ u, double* __restrict__ values,
                                                         float* __restrict__ values32, double* __restrict__ F,
                                                         double* __restrict__ load) {
  // the workgroup tiling of k_assemble_tile (SB of the S samples of a
  // 4 x 2 x 4 node block), the coefficient kept raw (kappa0 + sum) in LDS;
  // after the coefficients the factor area holds the advection table
  // C_ab = sum_q N_a (v . dN_b)
  using T = AsmTile<32, 2>;
  constexpr int NT = T::R * SB, G = S / SB;
  constexpr int TX = T::TX, TY = T::TY, EX = T::EX, EY = T::EY, NE = T::NE;
  constexpr int NTAB = tab_doubles<T::EX, T::EY, T::EZ>(kAsmMaxM);
  static_assert(NTAB >= 64, "tile shape");
  __shared__ double s_buf[NE * 8 * SB + NTAB];
  double* s_k = s_buf;
  double* s_tab = s_buf + NE * 8 * SB;
  double* s_adv = s_tab;
  int64_t tile_id;
  int sg, x0, y0, z0;
  tile_decode<TX, TY, T::TZ, G>(N, blockIdx.x, &tile_id, &sg, &x0, &y0, &z0);
  const int e0 = sg * SB;
  tile_coefficients<NT, SB, EX, EY, T::EZ, false, 8>(N, kl_sqrt_lam, kl_triple, kl_phi, M, kappa0, sigma, xi, e0,
                                                   x0 - 1, y0 - 1, z0 - 1, 1.0, s_tab, s_k);
  if (threadIdx.x < 64) {
    const int a = threadIdx.x >> 3, b = threadIdx.x & 7;
    double c = 0.0;
    for (int q = 0; q < 8; ++q)
      c += kQ1.N[q][a] * (vx * kQ1.dN[q][b][0] + vy * kQ1.dN[q][b][1] + vz * kQ1.dN[q][b][2]);
    s_adv[threadIdx.x] = c;
  }
  __syncthreads();

  const int n1 = N + 1;
  const int rr = threadIdx.x / SB, sbl = threadIdx.x % SB;
  const int rx = rr % TX, ry = (rr / TX) % TY, rz = rr / (TX * TY);
  const int ii = x0 + rx, jj = y0 + ry, kk = z0 + rz;
  if (ii > N || jj > N || kk > N) return;
  const int e = e0 + sbl;
  const int64_t row = (int64_t)ii + n1 * ((int64_t)jj + (int64_t)n1 * kk);
  const double h = 1.0 / (double)N;
  const double wd = h * 0.125;             // diffusion: w_q / h^2
  const double wa = h * h * 0.125 * alpha; // advection: alpha w_q / h
  const double wr = h * h * h * 0.125;     // reaction and source: w_q
  const double wb = wr * beta;
  const double wrf = wr * fsrc;     // an element's load on a node

  double acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = 0.0;
  double fa = 0.0, la = 0.0;
  const bool bnd_row = (ii == 0 || ii == N || jj == 0 || jj == N || kk == 0 || kk == N);
  const int64_t start = JAC ? (int64_t)row_ptr[row] : 0;
  int pos = 0;
  // the entries of neighbour plane dz are final once the elements below
  // it are added (plane -1 after the lower elements, planes 0 and +1 after
  // all): stored then, in entry order, so fewer accumulators stay live
  const bool deep = ii >= 2 && jj >= 2 && kk >= 2 && ii <= N - 2 && jj <= N - 2 && kk <= N - 2;
  auto store_plane = [&](int dz) {
    if (deep) {  // all 27 neighbours interior: entry t of the row is neighbour t
#pragma unroll
      for (int t = (dz + 1) * 9; t < (dz + 2) * 9; ++t) {
        if (values) values[(start + t) * S + e] = acc[t];
        if (values32) values32[(start + t) * S + e] = (float)acc[t];
      }
      return;
    }
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int x = ii + dx, y = jj + dy, z = kk + dz;
        if (x < 0 || y < 0 || z < 0 || x > N || y > N || z > N) continue;
        const int slot27 = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
        double v = acc[slot27];
        const bool bnd_col = (x == 0 || x == N || y == 0 || y == N || z == 0 || z == N);
        if (bnd_row) v = (slot27 == 13) ? 1.0 : 0.0;
        else if (bnd_col) v = 0.0;
        if (values) values[(start + pos) * S + e] = v;
        if (values32) values32[(start + pos) * S + e] = (float)v;
        ++pos;
      }
  };

#pragma unroll
  for (int ez_off = -1; ez_off <= 0; ++ez_off) {
#pragma unroll
    for (int ey_off = -1; ey_off <= 0; ++ey_off)
#pragma unroll
      for (int ex_off = -1; ex_off <= 0; ++ex_off) {
          const int ex = ii + ex_off, ey = jj + ey_off, ez = kk + ez_off;
          if (ex < 0 || ey < 0 || ez < 0 || ex >= N || ey >= N || ez >= N) continue;
          const int ai = (-ex_off) + 2 * (-ey_off) + 4 * (-ez_off);
          const int le = (rx + 1 + ex_off) + EX * ((ry + 1 + ey_off) + EY * (rz + 1 + ez_off));
          double kq[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) kq[q] = s_k[kslot<SB>(le, q, sbl)];
          double ue[8];
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            const int64_t node = (int64_t)(ex + (b & 1)) + n1 * ((int64_t)(ey + ((b >> 1) & 1)) +
                                                                (int64_t)n1 * (ez + ((b >> 2) & 1)));
            ue[b] = u[node * S + e];
          }
          // the reaction row rn_b = sum_q u_h(q) N_a(q) N_b(q) = sum_c T_abc u_c,
          // T_abc = sum_q N_a N_b N_c, a product over the axes of the 1D
          // sums t(a, b, c) = sum_q l_a l_b l_c over the two Gauss points,
          // which are 1/2 when a = b = c and 1/6 otherwise: three 2-point
          // contractions of the element's nodal values, each pair (x0, x1)
          // giving (x0 + x1)/6 and that plus x_a/3 at the row's own index
          // (u_h at the Gauss points is never formed)
          double rnv[8];
          {
            constexpr double k6 = 1.0 / 6.0, k3 = 1.0 / 3.0;
            const int ax = ai & 1, ay = (ai >> 1) & 1, az = ai >> 2;
            double t1[8], t2[8];
#pragma unroll
            for (int r = 0; r < 8; r += 2) {  // along x: (cx) -> (bx), r = 2 cy + 4 cz
              const double m = (ue[r] + ue[r + 1]) * k6;
              t1[r + ax] = fma(ue[r + ax], k3, m);
              t1[r + 1 - ax] = m;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {  // along y: i0 = bx + 4 cz
              const int i0 = (k & 1) + 4 * (k >> 1);
              const double m = (t1[i0] + t1[i0 + 2]) * k6;
              t2[i0 + 2 * ay] = fma(t1[i0 + 2 * ay], k3, m);
              t2[i0 + 2 * (1 - ay)] = m;
            }
#pragma unroll
            for (int i0 = 0; i0 < 4; ++i0) {  // along z: i0 = bx + 2 by
              const double m = (t2[i0] + t2[i0 + 4]) * k6;
              rnv[i0 + 4 * az] = fma(t2[i0 + 4 * az], k3, m);
              rnv[i0 + 4 * (1 - az)] = m;
            }
          }
          la += wrf;  // sum_q N_a(q) = 1 for the 2-point rule
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            double dg = 0.0;
            const double rn = rnv[b];
#pragma unroll
            for (int q = 0; q < 8; ++q) dg += kq[q] * kQ1.G[q][ai][b];
            const double lin = wd * dg + wa * s_adv[ai * 8 + b];
            fa += (lin + wb * rn) * ue[b];
            if (JAC) {
              const int dx = ex_off + (b & 1), dy = ey_off + ((b >> 1) & 1), dz = ez_off + ((b >> 2) & 1);
              acc[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] += lin + 2.0 * wb * rn;
            }
          }
        }
    if (JAC) {
      if (ez_off < 0) store_plane(-1);
      else {
        store_plane(0);
        store_plane(1);
      }
    }
  }

  F[row * S + e] = bnd_row ? u[row * S + e] : fa - la;
  if (load) load[row * S + e] = bnd_row ? 0.0 : la;
}

// Per-sample extremes of the coefficient over the 8 N^3 Gauss points of
// the mesh, one workgroup per sample: each lane scans a stride of the
// elements and the workgroup folds its lanes' extremes (exact in any
// order).  A non-finite value makes both extremes NaN.
__device__ inline double ext_min(double a, double b) { return (a != a || b != b) ? NAN : (b < a ? b : a); }
__device__ inline double ext_max(double a, double b) { return (a != a || b != b) ? NAN : (b > a ? b : a); }

__global__ __launch_bounds__(256) void k_kl_extrema(int N, const double* __restrict__ kl_sqrt_lam,
                                                     const int32_t* __restrict__ kl_triple,
                                                     const double* __restrict__ kl_phi, int M, double kappa0,
                                                     double sigma, const double* __restrict__ xi,
                                                     double* __restrict__ kmin, double* __restrict__ kmax) {
  __shared__ double s_cm[kAsmMaxM];
  __shared__ double s_lo[256], s_hi[256];
  const int64_t e = blockIdx.x;
  if (threadIdx.x < M) s_cm[threadIdx.x] = sigma * kl_sqrt_lam[threadIdx.x] * xi[e * M + threadIdx.x];
  __syncthreads();
  const int64_t ne = (int64_t)N * N * N, two_n = 2 * (int64_t)N;
  double lo = INFINITY, hi = -INFINITY;
  for (int64_t el = threadIdx.x; el < ne; el += blockDim.x) {
    const int ex = (int)(el % N), ey = (int)((el / N) % N), ez = (int)(el / ((int64_t)N * N));
    double kq[8];
    kl_points(kl_phi, kl_triple, s_cm, M, two_n, ex, ey, ez, kappa0, kq);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      lo = ext_min(lo, kq[q]);
      hi = ext_max(hi, kq[q]);
    }
  }
  s_lo[threadIdx.x] = lo;
  s_hi[threadIdx.x] = hi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s_lo[threadIdx.x] = ext_min(s_lo[threadIdx.x], s_lo[threadIdx.x + w]);
      s_hi[threadIdx.x] = ext_max(s_hi[threadIdx.x], s_hi[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    kmin[e] = s_lo[0];
    kmax[e] = s_hi[0];
  }
}

template <int R, int TY>
static int64_t tiles_of(int N) {
  using T = AsmTile<R, TY>;
  return (int64_t)((N + T::TX) / T::TX) * ((N + T::TY) / T::TY) * ((N + T::TZ) / T::TZ);
}

// Samples per workgroup of the nonlinear assembly: 8 (256 lanes, 3 per CU;
// at 128^3, s = 32 this ran 7.9 ms per launch against 8.1 ms for all 32
// samples in one workgroup, whose full-line stores do not pay for its
// single workgroup per CU in this arithmetic-bound kernel).
static constexpr int nl_sb(int S) { return S < 8 ? S : 8; }

// Tiles of both assemblies (rows of the linear one's fused bound partials).
int64_t asm_tiles(int N, int S) {
  (void)S;
  return tiles_of<32, 2>(N);
}

ens_status batch_assemble_launch(int S, const AsmGroupDev* groups, const int32_t* blk_grp, int64_t blocks,
                                 const ens_problem& prob, hipStream_t st) {
  if (blocks <= 0) return ENS_OK;
  switch (S) {
#define ENS_BASM(SS)                                                                                         \
  case SS:                                                                                                   \
    hipLaunchKernelGGL(kb_assemble<SS>, dim3((unsigned)blocks), dim3(32 * SS), 0, st, groups, blk_grp, prob.M, \
                       prob.kappa0, prob.sigma, prob.f);                                                     \
    break;
    ENS_BASM(8)
    ENS_BASM(16)
    ENS_BASM(32)
#undef ENS_BASM
    default:
      set_error("batch ensemble size %d not compiled in (8, 16, 32)", S);
      return ENS_E_UNSUPPORTED;
  }
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}

ens_status assemble_launch(int N, const ens_graph* graph, const double* sq, const int32_t* tr, const double* phi,
                           const ens_problem* prob, int s, const double* xi, double* values, float* values32,
                           double* rhs, int bnd, void* dinv, double* bpart, hipStream_t stream, const double* adv) {
  int64_t n = 0, nnz = 0;
  ens_status st = ens_mesh_sizes(N, &n, &nnz, nullptr);
  if (st != ENS_OK) return st;
  const bool with_adv = adv && adv[0] != 0.0;
  if (with_adv && bnd == 0) {
    set_error("the advection-diffusion assembly is built only with a fused multigrid set-up");
    return ENS_E_UNSUPPORTED;
  }
  const double av[4] = {with_adv ? adv[0] : 0.0, with_adv ? adv[1] : 0.0, with_adv ? adv[2] : 0.0,
                        with_adv ? adv[3] : 0.0};
  const int M = prob->M;
  prof_begin(ENS_K_ASSEMBLE, stream);
  switch (s) {
#define ENS_ASM_LAUNCH(SS, BB, AA)                                                                                \
  hipLaunchKernelGGL((k_assemble_tile<SS, BB, AA>), dim3((unsigned)asm_tiles(N, SS)), dim3(32 * SS), 0, stream, N, sq, \
                     tr, phi, M, prob->kappa0, prob->sigma, prob->f, av[0], av[1], av[2], av[3], xi, graph->row_ptr,  \
                     values, values32, rhs, dinv, bpart)
#define ENS_ASM_CASE(SS)                                         \
  case SS:                                                       \
    if (with_adv && bnd == 1) ENS_ASM_LAUNCH(SS, 1, true);       \
    else if (with_adv && bnd == 2) ENS_ASM_LAUNCH(SS, 2, true);  \
    else if (bnd == 1) ENS_ASM_LAUNCH(SS, 1, false);             \
    else if (bnd == 2) ENS_ASM_LAUNCH(SS, 2, false);             \
    else ENS_ASM_LAUNCH(SS, 0, false);                           \
    break;
    ENS_ASM_CASE(4)
    ENS_ASM_CASE(8)
    ENS_ASM_CASE(16)
    ENS_ASM_CASE(32)
#undef ENS_ASM_CASE
#undef ENS_ASM_LAUNCH
  }
  ENS_LAUNCH_CHECK();
  double bytes = (double)nnz * s * ((values ? 8.0 : 0.0) + (values32 ? 4.0 : 0.0)) + (double)n * s * 8.0 + 4.0 * (n + 1);
  if (bnd) bytes += (double)n * s * (bnd == 1 ? 4.0 : 8.0);
  prof_end(ENS_K_ASSEMBLE, stream, bytes);
  return ENS_OK;
}

// The KL table's parts (layout of ens_kl_build).
void kl_parts(const void* kl, int M, const double** sq, const int32_t** tr, const double** phi) {
  const char* base = (const char*)kl;
  const size_t phi_off = ((size_t)M * 5 * sizeof(double) + (size_t)M * 4 * sizeof(int32_t) + 15) & ~(size_t)15;
  *sq = (const double*)base;
  *tr = (const int32_t*)(base + (size_t)M * 5 * sizeof(double) + (size_t)M * sizeof(int32_t));
  *phi = (const double*)(base + phi_off);
}

}  // namespace ens

using namespace ens;

extern "C" ens_status ens_assemble(int32_t N, const ens_graph* graph, const void* kl, const ens_problem* prob,
                                   int32_t s, const double* xi, double* values, float* values32, double* rhs,
                                   hipStream_t stream) {
  int64_t n = 0, nnz = 0;
  ens_status st = ens_mesh_sizes(N, &n, &nnz, nullptr);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK(graph && prob, "null graph or problem");
  ENS_ARG_CHECK(graph->n == n && graph->nnz == nnz && graph->row_ptr && graph->col_idx,
                "graph does not match the mesh");
  ENS_ARG_CHECK(values && rhs, "null output");
  ENS_ARG_CHECK(prob->M >= 0 && prob->M <= kAsmMaxM, "M out of range");
  ENS_ARG_CHECK(prob->M == 0 || (kl && xi), "null KL table or inputs");
  if (!supported_s(s)) {
    set_error("ensemble size %d not compiled in", s);
    return ENS_E_UNSUPPORTED;
  }
  const double *sq = nullptr, *phi = nullptr;
  const int32_t* tr = nullptr;
  kl_parts(kl, prob->M, &sq, &tr, &phi);
  return assemble_launch(N, graph, sq, tr, phi, prob, s, xi, values, values32, rhs, 0, nullptr, nullptr, stream,
                         nullptr);
}

extern "C" ens_status ens_nl_assemble(int32_t N, const ens_graph* graph, const void* kl,
                                      const ens_nl_problem* prob, int32_t s, const double* xi, const double* u,
                                      double* values, float* values32, double* F, double* load,
                                      hipStream_t stream) {
  int64_t n = 0, nnz = 0;
  ens_status st = ens_mesh_sizes(N, &n, &nnz, nullptr);
  if (st != ENS_OK) return st;
  ENS_ARG_CHECK(graph && prob, "null graph or problem");
  ENS_ARG_CHECK(graph->n == n && graph->nnz == nnz && graph->row_ptr && graph->col_idx,
                "graph does not match the mesh");
  ENS_ARG_CHECK(u && F, "null u or F");
  ENS_ARG_CHECK(prob->M >= 0 && prob->M <= kAsmMaxM, "M out of range");
  ENS_ARG_CHECK(prob->M == 0 || (kl && xi), "null KL table or inputs");
  if (!supported_s(s)) {
    set_error("ensemble size %d not compiled in", s);
    return ENS_E_UNSUPPORTED;
  }
  const int M = prob->M;
  const double *sq, *phi;
  const int32_t* tr;
  kl_parts(kl, M, &sq, &tr, &phi);
  prof_begin(ENS_K_NL_ASSEMBLE, stream);
  switch (s) {
#define ENS_NL_LAUNCH(SS, JJ)                                                                                    \
  hipLaunchKernelGGL((k_nl_assemble<SS, nl_sb(SS), JJ>), dim3((unsigned)(asm_tiles(N, SS) * (SS / nl_sb(SS)))),      \
                     dim3(32 * nl_sb(SS)), 0, stream, N, sq, tr,                                                      \
                     phi, M, prob->kappa0, prob->sigma, prob->f, prob->alpha, prob->beta, prob->vx, prob->vy,       \
                     prob->vz, xi, graph->row_ptr, u, values, values32, F, load)
#define ENS_NL_CASE(SS)                                  \
  case SS:                                               \
    if (values || values32) ENS_NL_LAUNCH(SS, true);     \
    else ENS_NL_LAUNCH(SS, false);                       \
    break;
    ENS_NL_CASE(4)
    ENS_NL_CASE(8)
    ENS_NL_CASE(16)
    ENS_NL_CASE(32)
#undef ENS_NL_CASE
#undef ENS_NL_LAUNCH
  }
  ENS_LAUNCH_CHECK();
  const double bytes = (values ? (double)nnz * s * 8.0 : 0.0) + (values32 ? (double)nnz * s * 4.0 : 0.0) +
                       (double)n * s * 8.0 * (load ? 3.0 : 2.0) + 4.0 * (n + 1);
  prof_end(ENS_K_NL_ASSEMBLE, stream, bytes);
  return ENS_OK;
}

extern "C" ens_status ens_kl_extrema(int32_t N, const void* kl, const ens_problem* prob, int32_t s,
                                     const double* xi, double* kmin, double* kmax, hipStream_t stream) {
  ENS_ARG_CHECK(N >= 1 && N <= 1024, "N out of range");
  ENS_ARG_CHECK(prob && s >= 1, "null problem or no samples");
  ENS_ARG_CHECK(prob->M >= 0 && prob->M <= kAsmMaxM, "M out of range");
  ENS_ARG_CHECK(prob->M == 0 || (kl && xi), "null KL table or inputs");
  ENS_ARG_CHECK(kmin && kmax, "null output");
  const double *sq = nullptr, *phi = nullptr;
  const int32_t* tr = nullptr;
  kl_parts(kl, prob->M, &sq, &tr, &phi);
  hipLaunchKernelGGL(k_kl_extrema, dim3((unsigned)s), dim3(256), 0, stream, N, sq, tr, phi, prob->M, prob->kappa0,
                     prob->sigma, xi, kmin, kmax);
  ENS_LAUNCH_CHECK();
  return ENS_OK;
}
