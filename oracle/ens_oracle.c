/*
 * ens_oracle.c -- plain, slow, obviously-correct FP64 CPU oracle for the
 * ensemble diffusion solve of Phipps et al., "Embedded Ensemble Propagation
 * for Improving Performance, Portability and Scalability of Uncertainty
 * Quantification on Emerging Computational Architectures" (arXiv 1511.03703).
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no source, header,
 * table or helper with the GPU library; the two meet only through seeded
 * input arrays generated outside both.
 *
 * What it computes (each function names the passage it follows):
 *   - the Q1 hexahedral mesh of the unit cube and the CRS graph of its
 *     stiffness matrix (Sec. 2, Fig. "crs"; Sec. 4, Alg. "assembly":
 *     NodeIndex / ElemGraph maps);
 *   - the truncated Karhunen-Loeve coefficient kappa(x,y) (Sec. 4, equations
 *     for kappa and the exponential covariance C(x,x'));
 *   - per-sample scalar finite-element assembly of A and f (Sec. 4,
 *     Alg. "assembly"), one sample at a time, scattered in ascending element
 *     order (the atomic scatter of the paper made sequential);
 *   - the scalar CRS product (Fig. "crs") and the ensemble product in the
 *     commuted layout (Fig. "ensemble_crs", Eq. kron_sys_commuted);
 *   - textbook Jacobi-preconditioned CG, one sample at a time (Sec. 3.4 uses
 *     CG; the ensemble system is block diagonal, Eq. kron_sys, so an ensemble
 *     solve with per-sample scalars is s independent scalar solves);
 *   - a dense Cholesky solve for brute-force checks on tiny meshes;
 *   - the nonlinear advection-diffusion-reaction residual and its Jacobian
 *     (Sec. 4, Eq. diffusion_sys and fenl_lin_sys, Alg. "assembly" with
 *     alpha, beta != 0), restarted right-preconditioned GMRES for the
 *     nonsymmetric Newton systems, and Newton's method per sample.
 *
 * Readings of points the paper leaves open (source term, boundary condition,
 * KL scaling and mode order, quadrature, stopping rule) are listed where they
 * are used.  Floating point: FP64 throughout; build with -ffp-contract=off so
 * every product and sum rounds as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_NOMEM (-4)

/* per-sample solver outcomes */
#define ORC_CONVERGED 0
#define ORC_MAXITER 1
#define ORC_BREAKDOWN 2
#define ORC_NONFINITE 3

/* ------------------------------------------------------------------------ */
/* Mesh (Sec. 4: D = [0,1]^3, linear finite elements on hexahedra).          */
/* Reading: N elements per axis, h = 1/N; node (i,j,k) has id                */
/* i + (N+1)(j + (N+1)k); element (ex,ey,ez) has id ex + N(ey + N ez);       */
/* local vertex a has bits (a&1, (a>>1)&1, (a>>2)&1) along x, y, z.          */
/* ------------------------------------------------------------------------ */

int64_t orc_num_nodes(int N) { return (int64_t)(N + 1) * (N + 1) * (N + 1); }
int64_t orc_num_elems(int N) { return (int64_t)N * N * N; }

static int64_t node_id(int N, int i, int j, int k) {
  return (int64_t)i + (int64_t)(N + 1) * ((int64_t)j + (int64_t)(N + 1) * k);
}

/* NodeIndex(e, a) of Alg. "assembly". */
static int64_t elem_node(int N, int64_t e, int a) {
  int ex = (int)(e % N), ey = (int)((e / N) % N), ez = (int)(e / ((int64_t)N * N));
  return node_id(N, ex + (a & 1), ey + ((a >> 1) & 1), ez + ((a >> 2) & 1));
}

static int is_boundary_node(int N, int64_t id) {
  int i = (int)(id % (N + 1));
  int j = (int)((id / (N + 1)) % (N + 1));
  int k = (int)(id / ((int64_t)(N + 1) * (N + 1)));
  return i == 0 || i == N || j == 0 || j == N || k == 0 || k == N;
}

static int cmp_int(const void *p, const void *q) {
  int a = *(const int *)p, b = *(const int *)q;
  return (a > b) - (a < b);
}

/* Row lengths of the CRS graph by its definition: column j appears in row i
 * iff nodes i and j are vertices of a common element.  Brute force over the
 * (at most 8) elements around node i and their 8 vertices each.           */
static int row_columns(int N, int64_t i, int *cols) {
  int ii = (int)(i % (N + 1));
  int jj = (int)((i / (N + 1)) % (N + 1));
  int kk = (int)(i / ((int64_t)(N + 1) * (N + 1)));
  int cand[64];
  int nc = 0;
  for (int dz = -1; dz <= 0; ++dz)
    for (int dy = -1; dy <= 0; ++dy)
      for (int dx = -1; dx <= 0; ++dx) {
        int ex = ii + dx, ey = jj + dy, ez = kk + dz;
        if (ex < 0 || ey < 0 || ez < 0 || ex >= N || ey >= N || ez >= N) continue;
        int64_t e = (int64_t)ex + (int64_t)N * ((int64_t)ey + (int64_t)N * ez);
        for (int a = 0; a < 8; ++a) cand[nc++] = (int)elem_node(N, e, a);
      }
  qsort(cand, (size_t)nc, sizeof(int), cmp_int);
  int n = 0;
  for (int t = 0; t < nc; ++t)
    if (n == 0 || cand[t] != cols[n - 1]) cols[n++] = cand[t];
  return n;
}

/* CRS graph (Fig. "crs": row_map / col_entry), columns ascending per row,
 * Dirichlet rows and columns kept in the pattern.  row_ptr has n+1 entries;
 * col_idx must hold nnz = row_ptr[n] entries (query with orc_graph_nnz).   */
int64_t orc_graph_nnz(int N) {
  if (N < 1) return -1;
  int cols[64];
  int64_t n = orc_num_nodes(N), nnz = 0;
  for (int64_t i = 0; i < n; ++i) nnz += row_columns(N, i, cols);
  return nnz;
}

int orc_graph(int N, int32_t *row_ptr, int32_t *col_idx) {
  if (N < 1 || !row_ptr || !col_idx) return ORC_E_ARG;
  int cols[64];
  int64_t n = orc_num_nodes(N), pos = 0;
  row_ptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    int c = row_columns(N, i, cols);
    for (int t = 0; t < c; ++t) col_idx[pos + t] = cols[t];
    pos += c;
    row_ptr[i + 1] = (int32_t)pos;
  }
  return ORC_OK;
}

/* Position of column J inside row I (binary search over the sorted row). */
static int64_t find_slot(const int32_t *row_ptr, const int32_t *col_idx, int64_t I, int64_t J) {
  int64_t lo = row_ptr[I], hi = row_ptr[I + 1] - 1;
  while (lo <= hi) {
    int64_t mid = (lo + hi) / 2;
    if (col_idx[mid] == J) return mid;
    if (col_idx[mid] < J) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

/* ElemGraph(e, a, b) of Alg. "assembly": absolute CRS index of entry
 * (NodeIndex(e,a), NodeIndex(e,b)).  Output [N^3][8][8].                  */
int orc_elem_slot(int N, const int32_t *row_ptr, const int32_t *col_idx, int64_t *slot) {
  if (N < 1) return ORC_E_ARG;
  int64_t ne = orc_num_elems(N);
  for (int64_t e = 0; e < ne; ++e)
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b) {
        int64_t s = find_slot(row_ptr, col_idx, elem_node(N, e, a), elem_node(N, e, b));
        if (s < 0) return ORC_E_ARG;
        slot[(e * 8 + a) * 8 + b] = s;
      }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Karhunen-Loeve coefficient (Sec. 4): kappa(x,y) = kappa0 +               */
/* sigma * sum_i kappa_i(x) y_i, with kappa_i eigenfunctions of the          */
/* exponential covariance exp(-|x-x'|_1 / L).                                */
/* Readings: kappa_i = sqrt(lambda_i) phi_i of the unit-variance kernel      */
/* (sigma in front of the sum carries the variance); the L1 distance makes   */
/* the kernel a product of 1D kernels exp(-|t-t'|/L), so 3D modes are        */
/* products of 1D modes on [0,1] and lambda_3D = product of 1D lambdas;      */
/* modes are ranked by lambda descending, ties broken by ascending           */
/* (ix,iy,iz), and each 3D lambda is formed from its three 1D factors taken  */
/* in ascending index order so permuted triples tie exactly.                 */
/* 1D eigenpairs on [-a,a] (a = 1/2 after centring t = x - 1/2, c = 1/L):    */
/*   even: c - w tan(w a) = 0,  phi = cos(w t) / sqrt(a + sin(2wa)/(2w))     */
/*   odd:  w + c tan(w a) = 0,  phi = sin(w t) / sqrt(a - sin(2wa)/(2w))     */
/*   lambda = 2c / (w^2 + c^2).                                              */
/* ------------------------------------------------------------------------ */

/* plain bisection on [lo, hi] for a function with g(lo) < 0 < g(hi)
 * after the sign normalisation sgn; run until the interval stops shrinking */
static double bisect(double (*g)(double, double, double), double a, double c, double lo, double hi) {
  double glo = g(lo, a, c);
  for (int it = 0; it < 2000; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    double gm = g(mid, a, c);
    if (gm == 0.0) return mid;
    if ((gm < 0.0) == (glo < 0.0)) { lo = mid; glo = gm; } else hi = mid;
  }
  return 0.5 * (lo + hi);
}

static double even_eq(double w, double a, double c) { return c - w * tan(w * a); }
static double odd_eq(double w, double a, double c) { return w + c * tan(w * a); }

/* First K 1D eigenpairs on [0,1] in lambda-descending order.
 * parity[k] = 0 (even / cosine) or 1 (odd / sine); nrm[k] = 1/sqrt(...)   */
int orc_kl_1d(int K, double L, double *omega, double *lam, double *nrm, int32_t *parity) {
  if (K < 1 || !(L > 0.0)) return ORC_E_ARG;
  const double a = 0.5, c = 1.0 / L, pi = acos(-1.0);
  for (int k = 0; k < K; ++k) {
    int m = k / 2 + 1; /* m-th root of its parity */
    double w;
    if (k % 2 == 0) {
      /* root in ((m-1) pi / a, (m - 1/2) pi / a) */
      double lo = (m - 1) * pi / a, hi = (m - 0.5) * pi / a;
      double eps = 1e-15 * hi;
      w = bisect(even_eq, a, c, lo + (m == 1 ? 0.0 : eps), hi - eps);
      nrm[k] = 1.0 / sqrt(a + sin(2.0 * w * a) / (2.0 * w));
      parity[k] = 0;
    } else {
      double lo = (m - 0.5) * pi / a, hi = m * pi / a;
      double eps = 1e-15 * hi;
      w = bisect(odd_eq, a, c, lo + eps, hi - eps);
      nrm[k] = 1.0 / sqrt(a - sin(2.0 * w * a) / (2.0 * w));
      parity[k] = 1;
    }
    omega[k] = w;
    lam[k] = 2.0 * c / (w * w + c * c);
  }
  return ORC_OK;
}

static double phi1d(double w, double nrm, int parity, double x) {
  double t = x - 0.5;
  return parity == 0 ? nrm * cos(w * t) : nrm * sin(w * t);
}

typedef struct { double lam; int i, j, k; } orc_triple;

static int cmp_triple(const void *p, const void *q) {
  const orc_triple *A = (const orc_triple *)p, *B = (const orc_triple *)q;
  if (A->lam > B->lam) return -1;
  if (A->lam < B->lam) return 1;
  if (A->i != B->i) return A->i < B->i ? -1 : 1;
  if (A->j != B->j) return A->j < B->j ? -1 : 1;
  if (A->k != B->k) return A->k < B->k ? -1 : 1;
  return 0;
}

static double lam_product(const double *lam1, int i, int j, int k) {
  int v[3] = {i, j, k};
  /* ascending index order */
  for (int p = 0; p < 3; ++p)
    for (int q = p + 1; q < 3; ++q)
      if (v[q] < v[p]) { int t = v[p]; v[p] = v[q]; v[q] = t; }
  return (lam1[v[0]] * lam1[v[1]]) * lam1[v[2]];
}

/* First M 3D modes: triples[m] = (ix, iy, iz) 1D ranks, lam3[m].
 * A mode of rank m cannot use a 1D index >= M (the M modes (i,0,0), i < M,
 * dominate it), so M 1D modes per axis suffice.                          */
int orc_kl_modes(int M, double L, int32_t *triples, double *lam3) {
  if (M < 1) return ORC_E_ARG;
  double *w = malloc(sizeof(double) * M), *l1 = malloc(sizeof(double) * M), *nr = malloc(sizeof(double) * M);
  int32_t *par = malloc(sizeof(int32_t) * M);
  orc_triple *all = malloc(sizeof(orc_triple) * (size_t)M * M * M);
  if (!w || !l1 || !nr || !par || !all) return ORC_E_NOMEM;
  orc_kl_1d(M, L, w, l1, nr, par);
  int64_t t = 0;
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < M; ++j)
      for (int k = 0; k < M; ++k) {
        all[t].lam = lam_product(l1, i, j, k);
        all[t].i = i; all[t].j = j; all[t].k = k;
        ++t;
      }
  qsort(all, (size_t)t, sizeof(orc_triple), cmp_triple);
  for (int m = 0; m < M; ++m) {
    triples[3 * m] = all[m].i; triples[3 * m + 1] = all[m].j; triples[3 * m + 2] = all[m].k;
    lam3[m] = all[m].lam;
  }
  free(w); free(l1); free(nr); free(par); free(all);
  return ORC_OK;
}

/* kappa at arbitrary points pts[npts][3] for one sample y = xi[M]. */
int orc_kl_coef_points(int M, double L, double kappa0, double sigma, const double *xi,
                       int64_t npts, const double *pts, double *out) {
  if (M < 0 || (M > 0 && !xi)) return ORC_E_ARG;
  int Mk = M > 0 ? M : 1;
  double *w = malloc(sizeof(double) * Mk), *l1 = malloc(sizeof(double) * Mk), *nr = malloc(sizeof(double) * Mk);
  int32_t *par = malloc(sizeof(int32_t) * Mk), *tr = malloc(sizeof(int32_t) * 3 * Mk);
  double *l3 = malloc(sizeof(double) * Mk);
  if (M > 0) {
    orc_kl_1d(M, L, w, l1, nr, par);
    orc_kl_modes(M, L, tr, l3);
  }
  for (int64_t p = 0; p < npts; ++p) {
    double sum = 0.0;
    for (int m = 0; m < M; ++m) {
      int i = tr[3 * m], j = tr[3 * m + 1], k = tr[3 * m + 2];
      double phi = phi1d(w[i], nr[i], par[i], pts[3 * p]) *
                   phi1d(w[j], nr[j], par[j], pts[3 * p + 1]) *
                   phi1d(w[k], nr[k], par[k], pts[3 * p + 2]);
      sum += sqrt(l3[m]) * phi * xi[m];
    }
    out[p] = kappa0 + sigma * sum;
  }
  free(w); free(l1); free(nr); free(par); free(tr); free(l3);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Quadrature (Alg. "assembly": N_qp = 8).  Reading: the tensor 2x2x2        */
/* Gauss-Legendre rule; abscissae (1 -+ 1/sqrt 3)/2 on [0,1], weight 1/2     */
/* each; qp index q = qx + 2 qy + 4 qz; physical point                       */
/* ((ex + g_qx)/N, (ey + g_qy)/N, (ez + g_qz)/N), weight h^3/8.              */
/* ------------------------------------------------------------------------ */

static double gauss01(int q) {
  double r = 1.0 / sqrt(3.0);
  return q == 0 ? 0.5 * (1.0 - r) : 0.5 * (1.0 + r);
}

/* Coordinates of all quadrature points, [N^3][8][3]. */
int orc_qp_coords(int N, double *pts) {
  if (N < 1) return ORC_E_ARG;
  int64_t ne = orc_num_elems(N);
  for (int64_t e = 0; e < ne; ++e) {
    int ex = (int)(e % N), ey = (int)((e / N) % N), ez = (int)(e / ((int64_t)N * N));
    for (int q = 0; q < 8; ++q) {
      double *p = pts + (e * 8 + q) * 3;
      p[0] = ((double)ex + gauss01(q & 1)) / (double)N;
      p[1] = ((double)ey + gauss01((q >> 1) & 1)) / (double)N;
      p[2] = ((double)ez + gauss01((q >> 2) & 1)) / (double)N;
    }
  }
  return ORC_OK;
}

/* kappa at every quadrature point of every element, [N^3][8]. */
int orc_kl_coef_qp(int N, int M, double L, double kappa0, double sigma, const double *xi, double *acoef) {
  if (N < 1) return ORC_E_ARG;
  int64_t np = orc_num_elems(N) * 8;
  double *pts = malloc(sizeof(double) * 3 * (size_t)np);
  if (!pts) return ORC_E_NOMEM;
  orc_qp_coords(N, pts);
  int rc = orc_kl_coef_points(M, L, kappa0, sigma, xi, np, pts, acoef);
  free(pts);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Scalar assembly of one sample (Alg. "assembly", with alpha = beta = 0 so  */
/* the residual is linear and the Jacobian is the stiffness matrix).         */
/*   K_e[a][b] = sum_q kappa(x_q) grad N_a(x_q) . grad N_b(x_q) w_q          */
/*   f_e[a]    = sum_q f(x_q) N_a(x_q) w_q                                   */
/* Shape functions N_a = l_{ax}(s) l_{ay}(t) l_{az}(u), l0 = 1-t, l1 = t;    */
/* on the uniform mesh grad_x = grad_ref / h.  K_e is formed for a <= b and  */
/* mirrored.  The scatter runs over elements in ascending id, so each global */
/* entry is 0 + (contributions in ascending element order).                  */
/* Source: src_kind 0 -> f = fconst; 1 -> f = 3 pi^2 sin(pi x)sin(pi y)      */
/* sin(pi z) (manufactured solution u = sin sin sin at kappa = 1).           */
/* Dirichlet reading (u = 0 on the boundary): boundary rows become identity  */
/* rows, interior rows drop their boundary columns (stored as zeros), and    */
/* boundary load entries are zero.                                            */
/* ------------------------------------------------------------------------ */

static double lfun(int a, double t) { return a ? t : 1.0 - t; }
static double dlfun(int a) { return a ? 1.0 : -1.0; }

int orc_assemble_scalar(int N, const int32_t *row_ptr, const int32_t *col_idx,
                        const double *acoef, int src_kind, double fconst, int dirichlet,
                        double *values, double *rhs) {
  if (N < 1 || !row_ptr || !col_idx || !acoef || !values || !rhs) return ORC_E_ARG;
  const double h = 1.0 / (double)N;
  const double wq = h * h * h / 8.0;
  const double pi = acos(-1.0);
  int64_t n = orc_num_nodes(N), nnz = row_ptr[n], ne = orc_num_elems(N);
  for (int64_t k = 0; k < nnz; ++k) values[k] = 0.0;
  for (int64_t i = 0; i < n; ++i) rhs[i] = 0.0;

  /* reference values and gradients at the 8 quadrature points */
  double Nq[8][8], G[8][8][3];
  for (int q = 0; q < 8; ++q) {
    double s = gauss01(q & 1), t = gauss01((q >> 1) & 1), u = gauss01((q >> 2) & 1);
    for (int a = 0; a < 8; ++a) {
      int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
      Nq[q][a] = lfun(ax, s) * lfun(ay, t) * lfun(az, u);
      G[q][a][0] = dlfun(ax) * lfun(ay, t) * lfun(az, u) / h;
      G[q][a][1] = lfun(ax, s) * dlfun(ay) * lfun(az, u) / h;
      G[q][a][2] = lfun(ax, s) * lfun(ay, t) * dlfun(az) / h;
    }
  }
  for (int64_t e = 0; e < ne; ++e) {
    double Ke[8][8], fe[8];
    for (int a = 0; a < 8; ++a) {
      for (int b = a; b < 8; ++b) {
        double sum = 0.0;
        for (int q = 0; q < 8; ++q) {
          double dot = G[q][a][0] * G[q][b][0] + G[q][a][1] * G[q][b][1] + G[q][a][2] * G[q][b][2];
          sum += acoef[e * 8 + q] * dot * wq;
        }
        Ke[a][b] = sum;
        Ke[b][a] = sum;
      }
      double fs = 0.0;
      for (int q = 0; q < 8; ++q) {
        double f = fconst;
        if (src_kind == 1) {
          int ex = (int)(e % N), ey = (int)((e / N) % N), ez = (int)(e / ((int64_t)N * N));
          double x = ((double)ex + gauss01(q & 1)) / (double)N;
          double y = ((double)ey + gauss01((q >> 1) & 1)) / (double)N;
          double z = ((double)ez + gauss01((q >> 2) & 1)) / (double)N;
          f = 3.0 * pi * pi * sin(pi * x) * sin(pi * y) * sin(pi * z);
        }
        fs += f * Nq[q][a] * wq;
      }
      fe[a] = fs;
    }
    for (int a = 0; a < 8; ++a) {
      int64_t I = elem_node(N, e, a);
      rhs[I] += fe[a];
      for (int b = 0; b < 8; ++b) {
        int64_t slot = find_slot(row_ptr, col_idx, I, elem_node(N, e, b));
        values[slot] += Ke[a][b];
      }
    }
  }
  if (dirichlet) {
    for (int64_t i = 0; i < n; ++i) {
      int bi = is_boundary_node(N, i);
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        if (bi) values[k] = (col_idx[k] == i) ? 1.0 : 0.0;
        else if (is_boundary_node(N, col_idx[k])) values[k] = 0.0;
      }
      if (bi) rhs[i] = 0.0;
    }
  }
  return ORC_OK;
}

/* Ensemble assembly in the commuted layout (Eq. kron_sys_commuted):
 * values[k*s + e], rhs[i*s + e].  Plainly a loop over samples, each one a
 * scalar KL evaluation plus scalar assembly, interleaved afterwards.      */
int orc_assemble_ensemble(int N, const int32_t *row_ptr, const int32_t *col_idx,
                          int M, double L, double kappa0, double sigma, double fconst,
                          int s, const double *xi, double *values, double *rhs) {
  if (N < 1 || s < 1) return ORC_E_ARG;
  int64_t n = orc_num_nodes(N), nnz = row_ptr[n], ne = orc_num_elems(N);
  int rc = ORC_OK;
  #pragma omp parallel for schedule(dynamic, 1)
  for (int e = 0; e < s; ++e) {
    double *ac = malloc(sizeof(double) * 8 * (size_t)ne);
    double *v = malloc(sizeof(double) * (size_t)nnz);
    double *f = malloc(sizeof(double) * (size_t)n);
    if (!ac || !v || !f) { rc = ORC_E_NOMEM; free(ac); free(v); free(f); continue; }
    orc_kl_coef_qp(N, M, L, kappa0, sigma, xi + (int64_t)e * M, ac);
    orc_assemble_scalar(N, row_ptr, col_idx, ac, 0, fconst, 1, v, f);
    for (int64_t k = 0; k < nnz; ++k) values[k * s + e] = v[k];
    for (int64_t i = 0; i < n; ++i) rhs[i * s + e] = f[i];
    free(ac); free(v); free(f);
  }
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Sparse products                                                           */
/* ------------------------------------------------------------------------ */

/* z = A x for one scalar matrix (Fig. "crs"). */
void orc_spmv(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *values,
              const double *x, double *z) {
  for (int64_t row = 0; row < n; ++row) {
    double sum = 0.0;
    for (int64_t k = row_ptr[row]; k < row_ptr[row + 1]; ++k) sum += values[k] * x[col_idx[k]];
    z[row] = sum;
  }
}

/* Ensemble product in the commuted layout (Fig. "ensemble_crs"):
 * sample loop innermost, one partial sum per sample, values[k*s+e].       */
void orc_ens_spmv(int64_t n, int s, const int32_t *row_ptr, const int32_t *col_idx,
                  const double *values, const double *x, double *z) {
  double *sum = malloc(sizeof(double) * (size_t)s);
  for (int64_t row = 0; row < n; ++row) {
    for (int e = 0; e < s; ++e) sum[e] = 0.0;
    for (int64_t k = row_ptr[row]; k < row_ptr[row + 1]; ++k) {
      int64_t col = col_idx[k];
      for (int e = 0; e < s; ++e) sum[e] += values[k * s + e] * x[col * s + e];
    }
    for (int e = 0; e < s; ++e) z[row * s + e] = sum[e];
  }
  free(sum);
}

/* ------------------------------------------------------------------------ */
/* Jacobi-preconditioned CG for one sample (Sec. 3.4: CG; preconditioner     */
/* D = diag(A), the trivial instance of M_c = sum M_i (x) e_i e_i^T).        */
/* Readings: stop when the recursive residual satisfies |r|_2 <= rtol |b|_2  */
/* (one iteration = one product q = A p); |b| = 0 gives x = 0; a start with  */
/* |r0| <= rtol |b| takes 0 iterations; p.q <= 0 or non-finite scalars stop  */
/* the sample with a breakdown / non-finite status.  fixed_iters >= 0 runs   */
/* exactly that many iterations with the tolerance test switched off (used   */
/* to compare against another implementation at equal iteration counts).     */
/* rel_res is the true residual |b - A x| / |b| of the returned x.           */
/* ------------------------------------------------------------------------ */

static double dot(int64_t n, const double *u, const double *v) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += u[i] * v[i];
  return s;
}

int orc_pcg(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *values,
            const double *b, double *x, double rtol, int max_iter, int fixed_iters,
            int32_t *iters_out, double *rel_res_out, int32_t *status_out) {
  double *r = malloc(sizeof(double) * (size_t)n), *z = malloc(sizeof(double) * (size_t)n);
  double *p = malloc(sizeof(double) * (size_t)n), *q = malloc(sizeof(double) * (size_t)n);
  double *dinv = malloc(sizeof(double) * (size_t)n);
  if (!r || !z || !p || !q || !dinv) return ORC_E_NOMEM;
  int status = ORC_CONVERGED, iters = 0;
  for (int64_t i = 0; i < n; ++i) {
    double d = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
      if (col_idx[k] == i) d = values[k];
    dinv[i] = 1.0 / d;
  }
  double nb = sqrt(dot(n, b, b));
  if (nb == 0.0) {
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    *iters_out = 0; *rel_res_out = 0.0; *status_out = ORC_CONVERGED;
    free(r); free(z); free(p); free(q); free(dinv);
    return ORC_OK;
  }
  orc_spmv(n, row_ptr, col_idx, values, x, q);
  for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
  int limit = fixed_iters >= 0 ? fixed_iters : max_iter;
  int test = fixed_iters < 0;
  if (test && sqrt(dot(n, r, r)) <= rtol * nb) {
    limit = 0;
  } else {
    for (int64_t i = 0; i < n; ++i) { z[i] = dinv[i] * r[i]; p[i] = z[i]; }
    double rho = dot(n, r, z);
    status = ORC_MAXITER;
    for (int k = 1; k <= limit; ++k) {
      orc_spmv(n, row_ptr, col_idx, values, p, q);
      double eta = dot(n, p, q);
      if (!isfinite(eta) || !isfinite(rho)) { status = ORC_NONFINITE; break; }
      if (!(eta > 0.0)) { status = ORC_BREAKDOWN; break; }
      double alpha = rho / eta;
      for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
      iters = k;
      double rr = dot(n, r, r);
      if (!isfinite(rr)) { status = ORC_NONFINITE; break; }
      if (test && sqrt(rr) <= rtol * nb) { status = ORC_CONVERGED; break; }
      if (!test && k == limit) { status = ORC_CONVERGED; break; }
      for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
      double rho_new = dot(n, r, z);
      double beta = rho_new / rho;
      for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
      rho = rho_new;
    }
    if (!test && limit == 0) status = ORC_CONVERGED;
  }
  orc_spmv(n, row_ptr, col_idx, values, x, q);
  for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
  *iters_out = iters;
  *rel_res_out = sqrt(dot(n, r, r)) / nb;
  *status_out = status;
  free(r); free(z); free(p); free(q); free(dinv);
  return ORC_OK;
}

/* Ensemble solve with per-sample scalars: by the block-diagonal structure
 * of the Kronecker system (Eq. kron_sys) this is exactly s scalar solves.
 * values [nnz][s], b and x [n][s]; fixed_iters nullable ([s], -1 = off).  */
int orc_ens_pcg(int64_t n, int s, const int32_t *row_ptr, const int32_t *col_idx,
                const double *values, const double *b, double *x, double rtol, int max_iter,
                const int32_t *fixed_iters, int32_t *iters, double *rel_res, int32_t *status) {
  int64_t nnz = row_ptr[n];
  int rc = ORC_OK;
  #pragma omp parallel for schedule(dynamic, 1)
  for (int e = 0; e < s; ++e) {
    double *v = malloc(sizeof(double) * (size_t)nnz);
    double *be = malloc(sizeof(double) * (size_t)n), *xe = malloc(sizeof(double) * (size_t)n);
    if (!v || !be || !xe) { rc = ORC_E_NOMEM; free(v); free(be); free(xe); continue; }
    for (int64_t k = 0; k < nnz; ++k) v[k] = values[k * s + e];
    for (int64_t i = 0; i < n; ++i) { be[i] = b[i * s + e]; xe[i] = x[i * s + e]; }
    int r = orc_pcg(n, row_ptr, col_idx, v, be, xe, rtol, max_iter,
                    fixed_iters ? fixed_iters[e] : -1, &iters[e], &rel_res[e], &status[e]);
    if (r) rc = r;
    for (int64_t i = 0; i < n; ++i) x[i * s + e] = xe[i];
    free(v); free(be); free(xe);
  }
  return rc;
}

/* Coupled ensemble solve (the paper's solve of the whole commuted system,
 * Sec. 3.4 and Sec. 3.7): the ensemble inner products are summed over the
 * samples, so CG runs on the block-diagonal system blockdiag(A_1 .. A_s) of
 * Eq. kron_sys as ONE system, with one alpha and beta for all samples and one
 * stopping test on the norms over all samples.  Written out literally: the
 * block-diagonal CRS matrix (sample-major: row e*n + i) is built and the
 * scalar Jacobi-PCG above is run on it.  x, b [n][s] (commuted layout);
 * iters/rel_res/status describe the whole system.                         */
int orc_ens_pcg_coupled(int64_t n, int s, const int32_t *row_ptr, const int32_t *col_idx,
                        const double *values, const double *b, double *x, double rtol, int max_iter,
                        int fixed_iters, int32_t *iters, double *rel_res, int32_t *status) {
  int64_t nnz = row_ptr[n];
  int64_t N = n * s, NZ = nnz * s;
  if (s < 1 || N > INT32_MAX || NZ > INT32_MAX) return ORC_E_ARG;
  int32_t *rp = calloc((size_t)(N + 1), sizeof(int32_t)), *ci = calloc((size_t)NZ + 1, sizeof(int32_t));
  double *v = calloc((size_t)NZ + 1, sizeof(double));
  double *bb = calloc((size_t)N + 1, sizeof(double)), *xx = calloc((size_t)N + 1, sizeof(double));
  if (!rp || !ci || !v || !bb || !xx) {
    free(rp); free(ci); free(v); free(bb); free(xx);
    return ORC_E_NOMEM;
  }
  rp[0] = 0;
  for (int e = 0; e < s; ++e)
    for (int64_t i = 0; i < n; ++i) {
      const int64_t row = e * n + i;
      rp[row + 1] = (int32_t)(rp[row] + (row_ptr[i + 1] - row_ptr[i]));
      int64_t o = rp[row];
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k, ++o) {
        ci[o] = (int32_t)(e * n + col_idx[k]);
        v[o] = values[k * s + e];
      }
      bb[row] = b[i * s + e];
      xx[row] = x[i * s + e];
    }
  int rc = orc_pcg(N, rp, ci, v, bb, xx, rtol, max_iter, fixed_iters, iters, rel_res, status);
  for (int e = 0; e < s; ++e)
    for (int64_t i = 0; i < n; ++i) x[i * s + e] = xx[e * n + i];
  free(rp); free(ci); free(v); free(bb); free(xx);
  return rc;
}

/* One complete sample from scratch: graph, KL coefficient, assembly and
 * Jacobi-CG from a zero guess.  x [n] out.  Used for full-size checks and
 * as the CPU baseline.                                                    */
static double wall_seconds(void) {
#ifdef _OPENMP
  return omp_get_wtime();
#else
  return 0.0;
#endif
}

int orc_solve_sample(int N, int M, double L, double kappa0, double sigma, double fconst,
                     const double *xi, double rtol, int max_iter, double *x,
                     int32_t *iters, double *rel_res, int32_t *status, double *timing) {
  double t0 = wall_seconds();
  int64_t n = orc_num_nodes(N), ne = orc_num_elems(N);
  int64_t nnz = orc_graph_nnz(N);
  int32_t *rp = malloc(sizeof(int32_t) * (size_t)(n + 1)), *ci = malloc(sizeof(int32_t) * (size_t)nnz);
  double *ac = malloc(sizeof(double) * 8 * (size_t)ne), *v = malloc(sizeof(double) * (size_t)nnz);
  double *b = malloc(sizeof(double) * (size_t)n);
  if (!rp || !ci || !ac || !v || !b) return ORC_E_NOMEM;
  orc_graph(N, rp, ci);
  orc_kl_coef_qp(N, M, L, kappa0, sigma, xi, ac);
  orc_assemble_scalar(N, rp, ci, ac, 0, fconst, 1, v, b);
  for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
  double t1 = wall_seconds();
  int rc = orc_pcg(n, rp, ci, v, b, x, rtol, max_iter, -1, iters, rel_res, status);
  double t2 = wall_seconds();
  if (timing) { timing[0] = t1 - t0; timing[1] = t2 - t1; }
  free(rp); free(ci); free(ac); free(v); free(b);
  return rc;
}

/* Several samples of orc_solve_sample in parallel, one per thread.
 * xi [count][M]; x [count][n] (sample-major, nullable); timing [count][2]
 * (nullable) receives each sample's set-up and solve wall seconds; returns
 * the number of threads used in *threads_used.                            */
int orc_solve_samples(int N, int M, double L, double kappa0, double sigma, double fconst,
                      int count, const double *xi, double rtol, int max_iter, double *x,
                      int32_t *iters, double *rel_res, int32_t *status, int32_t *threads_used,
                      double *timing) {
  int64_t n = orc_num_nodes(N);
  int rc = ORC_OK;
  int used = 1;
  #pragma omp parallel
  {
#ifdef _OPENMP
    #pragma omp single
    used = omp_get_num_threads();
#endif
    #pragma omp for schedule(dynamic, 1)
    for (int e = 0; e < count; ++e) {
      double *xe = x ? x + (int64_t)e * n : malloc(sizeof(double) * (size_t)n);
      int r = orc_solve_sample(N, M, L, kappa0, sigma, fconst, xi + (int64_t)e * M, rtol, max_iter,
                               xe, &iters[e], &rel_res[e], &status[e], timing ? timing + 2 * e : NULL);
      if (r) rc = r;
      if (!x) free(xe);
    }
  }
  if (threads_used) *threads_used = used < count ? used : count;
  return rc;
}

/* True residual |b - A x| / |b| per sample in the commuted layout. */
void orc_ens_true_residual(int64_t n, int s, const int32_t *row_ptr, const int32_t *col_idx,
                           const double *values, const double *b, const double *x, double *rel) {
  double *ax = malloc(sizeof(double) * (size_t)(n * s));
  orc_ens_spmv(n, s, row_ptr, col_idx, values, x, ax);
  for (int e = 0; e < s; ++e) {
    double rr = 0.0, bb = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double d = b[i * s + e] - ax[i * s + e];
      rr += d * d;
      bb += b[i * s + e] * b[i * s + e];
    }
    rel[e] = bb > 0.0 ? sqrt(rr) / sqrt(bb) : sqrt(rr);
  }
  free(ax);
}

/* ------------------------------------------------------------------------ */
/* Dense brute force for tiny meshes                                         */
/* ------------------------------------------------------------------------ */

void orc_crs_to_dense(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                      const double *values, double *dense) {
  for (int64_t i = 0; i < n * n; ++i) dense[i] = 0.0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) dense[i * n + col_idx[k]] = values[k];
}

/* Cholesky A = L L^T of a dense SPD matrix (overwritten by L in its lower
 * triangle), then forward and back substitution.  Returns 1 if a pivot is
 * not positive (A is not SPD), 0 on success.                               */
int orc_cholesky_solve(int64_t n, double *A, const double *b, double *x) {
  for (int64_t j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int64_t k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0.0)) return 1;
    double ljj = sqrt(d);
    A[j * n + j] = ljj;
    for (int64_t i = j + 1; i < n; ++i) {
      double v = A[i * n + j];
      for (int64_t k = 0; k < j; ++k) v -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = v / ljj;
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    double v = b[i];
    for (int64_t k = 0; k < i; ++k) v -= A[i * n + k] * x[k];
    x[i] = v / A[i * n + i];
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    double v = x[i];
    for (int64_t k = i + 1; k < n; ++k) v -= A[k * n + i] * x[k];
    x[i] = v / A[i * n + i];
  }
  return 0;
}

/* ------------------------------------------------------------ multigrid
 *
 * V-cycle preconditioner (Sec. 3.5, Alg. vcycle) on the nested Q1 meshes
 * N, N/2, N/4, ... (coarsened while the element count per axis is even and
 * above 4).  Each level's operator is the Q1 matrix assembled on that mesh
 * with the same KL coefficient; prolongation P is trilinear interpolation
 * from the coarse nodes (the coarse Q1 basis written in the fine one) and
 * restriction is its transpose, both restricted to interior nodes so the
 * Dirichlet identity rows stay untouched.  Smoothers are order-2 Chebyshev
 * polynomials in D^-1 A on [lmax/4, lmax], lmax the Gershgorin bound
 * max_i sum_j |a_ij| / a_ii; the coarsest level is solved exactly (dense
 * Cholesky of its interior block; boundary rows are identities).  The
 * ensemble preconditioner applies each sample's own hierarchy
 * (M_c = sum_i M_i (x) e_i e_i^T).                                        */

#define ORC_MG_MAX_LEVELS 16
#define ORC_MG_RATIO 4.0

int orc_mg_levels(int N, int32_t *Ns) {
  int L = 0;
  Ns[L++] = N;
  while (L < ORC_MG_MAX_LEVELS && Ns[L - 1] % 2 == 0 && Ns[L - 1] > 4) {
    Ns[L] = Ns[L - 1] / 2;
    ++L;
  }
  return L;
}

/* Coarse neighbours of fine index i along one axis with their
 * interpolation weights: an even i sits on coarse node i/2, an odd i
 * halfway between (i-1)/2 and (i+1)/2. */
static int axis_parents(int i, int *I, double *w) {
  if (i % 2 == 0) {
    I[0] = i / 2; w[0] = 1.0;
    return 1;
  }
  I[0] = (i - 1) / 2; w[0] = 0.5;
  I[1] = (i + 1) / 2; w[1] = 0.5;
  return 2;
}

/* xf += P xc on the interior nodes of the fine mesh (2 Nc elements per
 * axis); coarse boundary nodes contribute nothing. */
void orc_mg_prolong_add(int Nc, const double *xc, double *xf) {
  const int Nf = 2 * Nc;
  for (int k = 1; k < Nf; ++k)
    for (int j = 1; j < Nf; ++j)
      for (int i = 1; i < Nf; ++i) {
        int Ii[2], Jj[2], Kk[2];
        double wi[2], wj[2], wk[2];
        const int ni = axis_parents(i, Ii, wi), nj = axis_parents(j, Jj, wj), nk = axis_parents(k, Kk, wk);
        double v = 0.0;
        for (int c = 0; c < nk; ++c)
          for (int b = 0; b < nj; ++b)
            for (int a = 0; a < ni; ++a) {
              const int I = Ii[a], J = Jj[b], K = Kk[c];
              if (I == 0 || J == 0 || K == 0 || I == Nc || J == Nc || K == Nc) continue;
              v += wi[a] * wj[b] * wk[c] * xc[node_id(Nc, I, J, K)];
            }
        xf[node_id(Nf, i, j, k)] += v;
      }
}

/* rc = P^T rf, written as the scatter of every interior fine residual onto
 * the interior coarse nodes it interpolates from. */
void orc_mg_restrict(int Nf, const double *rf, double *rc) {
  const int Nc = Nf / 2;
  const int64_t nc = orc_num_nodes(Nc);
  for (int64_t t = 0; t < nc; ++t) rc[t] = 0.0;
  for (int k = 1; k < Nf; ++k)
    for (int j = 1; j < Nf; ++j)
      for (int i = 1; i < Nf; ++i) {
        int Ii[2], Jj[2], Kk[2];
        double wi[2], wj[2], wk[2];
        const int ni = axis_parents(i, Ii, wi), nj = axis_parents(j, Jj, wj), nk = axis_parents(k, Kk, wk);
        const double r = rf[node_id(Nf, i, j, k)];
        for (int c = 0; c < nk; ++c)
          for (int b = 0; b < nj; ++b)
            for (int a = 0; a < ni; ++a) {
              const int I = Ii[a], J = Jj[b], K = Kk[c];
              if (I == 0 || J == 0 || K == 0 || I == Nc || J == Nc || K == Nc) continue;
              rc[node_id(Nc, I, J, K)] += wi[a] * wj[b] * wk[c] * r;
            }
      }
}

double orc_gershgorin(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *values) {
  double m = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0, d = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      s += fabs(values[k]);
      if (col_idx[k] == i) d = values[k];
    }
    const double q = s / d;
    if (q > m) m = q;
  }
  return m;
}

/* Order-2 Chebyshev smoother for A x = b preconditioned by D^-1 on the
 * interval [lmax/4, lmax] (the three-term Chebyshev iteration):
 *   theta = (hi + lo)/2, delta = (hi - lo)/2, sigma = theta/delta;
 *   d = D^-1 (b - A x) / theta; x += d;
 *   rho0 = 1/sigma, rho1 = 1/(2 sigma - rho0);
 *   d = rho1 rho0 d + (2 rho1/delta) D^-1 (b - A x); x += d.
 * x_is_zero skips the first product.  r, d, ax: scratch [n].  */
void orc_mg_cheb2(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *values,
                  double lmax, const double *b, double *x, int x_is_zero, double *r, double *d, double *ax) {
  const double hi = lmax, lo = lmax / ORC_MG_RATIO;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  if (x_is_zero) {
    for (int64_t i = 0; i < n; ++i) r[i] = b[i];
  } else {
    orc_spmv(n, row_ptr, col_idx, values, x, ax);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - ax[i];
  }
  for (int64_t i = 0; i < n; ++i) {
    double dg = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
      if (col_idx[k] == i) dg = values[k];
    d[i] = (r[i] / dg) / theta;
    x[i] = x_is_zero ? d[i] : x[i] + d[i];
  }
  const double rho0 = 1.0 / sigma, rho1 = 1.0 / (2.0 * sigma - rho0);
  orc_spmv(n, row_ptr, col_idx, values, x, ax);
  for (int64_t i = 0; i < n; ++i) {
    double dg = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
      if (col_idx[k] == i) dg = values[k];
    d[i] = rho1 * rho0 * d[i] + (2.0 * rho1 / delta) * ((b[i] - ax[i]) / dg);
    x[i] += d[i];
  }
}

typedef struct {
  int N;
  int64_t n, nnz;
  int32_t *rp, *ci;
  double *v, lmax;
  double *b, *x, *r, *d, *ax;
  int64_t m;        /* coarsest level: interior unknowns */
  int64_t *imap;    /* coarsest level: interior node ids */
  double *chol;     /* coarsest level: Cholesky factor (lu: LU factors) of the interior block */
  int lu;
} orc_level;

static void free_levels(orc_level *lv, int L) {
  for (int k = 0; k < L; ++k) {
    free(lv[k].rp); free(lv[k].ci); free(lv[k].v);
    free(lv[k].b); free(lv[k].x); free(lv[k].r); free(lv[k].d); free(lv[k].ax);
    free(lv[k].imap); free(lv[k].chol);
  }
}

static int chol_factor(int64_t m, double *A) {
  for (int64_t j = 0; j < m; ++j) {
    double dd = A[j * m + j];
    for (int64_t k = 0; k < j; ++k) dd -= A[j * m + k] * A[j * m + k];
    if (!(dd > 0.0)) return 1;
    const double ljj = sqrt(dd);
    A[j * m + j] = ljj;
    for (int64_t i = j + 1; i < m; ++i) {
      double v = A[i * m + j];
      for (int64_t k = 0; k < j; ++k) v -= A[i * m + k] * A[j * m + k];
      A[i * m + j] = v / ljj;
    }
  }
  return 0;
}

static void chol_solve(int64_t m, const double *Lf, const double *b, double *x) {
  for (int64_t i = 0; i < m; ++i) {
    double v = b[i];
    for (int64_t k = 0; k < i; ++k) v -= Lf[i * m + k] * x[k];
    x[i] = v / Lf[i * m + i];
  }
  for (int64_t i = m - 1; i >= 0; --i) {
    double v = x[i];
    for (int64_t k = i + 1; k < m; ++k) v -= Lf[k * m + i] * x[k];
    x[i] = v / Lf[i * m + i];
  }
}

int orc_nl_assemble_scalar(int N, const int32_t *row_ptr, const int32_t *col_idx, const double *acoef,
                           double fconst, double alpha, const double *vel, double beta, const double *u,
                           double *F, double *values, double *load);

/* Doolittle LU of a dense m x m matrix in place, without pivoting (unit
 * lower factor below the diagonal, upper factor on and above it).  Used for
 * matrices whose symmetric part is positive definite, whose pivots are then
 * all positive; a pivot that is not is reported. */
static int lu_factor(int64_t m, double *A) {
  for (int64_t k = 0; k < m; ++k) {
    const double p = A[k * m + k];
    if (!(p > 0.0)) return 1;
    for (int64_t i = k + 1; i < m; ++i) {
      const double l = A[i * m + k] / p;
      A[i * m + k] = l;
      for (int64_t j = k + 1; j < m; ++j) A[i * m + j] -= l * A[k * m + j];
    }
  }
  return 0;
}

static void lu_solve(int64_t m, const double *F, const double *b, double *x) {
  for (int64_t i = 0; i < m; ++i) {
    double v = b[i];
    for (int64_t k = 0; k < i; ++k) v -= F[i * m + k] * x[k];
    x[i] = v;
  }
  for (int64_t i = m - 1; i >= 0; --i) {
    double v = x[i];
    for (int64_t k = i + 1; k < m; ++k) v -= F[i * m + k] * x[k];
    x[i] = v / F[i * m + i];
  }
}

/* Galerkin coarse operator of Alg. vcycle: A^{k+1} = R^k A^k P^k with
 * R = P^T, P the trilinear interpolation of orc_mg_prolong_add (interior
 * coarse nodes onto interior fine nodes).  Written out by its definition,
 *   (P^T A P)_{IJ} = sum over fine i, j of P_{iI} A_{ij} P_{jJ},
 * one coarse row I at a time: for every interior fine child i of I (the
 * fine nodes whose interpolation uses I), every stored entry A_ij of fine
 * row i with j interior, and every interior coarse parent J of j, the term
 * P_{iI} A_{ij} P_{jJ} is added to entry (I, J).  Boundary coarse rows are
 * identity rows and boundary columns of interior rows stored zeros (the
 * Dirichlet treatment of the assembled levels; P has no boundary columns, so
 * P^T A P has no boundary entries).  Af: the fine level (Nf = 2 Nc elements
 * per axis) in the layout of orc_graph; vc: the coarse level's values on
 * orc_graph(Nc).  Returns ORC_E_ARG if a term falls outside the coarse
 * 27-point pattern (it cannot for nested Q1 meshes). */
int orc_mg_galerkin(int Nc, const int32_t *rpf, const int32_t *cif, const double *vf, const int32_t *rpc,
                    const int32_t *cic, double *vc) {
  const int Nf = 2 * Nc;
  const int64_t nc = orc_num_nodes(Nc);
  for (int64_t q = 0; q < rpc[nc]; ++q) vc[q] = 0.0;
  for (int K = 0; K <= Nc; ++K)
    for (int J = 0; J <= Nc; ++J)
      for (int I = 0; I <= Nc; ++I) {
        const int64_t row = node_id(Nc, I, J, K);
        if (is_boundary_node(Nc, row)) {
          for (int64_t q = rpc[row]; q < rpc[row + 1]; ++q)
            if (cic[q] == row) vc[q] = 1.0;
          continue;
        }
        /* children of (I,J,K): fine nodes 2I-1..2I+1 per axis */
        for (int ck = 2 * K - 1; ck <= 2 * K + 1; ++ck)
          for (int cj = 2 * J - 1; cj <= 2 * J + 1; ++cj)
            for (int cii = 2 * I - 1; cii <= 2 * I + 1; ++cii) {
              const int64_t i = node_id(Nf, cii, cj, ck);
              if (is_boundary_node(Nf, i)) continue;
              int Ai[2], Aj[2], Ak[2];
              double wi[2], wj[2], wk[2];
              const int na = axis_parents(cii, Ai, wi), nb = axis_parents(cj, Aj, wj);
              const int nc3 = axis_parents(ck, Ak, wk);
              double pI = 0.0; /* P_{iI} */
              for (int c = 0; c < nc3; ++c)
                for (int b = 0; b < nb; ++b)
                  for (int a = 0; a < na; ++a)
                    if (Ai[a] == I && Aj[b] == J && Ak[c] == K) pI = wi[a] * wj[b] * wk[c];
              for (int64_t q = rpf[i]; q < rpf[i + 1]; ++q) {
                const int64_t j = cif[q];
                if (is_boundary_node(Nf, j)) continue;
                const int fx = (int)(j % (Nf + 1)), fy = (int)((j / (Nf + 1)) % (Nf + 1)),
                          fz = (int)(j / ((int64_t)(Nf + 1) * (Nf + 1)));
                int Bi[2], Bj[2], Bk[2];
                double ui[2], uj[2], uk[2];
                const int ma = axis_parents(fx, Bi, ui), mb = axis_parents(fy, Bj, uj), mc = axis_parents(fz, Bk, uk);
                for (int c = 0; c < mc; ++c)
                  for (int b = 0; b < mb; ++b)
                    for (int a = 0; a < ma; ++a) {
                      const int64_t col = node_id(Nc, Bi[a], Bj[b], Bk[c]);
                      if (is_boundary_node(Nc, col)) continue;
                      /* an interior row holds the full 3x3x3 block of
                       * neighbours in ascending node order */
                      const int dx = Bi[a] - I, dy = Bj[b] - J, dz = Bk[c] - K;
                      if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1) return ORC_E_ARG;
                      const int64_t slot = rpc[row] + (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                      if (rpc[row + 1] - rpc[row] != 27 || cic[slot] != col) return ORC_E_ARG;
                      vc[slot] += pI * vf[q] * (ui[a] * uj[b] * uk[c]);
                    }
              }
            }
      }
  return ORC_OK;
}

/* Levels for one sample: matrices assembled on every mesh of the hierarchy
 * with the sample's KL coefficient (galerkin = 0), or, with galerkin = 1,
 * the fine matrix assembled and every coarser one the Galerkin product
 * P^T A P of the level above; level 0's load vector into b0 (nullable).
 * adv = 0: the diffusion matrix (Alg. assembly).  adv = 1: the linear part
 * D + alpha C of the nonlinear Jacobian (Eq. fenl_lin_sys with beta = 0,
 * i.e. the Jacobian at u = 0 of a problem without reaction) rediscretized on
 * every mesh; its coarsest interior block is factored by LU: on interior
 * nodes C is skew-symmetric (the basis functions of interior nodes vanish on
 * the boundary and v is constant), so the block's symmetric part is that of
 * the diffusion block and no pivoting is needed. */
static int build_levels(int N, int M, double L, double kappa0, double sigma, double fconst, const double *xi,
                        int adv, double alpha, const double *vel, int galerkin, orc_level *lv, int *nlev,
                        double *b0) {
  int32_t Ns[ORC_MG_MAX_LEVELS];
  const int nl = orc_mg_levels(N, Ns);
  memset(lv, 0, sizeof(orc_level) * (size_t)nl);
  *nlev = nl;
  for (int k = 0; k < nl; ++k) {
    orc_level *l = &lv[k];
    l->N = Ns[k];
    l->n = orc_num_nodes(l->N);
    l->nnz = orc_graph_nnz(l->N);
    const int64_t ne = orc_num_elems(l->N);
    l->rp = malloc(sizeof(int32_t) * (size_t)(l->n + 1));
    l->ci = malloc(sizeof(int32_t) * (size_t)l->nnz);
    l->v = malloc(sizeof(double) * (size_t)l->nnz);
    l->b = calloc((size_t)l->n, sizeof(double));
    l->x = calloc((size_t)l->n, sizeof(double));
    l->r = calloc((size_t)l->n, sizeof(double));
    l->d = calloc((size_t)l->n, sizeof(double));
    l->ax = calloc((size_t)l->n, sizeof(double));
    double *ac = malloc(sizeof(double) * 8 * (size_t)ne);
    double *load = malloc(sizeof(double) * (size_t)l->n);
    if (!l->rp || !l->ci || !l->v || !l->b || !l->x || !l->r || !l->d || !l->ax || !ac || !load) {
      free(ac); free(load);
      return ORC_E_NOMEM;
    }
    orc_graph(l->N, l->rp, l->ci);
    orc_kl_coef_qp(l->N, M, L, kappa0, sigma, xi, ac);
    if (galerkin && k > 0) {
      const orc_level *f = &lv[k - 1];
      if (orc_mg_galerkin(l->N, f->rp, f->ci, f->v, l->rp, l->ci, l->v) != ORC_OK) {
        free(ac); free(load);
        return ORC_E_ARG;
      }
    } else if (adv) {
      /* r and x are zero here: x serves as u = 0, r receives F(0) = -load */
      orc_nl_assemble_scalar(l->N, l->rp, l->ci, ac, fconst, alpha, vel, 0.0, l->x, l->r, l->v, load);
      for (int64_t t = 0; t < l->n; ++t) l->r[t] = 0.0;
    } else {
      orc_assemble_scalar(l->N, l->rp, l->ci, ac, 0, fconst, 1, l->v, load);
    }
    if (k == 0 && b0) memcpy(b0, load, sizeof(double) * (size_t)l->n);
    free(ac); free(load);
    l->lmax = orc_gershgorin(l->n, l->rp, l->ci, l->v);
  }
  orc_level *c = &lv[nl - 1];
  c->imap = malloc(sizeof(int64_t) * (size_t)c->n);
  if (!c->imap) return ORC_E_NOMEM;
  c->m = 0;
  for (int64_t t = 0; t < c->n; ++t)
    if (!is_boundary_node(c->N, t)) c->imap[c->m++] = t;
  c->chol = calloc((size_t)(c->m * c->m) + 1, sizeof(double));
  if (!c->chol) return ORC_E_NOMEM;
  for (int64_t a = 0; a < c->m; ++a) {
    const int64_t row = c->imap[a];
    for (int64_t k = c->rp[row]; k < c->rp[row + 1]; ++k)
      for (int64_t bcol = 0; bcol < c->m; ++bcol)
        if (c->imap[bcol] == c->ci[k]) c->chol[a * c->m + bcol] = c->v[k];
  }
  c->lu = adv;
  if (c->m > 0 && (adv ? lu_factor(c->m, c->chol) : chol_factor(c->m, c->chol))) return ORC_E_ARG;
  return ORC_OK;
}

/* x = V-cycle(b) on level k (x overwritten), in the order of Alg. vcycle. */
static void vcycle(orc_level *lv, int k, int nl, const double *b, double *x) {
  orc_level *l = &lv[k];
  if (k == nl - 1) {
    for (int64_t t = 0; t < l->n; ++t) x[t] = b[t];  /* identity rows */
    if (l->m > 0) {
      double *bi = l->r, *xi = l->d;
      for (int64_t a = 0; a < l->m; ++a) bi[a] = b[l->imap[a]];
      if (l->lu) lu_solve(l->m, l->chol, bi, xi);
      else chol_solve(l->m, l->chol, bi, xi);
      for (int64_t a = 0; a < l->m; ++a) x[l->imap[a]] = xi[a];
    }
    return;
  }
  orc_mg_cheb2(l->n, l->rp, l->ci, l->v, l->lmax, b, x, 1, l->r, l->d, l->ax);
  orc_spmv(l->n, l->rp, l->ci, l->v, x, l->ax);
  for (int64_t t = 0; t < l->n; ++t) l->r[t] = b[t] - l->ax[t];
  orc_level *c = &lv[k + 1];
  orc_mg_restrict(l->N, l->r, c->b);
  vcycle(lv, k + 1, nl, c->b, c->x);
  orc_mg_prolong_add(c->N, c->x, x);
  orc_mg_cheb2(l->n, l->rp, l->ci, l->v, l->lmax, b, x, 0, l->r, l->d, l->ax);
}

/* z = M r for one sample's hierarchy (for building M in tests). */
int orc_mg_apply(int N, int M, double L, double kappa0, double sigma, double fconst, const double *xi,
                 const double *r, double *z, int galerkin) {
  orc_level lv[ORC_MG_MAX_LEVELS];
  int nl = 0;
  int rc = build_levels(N, M, L, kappa0, sigma, fconst, xi, 0, 0.0, NULL, galerkin, lv, &nl, NULL);
  if (rc == ORC_OK) vcycle(lv, 0, nl, r, z);
  free_levels(lv, nl);
  return rc;
}

/* z = M r for the V-cycle of one sample's advection-diffusion operator
 * D + alpha C (every level rediscretized, as build_levels with adv = 1). */
int orc_mg_apply_adv(int N, int M, double L, double kappa0, double sigma, double fconst, double alpha,
                     const double *vel, const double *xi, const double *r, double *z) {
  if (!vel) return ORC_E_ARG;
  orc_level lv[ORC_MG_MAX_LEVELS];
  int nl = 0;
  int rc = build_levels(N, M, L, kappa0, sigma, fconst, xi, 1, alpha, vel, 0, lv, &nl, NULL);
  if (rc == ORC_OK) vcycle(lv, 0, nl, r, z);
  free_levels(lv, nl);
  return rc;
}

/* Multigrid-preconditioned CG for one sample: textbook PCG with z = M r,
 * the same stopping rule and failure handling as orc_pcg.  x in: x0. */
int orc_mg_pcg(int N, int M, double L, double kappa0, double sigma, double fconst, const double *xi, double *x,
               double rtol, int max_iter, int fixed_iters, int32_t *iters_out, double *rel_res_out,
               int32_t *status_out, double *lmax_out, int galerkin) {
  orc_level lv[ORC_MG_MAX_LEVELS];
  int nl = 0;
  const int64_t n = orc_num_nodes(N);
  double *b = malloc(sizeof(double) * (size_t)n);
  double *r = malloc(sizeof(double) * (size_t)n), *z = malloc(sizeof(double) * (size_t)n);
  double *p = malloc(sizeof(double) * (size_t)n), *q = malloc(sizeof(double) * (size_t)n);
  if (!b || !r || !z || !p || !q) return ORC_E_NOMEM;
  int rc = build_levels(N, M, L, kappa0, sigma, fconst, xi, 0, 0.0, NULL, galerkin, lv, &nl, b);
  if (rc != ORC_OK) { free_levels(lv, nl); free(b); free(r); free(z); free(p); free(q); return rc; }
  if (lmax_out)
    for (int k = 0; k < nl; ++k) lmax_out[k] = lv[k].lmax;
  const int32_t *rp = lv[0].rp, *ci = lv[0].ci;
  const double *vals = lv[0].v;
  int status = ORC_CONVERGED, iters = 0;
  const double nb = sqrt(dot(n, b, b));
  orc_spmv(n, rp, ci, vals, x, q);
  for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
  int limit = fixed_iters >= 0 ? fixed_iters : max_iter;
  const int test = fixed_iters < 0;
  if (nb == 0.0) {
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    limit = 0;
  } else if (test && sqrt(dot(n, r, r)) <= rtol * nb) {
    limit = 0;
  } else {
    vcycle(lv, 0, nl, r, z);
    for (int64_t i = 0; i < n; ++i) p[i] = z[i];
    double rho = dot(n, r, z);
    status = ORC_MAXITER;
    for (int k = 1; k <= limit; ++k) {
      orc_spmv(n, rp, ci, vals, p, q);
      const double eta = dot(n, p, q);
      if (!isfinite(eta) || !isfinite(rho)) { status = ORC_NONFINITE; break; }
      if (!(eta > 0.0)) { status = ORC_BREAKDOWN; break; }
      const double alpha = rho / eta;
      for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
      iters = k;
      const double rr = dot(n, r, r);
      if (!isfinite(rr)) { status = ORC_NONFINITE; break; }
      if (test && sqrt(rr) <= rtol * nb) { status = ORC_CONVERGED; break; }
      if (!test && k == limit) { status = ORC_CONVERGED; break; }
      vcycle(lv, 0, nl, r, z);
      const double rho_new = dot(n, r, z);
      const double beta = rho_new / rho;
      for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
      rho = rho_new;
    }
    if (!test && limit == 0) status = ORC_CONVERGED;
  }
  orc_spmv(n, rp, ci, vals, x, q);
  for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
  *iters_out = iters;
  *rel_res_out = nb > 0.0 ? sqrt(dot(n, r, r)) / nb : 0.0;
  *status_out = status;
  free_levels(lv, nl);
  free(b); free(r); free(z); free(p); free(q);
  return ORC_OK;
}

/* The ensemble of orc_mg_pcg, one sample per thread: xi [s][M], x [n][s]
 * (commuted layout, in: x0), fixed_iters [s] nullable, lmax [s][16]
 * nullable (each level's Chebyshev bound). */
int orc_ens_mg_pcg(int N, int M, double L, double kappa0, double sigma, double fconst, int s, const double *xi,
                   double *x, double rtol, int max_iter, const int32_t *fixed_iters, int32_t *iters,
                   double *rel_res, int32_t *status, double *lmax, int galerkin) {
  const int64_t n = orc_num_nodes(N);
  int rc = ORC_OK;
  #pragma omp parallel for schedule(dynamic, 1)
  for (int e = 0; e < s; ++e) {
    double *xe = malloc(sizeof(double) * (size_t)n);
    if (!xe) { rc = ORC_E_NOMEM; continue; }
    for (int64_t i = 0; i < n; ++i) xe[i] = x[i * s + e];
    int r = orc_mg_pcg(N, M, L, kappa0, sigma, fconst, xi + (int64_t)e * M, xe, rtol, max_iter,
                       fixed_iters ? fixed_iters[e] : -1, &iters[e], &rel_res[e], &status[e],
                       lmax ? lmax + (int64_t)e * ORC_MG_MAX_LEVELS : NULL, galerkin);
    if (r) rc = r;
    for (int64_t i = 0; i < n; ++i) x[i * s + e] = xe[i];
    free(xe);
  }
  return rc;
}

/* ------------------------------------------------------------------------ */
/* The nonlinear problem (Sec. 4, Eq. diffusion_sys):                        */
/*   -div(kappa grad u) + alpha v.grad u + beta u^2 = f,  u = 0 on the       */
/* boundary (the source f = fconst and the boundary condition as in the      */
/* linear case; v a constant velocity vector).  Galerkin Q1 with the same    */
/* 2x2x2 Gauss rule.  For interior node i                                    */
/*   F_i(u) = sum_e sum_q w_q [ kappa grad N_a . grad u_h                    */
/*            + alpha N_a (v . grad u_h) + beta N_a u_h^2 - f N_a ]          */
/* with u_h = sum_b N_b u_b over the element's 8 nodes (boundary nodes       */
/* included with their values), and the Jacobian A = dF/du of Eq.            */
/* fenl_lin_sys:                                                             */
/*   A_ij = sum_e sum_q w_q [ kappa grad N_a . grad N_b                      */
/*            + alpha N_a (v . grad N_b) + 2 beta u_h N_a N_b ].             */
/* Boundary rows: F_i = u_i and an identity row; the boundary columns of     */
/* interior rows are stored zeros (Dirichlet elimination, as for the linear  */
/* matrix).  `load` (nullable) receives the source part sum w_q f N_a of     */
/* interior rows (zero on the boundary): F(0) = -load.                        */
/* ------------------------------------------------------------------------ */

int orc_nl_assemble_scalar(int N, const int32_t *row_ptr, const int32_t *col_idx, const double *acoef,
                           double fconst, double alpha, const double *vel, double beta, const double *u,
                           double *F, double *values, double *load) {
  if (N < 1 || !row_ptr || !col_idx || !acoef || !vel || !u || !F) return ORC_E_ARG;
  const double h = 1.0 / (double)N;
  const double wq = h * h * h / 8.0;
  int64_t n = orc_num_nodes(N), nnz = row_ptr[n], ne = orc_num_elems(N);
  for (int64_t i = 0; i < n; ++i) F[i] = 0.0;
  if (values)
    for (int64_t k = 0; k < nnz; ++k) values[k] = 0.0;
  if (load)
    for (int64_t i = 0; i < n; ++i) load[i] = 0.0;
  double Nq[8][8], G[8][8][3];
  for (int q = 0; q < 8; ++q) {
    double s = gauss01(q & 1), t = gauss01((q >> 1) & 1), w = gauss01((q >> 2) & 1);
    for (int a = 0; a < 8; ++a) {
      int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
      Nq[q][a] = lfun(ax, s) * lfun(ay, t) * lfun(az, w);
      G[q][a][0] = dlfun(ax) * lfun(ay, t) * lfun(az, w) / h;
      G[q][a][1] = lfun(ax, s) * dlfun(ay) * lfun(az, w) / h;
      G[q][a][2] = lfun(ax, s) * lfun(ay, t) * dlfun(az) / h;
    }
  }
  for (int64_t e = 0; e < ne; ++e) {
    double ue[8], Fe[8], Ae[8][8], Le[8];
    for (int a = 0; a < 8; ++a) ue[a] = u[elem_node(N, e, a)];
    for (int a = 0; a < 8; ++a) {
      Fe[a] = 0.0;
      Le[a] = 0.0;
      for (int b = 0; b < 8; ++b) Ae[a][b] = 0.0;
    }
    for (int q = 0; q < 8; ++q) {
      const double kap = acoef[e * 8 + q];
      double uq = 0.0, gu[3] = {0.0, 0.0, 0.0};
      for (int b = 0; b < 8; ++b) {
        uq += Nq[q][b] * ue[b];
        for (int d = 0; d < 3; ++d) gu[d] += G[q][b][d] * ue[b];
      }
      const double vgu = vel[0] * gu[0] + vel[1] * gu[1] + vel[2] * gu[2];
      for (int a = 0; a < 8; ++a) {
        const double diff = G[q][a][0] * gu[0] + G[q][a][1] * gu[1] + G[q][a][2] * gu[2];
        Fe[a] += wq * (kap * diff + alpha * Nq[q][a] * vgu + beta * Nq[q][a] * uq * uq - fconst * Nq[q][a]);
        Le[a] += wq * fconst * Nq[q][a];
        for (int b = 0; b < 8; ++b) {
          const double gg = G[q][a][0] * G[q][b][0] + G[q][a][1] * G[q][b][1] + G[q][a][2] * G[q][b][2];
          const double vgb = vel[0] * G[q][b][0] + vel[1] * G[q][b][1] + vel[2] * G[q][b][2];
          Ae[a][b] += wq * (kap * gg + alpha * Nq[q][a] * vgb + 2.0 * beta * uq * Nq[q][a] * Nq[q][b]);
        }
      }
    }
    for (int a = 0; a < 8; ++a) {
      int64_t I = elem_node(N, e, a);
      F[I] += Fe[a];
      if (load) load[I] += Le[a];
      if (values)
        for (int b = 0; b < 8; ++b) values[find_slot(row_ptr, col_idx, I, elem_node(N, e, b))] += Ae[a][b];
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    const int bi = is_boundary_node(N, i);
    if (bi) {
      F[i] = u[i];
      if (load) load[i] = 0.0;
    }
    if (values)
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        if (bi) values[k] = (col_idx[k] == i) ? 1.0 : 0.0;
        else if (is_boundary_node(N, col_idx[k])) values[k] = 0.0;
      }
  }
  return ORC_OK;
}

/* The ensemble of orc_nl_assemble_scalar in the commuted layout: u, F, load
 * [n][s]; values [nnz][s] (nullable); vel[3]. */
int orc_ens_nl_assemble(int N, const int32_t *row_ptr, const int32_t *col_idx, int M, double L, double kappa0,
                        double sigma, double fconst, double alpha, const double *vel, double beta, int s,
                        const double *xi, const double *u, double *F, double *values, double *load) {
  if (N < 1 || s < 1) return ORC_E_ARG;
  int64_t n = orc_num_nodes(N), nnz = row_ptr[n], ne = orc_num_elems(N);
  int rc = ORC_OK;
  #pragma omp parallel for schedule(dynamic, 1)
  for (int e = 0; e < s; ++e) {
    double *ac = malloc(sizeof(double) * 8 * (size_t)ne);
    double *ue = malloc(sizeof(double) * (size_t)n), *fe = malloc(sizeof(double) * (size_t)n);
    double *le = malloc(sizeof(double) * (size_t)n);
    double *v = values ? malloc(sizeof(double) * (size_t)nnz) : NULL;
    if (!ac || !ue || !fe || !le || (values && !v)) {
      rc = ORC_E_NOMEM;
      free(ac); free(ue); free(fe); free(le); free(v);
      continue;
    }
    for (int64_t i = 0; i < n; ++i) ue[i] = u[i * s + e];
    orc_kl_coef_qp(N, M, L, kappa0, sigma, xi + (int64_t)e * M, ac);
    orc_nl_assemble_scalar(N, row_ptr, col_idx, ac, fconst, alpha, vel, beta, ue, fe, v, le);
    for (int64_t i = 0; i < n; ++i) F[i * s + e] = fe[i];
    if (load)
      for (int64_t i = 0; i < n; ++i) load[i * s + e] = le[i];
    if (values)
      for (int64_t k = 0; k < nnz; ++k) values[k * s + e] = v[k];
    free(ac); free(ue); free(fe); free(le); free(v);
  }
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Restarted GMRES(m) with right preconditioning, one sample, for the        */
/* nonsymmetric Newton systems (the Krylov solve of Eq. fenl_lin_sys when    */
/* alpha != 0).  Textbook form: Arnoldi with modified Gram-Schmidt on        */
/* A M, Givens rotations on the Hessenberg matrix, the residual estimate     */
/* |g_{j+1}| tested against rtol ||b|| after every step, at a cycle's end    */
/* y = R^{-1} g and x += M (V y), then the true residual r = b - A x.  The   */
/* solve has converged when the true residual meets the tolerance; a cycle   */
/* whose estimate met it but whose true residual does not is followed by     */
/* another.  M: prec 0 Jacobi (the diagonal of A), 1 the multigrid V-cycle   */
/* of the sample's diffusion operator (the alpha = beta = 0 matrix), 2 the    */
/* V-cycle of its advection-diffusion operator D + alpha C (beta = 0) with    */
/* every level rediscretized (alpha and vel used only by 2).                  */
/* fixed_iters >= 0: exactly that many Arnoldi steps in one cycle (needs     */
/* fixed_iters <= restart), no residual test.  Iterations count Arnoldi      */
/* steps (products with A) over all cycles.                                  */
/* ------------------------------------------------------------------------ */

#define ORC_GM_MAX_RESTART 64

typedef struct {
  int kind;             /* 0 Jacobi, 1 or 2 multigrid */
  const double *dinv;   /* Jacobi */
  orc_level *lv;        /* multigrid levels */
  int nl;
} orc_prec;

static void prec_apply(const orc_prec *P, int64_t n, const double *r, double *z) {
  if (P->kind == 0) {
    for (int64_t i = 0; i < n; ++i) z[i] = P->dinv[i] * r[i];
  } else {
    vcycle(P->lv, 0, P->nl, r, z);
  }
}

static int gmres_core(int64_t n, const int32_t *rp, const int32_t *ci, const double *vals, const double *b,
                      double *x, const orc_prec *P, double rtol, int restart, int max_iter, int fixed_iters,
                      int32_t *iters_out, double *rel_res_out, int32_t *status_out) {
  if (restart < 1 || restart > ORC_GM_MAX_RESTART) return ORC_E_ARG;
  if (fixed_iters > restart) return ORC_E_ARG;
  const int m = restart;
  double *V = malloc(sizeof(double) * (size_t)n * (size_t)(m + 1));
  double *w = malloc(sizeof(double) * (size_t)n), *z = malloc(sizeof(double) * (size_t)n);
  double *r = malloc(sizeof(double) * (size_t)n), *t = malloc(sizeof(double) * (size_t)n);
  double H[ORC_GM_MAX_RESTART + 1][ORC_GM_MAX_RESTART], cs[ORC_GM_MAX_RESTART], sn[ORC_GM_MAX_RESTART];
  double g[ORC_GM_MAX_RESTART + 1], y[ORC_GM_MAX_RESTART];
  if (!V || !w || !z || !r || !t) {
    free(V); free(w); free(z); free(r); free(t);
    return ORC_E_NOMEM;
  }
  const int test = fixed_iters < 0;
  const int limit = test ? max_iter : fixed_iters;
  const double nb = sqrt(dot(n, b, b));
  const double tol = rtol * nb;
  int total = 0, status = ORC_MAXITER;
  double beta = 0.0;
  if (nb == 0.0) {
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    status = ORC_CONVERGED;
  } else {
    orc_spmv(n, rp, ci, vals, x, t);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - t[i];
    beta = sqrt(dot(n, r, r));
    if (!isfinite(beta)) status = ORC_NONFINITE;
    else if (test && beta <= tol) status = ORC_CONVERGED;
    else if (!test && limit == 0) status = ORC_CONVERGED;
    while (status == ORC_MAXITER) {
      for (int64_t i = 0; i < n; ++i) V[i] = r[i] / beta;
      for (int i = 0; i <= m; ++i) g[i] = 0.0;
      g[0] = beta;
      int k = 0;
      for (int j = 0; j < m && total < limit; ++j) {
        double *vj = V + (size_t)j * n;
        prec_apply(P, n, vj, z);
        orc_spmv(n, rp, ci, vals, z, w);
        for (int i = 0; i <= j; ++i) {
          const double *vi = V + (size_t)i * n;
          H[i][j] = dot(n, w, vi);
          for (int64_t q = 0; q < n; ++q) w[q] -= H[i][j] * vi[q];
        }
        const double hnext = sqrt(dot(n, w, w));
        H[j + 1][j] = hnext;
        for (int i = 0; i < j; ++i) {
          const double a = H[i][j], c = H[i + 1][j];
          H[i][j] = cs[i] * a + sn[i] * c;
          H[i + 1][j] = -sn[i] * a + cs[i] * c;
        }
        const double a = H[j][j], c = H[j + 1][j];
        const double den = sqrt(a * a + c * c);
        ++total;
        k = j + 1;
        if (!isfinite(den)) { status = ORC_NONFINITE; break; }
        if (den == 0.0) { status = ORC_BREAKDOWN; break; }
        cs[j] = a / den;
        sn[j] = c / den;
        H[j][j] = den;
        H[j + 1][j] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        if (test && fabs(g[j + 1]) <= tol) break;
        if (hnext == 0.0) break; /* the Krylov space is invariant: x is exact */
        double *vn = V + (size_t)(j + 1) * n;
        for (int64_t q = 0; q < n; ++q) vn[q] = w[q] / hnext;
      }
      if (status != ORC_MAXITER) break;
      /* y = R^-1 g, x += M (V y) */
      for (int i = k - 1; i >= 0; --i) {
        double v = g[i];
        for (int l = i + 1; l < k; ++l) v -= H[i][l] * y[l];
        y[i] = v / H[i][i];
      }
      for (int64_t q = 0; q < n; ++q) t[q] = 0.0;
      for (int i = 0; i < k; ++i)
        for (int64_t q = 0; q < n; ++q) t[q] += y[i] * V[(size_t)i * n + q];
      prec_apply(P, n, t, z);
      for (int64_t q = 0; q < n; ++q) x[q] += z[q];
      orc_spmv(n, rp, ci, vals, x, t);
      for (int64_t i = 0; i < n; ++i) r[i] = b[i] - t[i];
      beta = sqrt(dot(n, r, r));
      if (!isfinite(beta)) { status = ORC_NONFINITE; break; }
      if (!test) { status = ORC_CONVERGED; break; }
      if (beta <= tol) { status = ORC_CONVERGED; break; }
      if (total >= limit || k == 0) break;
    }
  }
  *iters_out = total;
  *rel_res_out = nb > 0.0 ? beta / nb : 0.0;
  *status_out = status;
  free(V); free(w); free(z); free(r); free(t);
  return ORC_OK;
}

/* One sample's GMRES on the matrix `values` of the N^3 mesh's graph; prec 1
 * builds the multigrid levels of the sample's diffusion problem (M, L,
 * kappa0, sigma, xi). */
int orc_gmres(int N, const int32_t *rp, const int32_t *ci, const double *values, const double *b, double *x,
              int prec, int M, double L, double kappa0, double sigma, const double *xi, double alpha,
              const double *vel, double rtol, int restart, int max_iter, int fixed_iters, int32_t *iters,
              double *rel_res, int32_t *status) {
  const int64_t n = orc_num_nodes(N);
  orc_prec P;
  memset(&P, 0, sizeof(P));
  P.kind = prec;
  orc_level lv[ORC_MG_MAX_LEVELS];
  double *dinv = NULL;
  int rc = ORC_OK;
  if (prec == 0) {
    dinv = malloc(sizeof(double) * (size_t)n);
    if (!dinv) return ORC_E_NOMEM;
    for (int64_t i = 0; i < n; ++i) {
      double dg = 0.0;
      for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
        if (ci[k] == i) dg = values[k];
      dinv[i] = 1.0 / dg;
    }
    P.dinv = dinv;
  } else {
    rc = build_levels(N, M, L, kappa0, sigma, 1.0, xi, prec == 2, alpha, vel, 0, lv, &P.nl, NULL);
    P.lv = lv;
  }
  if (rc == ORC_OK)
    rc = gmres_core(n, rp, ci, values, b, x, &P, rtol, restart, max_iter, fixed_iters, iters, rel_res, status);
  if (prec != 0) free_levels(lv, P.nl);
  free(dinv);
  return rc;
}

/* GMRES for every sample of an ensemble (matrix values [nnz][s], b and x
 * [n][s], one sample per thread); fixed_iters [s] nullable. */
int orc_ens_gmres(int N, const int32_t *rp, const int32_t *ci, int s, const double *values, const double *b,
                  double *x, int prec, int M, double L, double kappa0, double sigma, const double *xi, double alpha,
                  const double *vel, double rtol, int restart, int max_iter, const int32_t *fixed_iters,
                  int32_t *iters, double *rel_res, int32_t *status) {
  const int64_t n = orc_num_nodes(N), nnz = rp[n];
  int rc = ORC_OK;
  #pragma omp parallel for schedule(dynamic, 1)
  for (int e = 0; e < s; ++e) {
    double *ve = malloc(sizeof(double) * (size_t)nnz);
    double *be = malloc(sizeof(double) * (size_t)n), *xe = malloc(sizeof(double) * (size_t)n);
    if (!ve || !be || !xe) { rc = ORC_E_NOMEM; free(ve); free(be); free(xe); continue; }
    for (int64_t k = 0; k < nnz; ++k) ve[k] = values[k * s + e];
    for (int64_t i = 0; i < n; ++i) { be[i] = b[i * s + e]; xe[i] = x[i * s + e]; }
    int r = orc_gmres(N, rp, ci, ve, be, xe, prec, M, L, kappa0, sigma, xi + (int64_t)e * M, alpha, vel, rtol,
                      restart, max_iter, fixed_iters ? fixed_iters[e] : -1, &iters[e], &rel_res[e], &status[e]);
    if (r) rc = r;
    for (int64_t i = 0; i < n; ++i) x[i * s + e] = xe[i];
    free(ve); free(be); free(xe);
  }
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Newton's method on F(u) = 0 (Sec. 4, Eq. fenl_lin_sys), one sample:       */
/*   k = 0, 1, ...: F, A at u_k; stop when ||F(u_k)|| <= rtol ||load||        */
/*   (||F(u_0)|| when the load is zero); otherwise A d = F by GMRES to the   */
/*   relative tolerance eta_k from d = 0, and u_{k+1} = u_k - d.             */
/* forcing 0: eta_k = lin_rtol.  forcing 1: the second choice of Eisenstat   */
/* and Walker (SIAM J. Sci. Comput. 17, 1996) with gamma = 0.9, exponent 2,  */
/* eta_0 = eta_max = lin_rtol: eta_k = gamma (|F_k| / |F_{k-1}|)^2, raised   */
/* to gamma eta_{k-1}^2 when that exceeds 0.1, capped at eta_max, and kept   */
/* at least 0.5 rtol ref / |F_k| (no solve tighter than the Newton test      */
/* needs).                                                                   */
/* Statuses: converged; max steps; breakdown (the linear solve broke down);  */
/* non-finite.  fnorm (nullable, max_newton + 1 entries) receives ||F(u_k)||; */
/* eta (nullable, max_newton + 1 entries) the tolerance of each Newton       */
/* system solved (0 where no system was solved).                             */
/* ------------------------------------------------------------------------ */

/* The forcing term of Newton step k >= 0 (exported for its pins):
 * k = 0 gives lin_rtol (= eta_max); later steps the Eisenstat-Walker
 * choice 2 value from |F_k| = fn, |F_{k-1}| = fprev and eta_{k-1} =
 * eta_prev, with the safeguard, the cap and the floor floor_tol. */
double orc_ew_forcing(int k, double eta_prev, double fn, double fprev, double lin_rtol, double floor_tol) {
  if (k == 0) return lin_rtol;
  const double gamma = 0.9;
  double eta = gamma * (fn / fprev) * (fn / fprev);
  const double safe = gamma * eta_prev * eta_prev;
  if (safe > 0.1 && safe > eta) eta = safe;
  if (eta > lin_rtol) eta = lin_rtol;
  if (eta < floor_tol) eta = floor_tol;
  return eta;
}

int orc_newton(int N, int M, double L, double kappa0, double sigma, double fconst, double alpha, const double *vel,
               double beta, const double *xi, double *u, int prec, double rtol, int max_newton, double lin_rtol,
               int restart, int lin_max_iter, int forcing, int32_t *newton_iters, int32_t *lin_iters,
               double *rel_res, int32_t *status, double *fnorm, double *etas) {
  const int64_t n = orc_num_nodes(N), nnz = orc_graph_nnz(N), ne = orc_num_elems(N);
  int32_t *rp = malloc(sizeof(int32_t) * (size_t)(n + 1)), *ci = malloc(sizeof(int32_t) * (size_t)nnz);
  double *ac = malloc(sizeof(double) * 8 * (size_t)ne), *vals = malloc(sizeof(double) * (size_t)nnz);
  double *F = malloc(sizeof(double) * (size_t)n), *ld = malloc(sizeof(double) * (size_t)n);
  double *d = malloc(sizeof(double) * (size_t)n), *dinv = malloc(sizeof(double) * (size_t)n);
  orc_level lv[ORC_MG_MAX_LEVELS];
  orc_prec P;
  memset(&P, 0, sizeof(P));
  int rc = ORC_OK;
  if (!rp || !ci || !ac || !vals || !F || !ld || !d || !dinv) rc = ORC_E_NOMEM;
  if (rc == ORC_OK) {
    orc_graph(N, rp, ci);
    orc_kl_coef_qp(N, M, L, kappa0, sigma, xi, ac);
    P.kind = prec;
    if (prec != 0) {
      rc = build_levels(N, M, L, kappa0, sigma, fconst, xi, prec == 2, alpha, vel, 0, lv, &P.nl, NULL);
      P.lv = lv;
    }
  }
  int st = ORC_MAXITER, k = 0, lin_total = 0;
  double ref = 0.0, fn = 0.0, fprev = 0.0, eta = lin_rtol;
  for (; rc == ORC_OK; ++k) {
    orc_nl_assemble_scalar(N, rp, ci, ac, fconst, alpha, vel, beta, u, F, vals, ld);
    fn = sqrt(dot(n, F, F));
    if (k == 0) {
      ref = sqrt(dot(n, ld, ld));
      if (ref == 0.0) ref = fn;
    }
    if (fnorm) fnorm[k] = fn;
    if (etas) etas[k] = 0.0;
    if (!isfinite(fn)) { st = ORC_NONFINITE; break; }
    if (fn <= rtol * ref) { st = ORC_CONVERGED; break; }
    if (k == max_newton) { st = ORC_MAXITER; break; }
    if (prec == 0) {
      for (int64_t i = 0; i < n; ++i) {
        double dg = 0.0;
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q)
          if (ci[q] == i) dg = vals[q];
        dinv[i] = 1.0 / dg;
      }
      P.dinv = dinv;
    }
    if (forcing == 1) eta = orc_ew_forcing(k, eta, fn, fprev, lin_rtol, 0.5 * rtol * ref / fn);
    if (etas) etas[k] = forcing == 1 ? eta : lin_rtol;
    fprev = fn;
    for (int64_t i = 0; i < n; ++i) d[i] = 0.0;
    int32_t it = 0, ls = 0;
    double lr = 0.0;
    rc = gmres_core(n, rp, ci, vals, F, d, &P, forcing == 1 ? eta : lin_rtol, restart, lin_max_iter, -1, &it, &lr,
                    &ls);
    lin_total += it;
    if (ls == ORC_NONFINITE) { st = ORC_NONFINITE; break; }
    if (ls == ORC_BREAKDOWN) { st = ORC_BREAKDOWN; break; }
    for (int64_t i = 0; i < n; ++i) u[i] -= d[i];
  }
  *newton_iters = k;
  *lin_iters = lin_total;
  *rel_res = ref > 0.0 ? fn / ref : 0.0;
  *status = st;
  if (prec != 0 && P.lv) free_levels(lv, P.nl);
  free(rp); free(ci); free(ac); free(vals); free(F); free(ld); free(d); free(dinv);
  return rc;
}

/* Newton for every sample (u [n][s] in/out, one sample per thread); fnorm
 * and etas [s][max_newton + 1] nullable. */
int orc_ens_newton(int N, int M, double L, double kappa0, double sigma, double fconst, double alpha,
                   const double *vel, double beta, int s, const double *xi, double *u, int prec, double rtol,
                   int max_newton, double lin_rtol, int restart, int lin_max_iter, int forcing,
                   int32_t *newton_iters, int32_t *lin_iters, double *rel_res, int32_t *status, double *fnorm,
                   double *etas) {
  const int64_t n = orc_num_nodes(N);
  int rc = ORC_OK;
  #pragma omp parallel for schedule(dynamic, 1)
  for (int e = 0; e < s; ++e) {
    double *ue = malloc(sizeof(double) * (size_t)n);
    if (!ue) { rc = ORC_E_NOMEM; continue; }
    for (int64_t i = 0; i < n; ++i) ue[i] = u[i * s + e];
    int r = orc_newton(N, M, L, kappa0, sigma, fconst, alpha, vel, beta, xi + (int64_t)e * M, ue, prec, rtol,
                       max_newton, lin_rtol, restart, lin_max_iter, forcing, &newton_iters[e], &lin_iters[e],
                       &rel_res[e], &status[e], fnorm ? fnorm + (int64_t)e * (max_newton + 1) : NULL,
                       etas ? etas + (int64_t)e * (max_newton + 1) : NULL);
    if (r) rc = r;
    for (int64_t i = 0; i < n; ++i) u[i * s + e] = ue[i];
    free(ue);
  }
  return rc;
}

/* Threads an OpenMP loop of the oracle may use (1 without OpenMP). */
int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int orc_version(void) { return 1; }
