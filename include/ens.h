/*
 * ens.h -- C ABI of libens, an MI355X (gfx950) implementation of embedded
 * ensemble propagation for the sampled diffusion problem
 *     -div(kappa(x,y) grad u) = f  on D = [0,1]^3,  u = 0 on the boundary,
 * discretised with trilinear (Q1) hexahedra (Phipps et al., arXiv 1511.03703,
 * Sec. 4, with alpha = beta = 0 so the system is linear, symmetric and
 * positive definite).
 *
 * s samples y_1..y_s share one CRS graph.  Following the commuted Kronecker
 * system (Sec. 2, Eq. kron_sys_commuted) every matrix value and vector entry
 * is an s-long ensemble stored contiguously:
 *     values[k*s + e]   (k = CRS entry, e = sample)     "[nnz][s]"
 *     x[i*s + e]        (i = node)                      "[n][s]"
 *     xi[e*M + m]       (KL inputs of sample e)         "[s][M]"
 *
 * Conventions for every entry point:
 *   - Pointers marked (device) are device memory the caller allocated and
 *     owns; the library never frees them and keeps no reference after the
 *     call.  Pointers marked (host) are host memory.
 *   - Device buffers holding ensembles must be 16-byte aligned.
 *   - Work is enqueued on `stream` (a hipStream_t) in stream order.  Entry
 *     points that return results on the host (ens_cg, ens_scalar_cg,
 *     ens_solve_batch) synchronise that stream before returning; the others
 *     never synchronise.
 *   - Errors are reported by the return value, never by aborting: arguments
 *     are validated on the host before any launch (ENS_E_ARG,
 *     ENS_E_UNSUPPORTED, ENS_E_RANGE); HIP failures return ENS_E_HIP.  A
 *     text description of the last error of the calling thread is available
 *     from ens_last_error().  Numerical outcomes of solves are reported per
 *     sample in ens_cg_stat.status.
 *   - Indices are int32 (4 bytes per column entry, as in the paper's byte
 *     model, Sec. 4); all value offsets are computed in 64-bit.
 *   - Supported ensemble sizes s: 4, 8, 16, 32 (compile-time instantiations,
 *     the role explicit template instantiation plays in Sec. 3.6).
 */
#ifndef ENS_H
#define ENS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ens_status;
enum {
  ENS_OK = 0,
  ENS_W_NOT_CONVERGED = 1, /* a solve finished but some sample did not converge */
  ENS_E_ARG = -1,          /* null / misaligned pointer, bad size or option     */
  ENS_E_UNSUPPORTED = -2,  /* ensemble size or dtype not compiled in            */
  ENS_E_HIP = -3,          /* a HIP runtime call or kernel launch failed        */
  ENS_E_NOMEM = -4,        /* caller workspace smaller than required            */
  ENS_E_RANGE = -5         /* sizes beyond the 32-bit index range               */
};

/* per-sample outcome of a solve (ens_cg_stat.status) */
enum {
  ENS_SAMPLE_CONVERGED = 0,
  ENS_SAMPLE_MAXITER = 1,   /* iteration cap reached                            */
  ENS_SAMPLE_BREAKDOWN = 2, /* p.Ap <= 0: the sample's matrix is not SPD        */
  ENS_SAMPLE_NONFINITE = 3, /* NaN or Inf in a scalar of the iteration          */
  ENS_SAMPLE_STAGNATED = 4  /* refinement: outer residual stopped decreasing     */
};

typedef enum { ENS_F64 = 0, ENS_F32 = 1 } ens_dtype;

/* CRS graph (Sec. 2, Fig. "crs"): row_ptr[n+1], col_idx[nnz], columns
 * ascending within a row.  Both arrays are device memory. */
typedef struct {
  int32_t n;
  int64_t nnz;
  const int32_t* row_ptr;
  const int32_t* col_idx;
} ens_graph;

/* Diffusion coefficient (Sec. 4): kappa(x,y) = kappa0 + sigma *
 * sum_{m<M} sqrt(lambda_m) phi_m(x) y_m with (lambda_m, phi_m) the
 * eigenpairs of exp(-|x-x'|_1 / L) on [0,1]^3 ranked by lambda descending
 * (ties by ascending 1D index triple); source f is a constant. */
typedef struct {
  int32_t M;
  double L;
  double kappa0;
  double sigma;
  double f;
} ens_problem;

const char* ens_last_error(void);
const char* ens_status_string(ens_status st);
int32_t ens_abi_version(void);
/* Release the library's own per-device state: each device context (its
 * pinned poll word, work stream, join events and the concurrent baseline's
 * side streams, whose queued work is waited for first) and the pool of
 * profiling events (pending timings are completed and kept; profiling is
 * switched off).  Caller-owned buffers are untouched, and the state is
 * created again on the next call that needs it.  No library call may be
 * in flight on any thread when it runs.  Returns ENS_E_HIP with the first
 * runtime error met, after releasing what it could. */
ens_status ens_shutdown(void);

/* ------------------------------------------------------------ mesh/graph */

/* Sizes of the N x N x N element mesh of the unit cube (host, no GPU use):
 * n = (N+1)^3 nodes, nnz = (3N+1)^3 stored entries (full 27-point pattern,
 * Dirichlet rows and columns kept), N^3 elements.  ENS_E_RANGE if nnz*32
 * exceeds the 64-bit range or n exceeds int32. */
ens_status ens_mesh_sizes(int32_t N, int64_t* n, int64_t* nnz, int64_t* n_elem);

/* CRS graph of the Q1 stiffness matrix (Fig. "crs"; NodeIndex/ElemGraph
 * maps of Alg. "assembly").  Node (i,j,k) has id i + (N+1)(j + (N+1)k);
 * row i lists, ascending, every node that shares an element with i.
 * row_ptr (device) [n+1], col_idx (device) [nnz].  Never synchronises. */
ens_status ens_graph_build(int32_t N, int32_t* row_ptr, int32_t* col_idx, hipStream_t stream);

/* ------------------------------------------------------------------- KL */

/* Bytes of the device KL table for an N-element mesh and M terms. */
ens_status ens_kl_bytes(int32_t N, int32_t M, size_t* bytes);

/* Build the KL table on the device (Sec. 4, KL expansion of kappa): the
 * first M 1D eigenpairs of exp(-|t-t'|/L) on [0,1], the top-M 3D modes,
 * and the 1D eigenfunctions at the 2N Gauss abscissae of each axis.
 * Layout of `kl` (device, ens_kl_bytes bytes, 16-byte aligned):
 *   double sqrt_lam3[M]; double lam3[M]; double omega[M]; double lam1[M];
 *   double norm1[M]; int32 parity1[M]; int32 triple[M][3];
 *   (padding to 8 bytes) double phi1d[M][2N]   (phi of 1D mode k at
 *   abscissa (e + g_q)/N, index 2e+q, g_0 < g_1 the 2-point Gauss nodes). */
ens_status ens_kl_build(int32_t N, int32_t M, double L, void* kl, hipStream_t stream);

/* ------------------------------------------------------------ grouping */

/* Per-sample extremes of the coefficient over the Gauss points of the N^3
 * mesh: kmin[e] and kmax[e] (device FP64 [s]) are the minimum and maximum of
 * kappa(x_q, xi_e) = kappa0 + sigma sum_m sqrt(lambda_m) phi_m(x_q) xi_e[m]
 * over the 8 N^3 Gauss points (Sec. 4, KL expansion of kappa), for any
 * s >= 1.  The spread kmax / kmin is the paper's suggested predictor of a
 * sample's iteration count (Sec. 3.7: the variation of the sample's
 * parameters over the domain).  kl from ens_kl_build(N, M, L); xi [s][M]
 * device.  A sample with a non-finite coefficient gets NaN extremes.
 * Stream ordered; allocates nothing. */
ens_status ens_kl_extrema(int32_t N, const void* kl, const ens_problem* problem, int32_t s, const double* xi,
                          double* kmin, double* kmax, hipStream_t stream);
/* Order `count` samples for grouping into ensembles (Sec. 3.7: samples of
 * similar iteration counts belong in one ensemble): perm (host, [count])
 * lists the sample indices by ascending key (host, [count]), equal keys in
 * index order, non-finite keys last in index order; consecutive runs of
 * perm are the ensembles.  Host only; count = 0 is a no-op. */
ens_status ens_group_order(int64_t count, const double* key, int32_t* perm);

/* ------------------------------------------------------------- assembly */

/* Ensemble assembly of A and f (Alg. "assembly" made atomic-free): every
 * stored entry A_ij[e] is the sum over the elements containing i and j, in
 * ascending element id, of the element stiffness
 *   K_e[a][b] = sum_q kappa(x_q, y_e) grad N_a(x_q).grad N_b(x_q) h^3/8
 * over the 2x2x2 Gauss points; f_i[e] = sum over elements of f h^3/8.
 * Dirichlet u = 0: boundary rows become identity rows, boundary columns of
 * interior rows are stored zeros, boundary loads are zero.
 *   graph      from ens_graph_build(N)
 *   kl         from ens_kl_build(N, problem->M, problem->L)
 *   xi         (device) [s][M] KL inputs y
 *   values     (device) [nnz][s] FP64 out
 *   values32   (device) [nnz][s] FP32 out, round-to-nearest of values; may be NULL
 *   rhs        (device) [n][s] FP64 out
 * Never synchronises. */
ens_status ens_assemble(int32_t N, const ens_graph* graph, const void* kl, const ens_problem* problem,
                        int32_t s, const double* xi, double* values, float* values32, double* rhs,
                        hipStream_t stream);

/* The nonlinear problem of Sec. 4 (Eq. diffusion_sys):
 *   -div(kappa grad u) + alpha v.grad u + beta u^2 = f,  u = 0 on the boundary,
 * kappa as in ens_problem, v = (vx, vy, vz) a constant velocity. */
typedef struct {
  int32_t M;
  double L;
  double kappa0;
  double sigma;
  double f;
  double alpha;
  double beta;
  double vx, vy, vz;
} ens_nl_problem;

/* Residual F(u) and Jacobian A = dF/du (Eq. fenl_lin_sys) of the Q1
 * Galerkin discretisation with the 2x2x2 Gauss rule, per sample, assembled
 * like ens_assemble (row-owned, ascending element order, no atomics):
 *   F_i = sum_e sum_q w_q [kappa grad N_a.grad u_h + alpha N_a v.grad u_h
 *                          + beta N_a u_h^2 - f N_a]
 *   A_ij = sum_e sum_q w_q [kappa grad N_a.grad N_b + alpha N_a v.grad N_b
 *                           + 2 beta u_h N_a N_b]
 * with u_h interpolating u at the element's 8 nodes (boundary nodes with
 * their values).  Boundary rows: F_i = u_i and identity rows; boundary
 * columns of interior rows are stored zeros.
 *   u       (device) [n][s] in
 *   values  (device) [nnz][s] FP64 Jacobian out; may be NULL
 *   values32 (device) [nnz][s] the Jacobian rounded to FP32, out; may be
 *           NULL (both NULL: residual only)
 *   F       (device) [n][s] out
 *   load    (device) [n][s] out, the source part sum w_q f N_a of interior
 *           rows (zero on the boundary, so F(0) = -load); may be NULL
 * Other arguments as for ens_assemble.  Never synchronises. */
ens_status ens_nl_assemble(int32_t N, const ens_graph* graph, const void* kl, const ens_nl_problem* problem,
                           int32_t s, const double* xi, const double* u, double* values, float* values32, double* F,
                           double* load, hipStream_t stream);

/* ----------------------------------------------------------------- SpMV */

/* Ensemble CRS product y = A x in the commuted layout (Fig.
 * "ensemble_crs"): y[i][e] = sum_k values[k][e] x[col_idx[k]][e], entries
 * summed in ascending k.  values [nnz][s], x and y [n][s] (device) of the
 * dtype given; y must not overlap x or values.  Never synchronises. */
ens_status ens_spmv(const ens_graph* graph, int32_t s, ens_dtype dtype, const void* values,
                    const void* x, void* y, hipStream_t stream);

/* Scalar CRS product (Fig. "crs") of ONE sample: values [nnz], x and y [n]
 * (device).  This is the one-sample-at-a-time baseline of the paper's
 * speed-up definition (Sec. 4).  lanes_per_row 0 (the default): each
 * 256-lane workgroup reads the entries of 64 (FP64) or 32 (FP32)
 * consecutive rows in coalesced sweeps, forms the products in LDS and sums
 * each row in ascending entry order, every product rounded once;
 * lanes_per_row in {4, 8, 16, 32, 64}: that many lanes share a row.
 * Negative or other values: ENS_E_ARG. */
ens_status ens_scalar_spmv(const ens_graph* graph, ens_dtype dtype, const void* values, const void* x,
                           void* y, int32_t lanes_per_row, hipStream_t stream);

/* ------------------------------------------------------------------ CG */

typedef struct {
  double rtol;            /* stop sample e when |r_e|_2 <= rtol |b_e|_2      */
  int32_t max_iter;       /* FP64 CG: iteration cap per sample (<=0: 10000)   */
  int32_t mixed;          /* 0: FP64 Jacobi-CG; 1: FP32 Jacobi-CG inside FP64
                             iterative refinement (needs values32)           */
  double inner_rtol;      /* mixed: inner stop |r_in| <= inner_rtol |r_out|   */
  int32_t inner_max_iter; /* mixed: cap per inner solve (<=0: 10000)          */
  int32_t max_outer;      /* mixed: cap on refinement steps (<=0: 10)         */
  int32_t check_every;    /* iterations between polls of the device done flag
                             (<=0: 16)                                       */
  int32_t coupled;        /* 0: per-sample scalars and masks (default);
                             1: the coupled solve of the whole commuted
                             system (Sec. 3.4, Sec. 3.7): inner products are
                             summed over the ensemble, so every sample takes
                             the same alpha, beta and iteration count, and
                             the test is |r| <= rtol |b| over all samples
                             together.  FP64 only (mixed must be 0); stats
                             still report each sample's true residual. */
  int32_t compact;        /* 1: compaction of finished samples (Sec. 3.7: a
                             finished sample still costs its share of every
                             pass over the ensemble).  FP64 per-sample CG
                             only (mixed and coupled 0; ENS_E_ARG otherwise),
                             s >= 8 (no effect for s = 4): at the first poll
                             where at most s/2 samples still iterate, those
                             samples move to an ensemble of s/2 (matrix
                             values, x, r, p, D^-1 and their CG state
                             gathered), finish there, and x and the stats are
                             scattered back.  Each sample's iterates are
                             those of the uncompacted solve up to rounding;
                             the workspace grows by the s/2 ensemble.
                             Only ens_cg compacts: ens_cg_mg, ens_scalar_cg
                             and ens_scalar_cg_concurrent return ENS_E_ARG
                             for compact = 1. */
} ens_cg_opts;

typedef struct {
  int32_t iters;       /* CG iterations (mixed: total inner iterations)      */
  int32_t outer_iters; /* mixed: refinement steps taken; 0 for FP64 CG       */
  int32_t status;      /* ENS_SAMPLE_*                                       */
  int32_t compacted;   /* 1 if the sample finished in the compacted ensemble */
  double rel_res;      /* true FP64 residual |b - A x| / |b| of the result   */
} ens_cg_stat;

/* Bytes of caller workspace ens_cg needs for this graph, s and options. */
ens_status ens_cg_workspace_bytes(const ens_graph* graph, int32_t s, const ens_cg_opts* opts,
                                  size_t* bytes);

/* Ensemble Jacobi-preconditioned CG with per-sample scalars (Sec. 3.4: CG
 * on the ensemble system; preconditioner D_c = sum_i D_i (x) e_i e_i^T,
 * the diagonal instance of Sec. 3.5's M_c).  Every sample e keeps its own
 * alpha_e, beta_e, rho_e and convergence mask, so the ensemble iteration is
 * sample by sample the scalar iteration (Eq. kron_sys block structure);
 * a converged sample's x, r and p are frozen.  Iteration:
 *   q = A p; alpha = rho/(p.q); x += alpha p; r -= alpha q;
 *   stop if |r| <= rtol |b|; z = D^-1 r; rho' = r.z; p = z + (rho'/rho) p.
 *   values   (device) [nnz][s] FP64
 *   values32 (device) [nnz][s] FP32, used only when opts->mixed
 *   b        (device) [n][s] FP64
 *   x        (device) [n][s] FP64 in: initial guess x0, out: solution
 *   workspace(device) >= ens_cg_workspace_bytes, 256-byte aligned
 *   stats    (host)   [s] out
 * Mixed mode: outer FP64 residual r = b - A x, then the FP32 Jacobi-CG
 * above on the FP32 matrix for the correction d to inner_rtol, then
 * x += d in FP64; repeated until |b - A x| <= rtol |b| per sample.
 * Synchronises the stream; returns ENS_W_NOT_CONVERGED if any sample ends
 * with a status other than ENS_SAMPLE_CONVERGED. */
ens_status ens_cg(const ens_graph* graph, int32_t s, const double* values, const float* values32,
                  const double* b, double* x, const ens_cg_opts* opts, void* workspace,
                  size_t ws_bytes, ens_cg_stat* stats, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ens_cg with
 * the workspace taken from a scratch array inside the library instead of a
 * caller buffer.  Arguments, results and errors as for ens_cg, bitwise the
 * same results.  The scratch is a file-scope device array of 256 MiB
 * (ENS_CG_NOALLOC_SCRATCH_BYTES), one per GPU the library runs on, held
 * until the process ends; a solve whose ens_cg_workspace_bytes exceeds it
 * returns ENS_E_NOMEM before any device work (for FP64 CG about
 * 40 n s bytes: 64^3 elements at s = 16 fits, at s = 32 it does not).  The
 * first call on a device resolves the array's address there
 * (hipGetSymbolAddress); no call allocates memory: polls copy into host
 * stack words and the library's profiling events are not used.  Every call
 * on a GPU uses that GPU's one array, which keeps the last call's contents
 * (each call initialises what it reads): calls that overlap on one GPU
 * (other threads or streams) race and must be serialised by the caller.
 * Synchronises the stream. */
#define ENS_CG_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
ens_status ens_cg_noalloc(const ens_graph* graph, int32_t s, const double* values, const float* values32,
                          const double* b, double* x, const ens_cg_opts* opts, ens_cg_stat* stats,
                          hipStream_t stream);

/* The same Jacobi-CG for s independent systems solved one after another
 * with one-sample kernels on the sample-major layout of Eq. kron_sys:
 * values [s][nnz], b and x [s][n] (device).  FP64 only (opts->mixed must
 * be 0).  This is the "s times a single sample" side of the speed-up
 * definition of Sec. 4.  lanes_per_row selects the one-sample product as
 * in ens_scalar_spmv (0, the default, or 4, 8, 16, 32).  Workspace from
 * ens_cg_workspace_bytes(graph, 4, opts) suffices.  Synchronises. */
ens_status ens_scalar_cg(const ens_graph* graph, int32_t s, const double* values, const double* b,
                         double* x, const ens_cg_opts* opts, int32_t lanes_per_row, void* workspace,
                         size_t ws_bytes, ens_cg_stat* stats, hipStream_t stream);

/* ---------------------------------------------------------------- batch */

/* One sample group of a batch: an ensemble of s samples on its own mesh. */
typedef struct {
  const ens_graph* graph; /* (host struct) device graph of the group's mesh      */
  const double* values;   /* (device) [nnz][s] FP64                              */
  const double* b;        /* (device) [n][s]                                     */
  double* x;              /* (device) [n][s]: in initial guess, out solution     */
  ens_cg_stat* stats;     /* (host) [s] out                                      */
} ens_group;

typedef struct {
  double rtol;          /* per sample: |r| <= rtol |b|                          */
  int32_t max_iter;     /* per sample (<= 0: 10000)                             */
  int32_t check_every;  /* iterations per graph replay / host poll (<= 0: 16)   */
  int32_t tile;         /* wavefronts per row-tile workgroup: 2, 4 or 8          */
  int32_t use_graph;    /* 1: capture one chunk of iterations in a HIP graph and
                           replay it; 0: launch the same kernels directly      */
} ens_batch_opts;

/* Bytes of workspace ens_solve_batch needs for these groups. */
ens_status ens_batch_workspace_bytes(const ens_group* groups, int32_t n_groups, int32_t s,
                                     const ens_batch_opts* opts, size_t* bytes);

/* FP64 Jacobi-CG (the iteration of ens_cg, per-sample scalars and masks) of
 * all groups at once: every CG phase is one launch over the row tiles or
 * vector blocks of all groups, groups of different mesh sizes included, and
 * each group's reductions and stopping decisions are its own.  Groups are
 * independent systems (the block structure of Eq. kron_sys; Sec. 5 notes
 * that grouped ensembles propagate independently).  s in {8, 16, 32}, the
 * same for all groups.  Work runs on a library stream ordered after
 * `stream` and joined back to it; synchronises; per-sample stats written to
 * each group's host array; ENS_W_NOT_CONVERGED if any sample did not
 * converge. */
ens_status ens_solve_batch(const ens_group* groups, int32_t n_groups, int32_t s, const ens_batch_opts* opts,
                           void* workspace, size_t ws_bytes, hipStream_t stream);

/* The KL inputs of one group for ens_assemble_solve_batch. */
typedef struct {
  int32_t N;          /* the group's mesh: N^3 elements (graph of ens_graph_build(N)) */
  const void* kl;     /* (device) ens_kl_build(N, problem->M, problem->L)             */
  const double* xi;   /* (device) [s][M] KL inputs of the group's samples             */
} ens_group_input;

/* Assembly and batched solve of a wave of groups in one call: every group's
 * matrix and load vector are assembled (ens_assemble's operator, FP64
 * values, Alg. assembly) into its values and b (outputs here; the const of
 * ens_group does not apply), its x set to zero, and the groups solved as by
 * ens_solve_batch.  The assemblies of all groups run as one launch over
 * all their tiles, and with opts->use_graph that launch, the solver's
 * set-up and the first chunk of iterations are one captured graph, the
 * further chunks another, replayed.  Results equal ens_assemble per group
 * followed by ens_solve_batch, bitwise.  Workspace from
 * ens_assemble_solve_batch_workspace_bytes (the solver's plus the assembly
 * tables); s in {8, 16, 32}; synchronises. */
ens_status ens_assemble_solve_batch_workspace_bytes(const ens_group* groups, const ens_group_input* inputs,
                                                    int32_t n_groups, int32_t s, const ens_problem* problem,
                                                    const ens_batch_opts* opts, size_t* bytes);
ens_status ens_assemble_solve_batch(const ens_group* groups, const ens_group_input* inputs, int32_t n_groups,
                                    int32_t s, const ens_problem* problem, const ens_batch_opts* opts,
                                    void* workspace, size_t ws_bytes, hipStream_t stream);

/* Autotuner for ens_solve_batch (the ensemble size must suit the
 * architecture, Sec. 3 and Sec. 5): for every candidate ensemble size
 * s_cand[ns] (8, 16, 32) and row-tile shape tile_cand[nt] (2, 4, 8
 * wavefronts per workgroup), solves the same 32 samples of each mesh in
 * meshes[nm] (N per axis), split into 32/s groups, with ens_solve_batch
 * under the options *base (its tile ignored), and returns the pair with the
 * most solved samples per second.  xi_host (host) [nm][32][problem->M] holds
 * the KL inputs.  scores (host, nullable) [ns*nt] receives every score
 * (samples/s, index a*nt + c).  With scores NULL and an entry for the same
 * meshes, problem and options in cache_path (nullable; a text file of lines
 * "key s tile", the last one wins), the cached pair is returned without
 * trials (workspace may then be NULL); every completed search appends its
 * result.  The trial buffers (each mesh's graph, KL table and 32 samples'
 * values, b and x, then the largest solver workspace of the candidates)
 * live in the caller-owned device `workspace` (256-byte aligned) of
 * ws_bytes >= ens_batch_autotune_workspace_bytes(...) bytes, about
 * 32 * 8 * (nnz + 3 n) bytes per mesh; the library allocates no device
 * memory.  Synchronises (the timing of each trial needs it); on an error
 * the stream is drained before returning. */
ens_status ens_batch_autotune_workspace_bytes(const int32_t* meshes, int32_t nm, const ens_problem* problem,
                                              const int32_t* s_cand, int32_t ns, const int32_t* tile_cand,
                                              int32_t nt, const ens_batch_opts* base, size_t* bytes);
ens_status ens_batch_autotune(const int32_t* meshes, int32_t nm, const ens_problem* problem, const double* xi_host,
                              const int32_t* s_cand, int32_t ns, const int32_t* tile_cand, int32_t nt,
                              const ens_batch_opts* base, const char* cache_path, int32_t* best_s,
                              int32_t* best_tile, double* scores, void* workspace, size_t ws_bytes,
                              hipStream_t stream);

/* ------------------------------------------------------------ multigrid */

/* Multigrid preconditioner (Sec. 3.5, Alg. vcycle) for the ensemble Q1
 * problem on the N^3 mesh: levels N, N/2, ... (halved while even and above
 * 4; the coarsest level must have at most 512 interior nodes), each level's
 * ensemble matrix assembled on its own mesh with the samples' KL inputs;
 * trilinear prolongation onto interior nodes and its transpose as
 * restriction; order-2 Chebyshev smoothers in D^-1 A on [lmax/4, lmax] with
 * lmax each sample's Gershgorin bound max_i sum_j |a_ij| / a_ii; the
 * coarsest interior block solved exactly (per-sample dense inverse).  Each
 * sample has its own hierarchy, so the ensemble preconditioner is
 * M_c = sum_i M_i (x) e_i e_i^T.  The hierarchy lives in one caller-owned
 * device buffer (256-byte aligned, ens_mg_bytes). */
typedef struct {
  int32_t N;      /* fine mesh: N elements per axis                        */
  int32_t M;      /* KL terms of the problem                                */
  int32_t s;      /* ensemble size (4, 8, 16, 32)                            */
  int32_t fp32;   /* 0: FP64 cycle; 1: FP32 cycle on FP32 matrices (for the
                     refinement's inner solve)                            */
  void* buffer;   /* (device) hierarchy storage                             */
  size_t bytes;   /* its size, >= ens_mg_bytes(N, M, s, fp32)               */
} ens_mg;

ens_status ens_mg_bytes(int32_t N, int32_t M, int32_t s, int32_t fp32, size_t* bytes);
/* The sample-independent part of the hierarchy: the coarse meshes' graphs
 * and KL tables (correlation length L).  Once per buffer, before any
 * ens_mg_setup; stream ordered.  The library records which buffers (by
 * address and shape) are built and set up, and for which L: ens_mg_setup on
 * an unbuilt buffer or with another problem->L, and ens_cg_mg on a buffer
 * not set up, return ENS_E_ARG. */
ens_status ens_mg_build(const ens_mg* mg, double L, hipStream_t stream);
/* Set the hierarchy up for one ensemble: the coarse levels' matrices for the
 * KL inputs xi [s][M] (device) and `problem` (whose M and L are those of
 * ens_mg_build), D^-1 and bounds of every level, the coarsest inverse.
 * `values` [nnz][s] is the fine matrix of `graph` (the N^3 mesh); with fp32
 * also its FP32 copy values32.  Stream ordered; never synchronises.  The fine
 * matrices must stay unchanged while the hierarchy is used. */
ens_status ens_mg_setup(const ens_mg* mg, const ens_graph* graph, const double* values, const float* values32,
                        const ens_problem* problem, const double* xi, hipStream_t stream);
/* ens_assemble of the fine matrix (values, values32, rhs as there; kl from
 * ens_kl_build(N, M, L)) followed by ens_mg_setup, with the fine level's D^-1
 * and Gershgorin bound formed inside the assembly (the same values, bitwise,
 * without a separate pass over the fine matrix).  An FP32 hierarchy of more
 * than one level does not read the FP64 fine matrix: values may then be
 * NULL, and only values32 is formed.  Arguments and errors as for the two
 * calls; stream ordered. */
ens_status ens_mg_assemble_setup(const ens_mg* mg, const ens_graph* graph, const void* kl,
                                 const ens_problem* problem, const double* xi, double* values, float* values32,
                                 double* rhs, hipStream_t stream);
/* ens_mg_assemble_setup for the advection-diffusion operator D + alpha C,
 * the linear part of the nonlinear problem's Jacobian (Sec. 4, Eq.
 * fenl_lin_sys with beta = 0; D the diffusion matrix of Alg. assembly,
 * C_ab = int N_a v.grad N_b), rediscretized on every level with the
 * problem's kappa, alpha and v: the fine matrix into values / values32 (rhs:
 * the load), D^-1 and Gershgorin bounds max_i sum_j |a_ij| / a_ii of every
 * level, the coarsest inverse (Gauss-Jordan without pivoting: on interior
 * nodes C is skew-symmetric, so the block's symmetric part is the diffusion
 * block's, positive definite).  Meant as the right preconditioner of
 * ens_gmres and ens_newton (mg_values = values, or values32 for an FP32
 * hierarchy): it sees the advection the diffusion cycle misses.
 * problem->beta is not used.  ens_cg_mg refuses a hierarchy set up this way
 * (ENS_E_ARG) until ens_mg_setup or ens_mg_assemble_setup sets it up again.
 * Arguments and errors otherwise as for ens_mg_assemble_setup; non-finite
 * alpha or v: ENS_E_ARG. */
ens_status ens_mg_assemble_setup_adv(const ens_mg* mg, const ens_graph* graph, const void* kl,
                                     const ens_nl_problem* problem, const double* xi, double* values,
                                     float* values32, double* rhs, hipStream_t stream);
/* ens_mg_setup with the coarse operators of Alg. vcycle as printed (Sec.
 * 3.5): A^{k+1} = R^k A^k P^k, R = P^T, each coarse level the Galerkin
 * product of the level above instead of an assembly on its own mesh.  Per
 * sample, in FP64 from the FP64 matrix of the level above (the fine one:
 * `values`, required); an FP32 cycle's coarse copies are rounded from them.
 * Every term P_iI A_ij P_jJ is exact (the weights are powers of two) and
 * the terms of an entry are summed in a fixed order (children of I, then
 * row entries, then parents of j, each ascending in z, y, x), so the result
 * is deterministic.  Coarse boundary rows are identity rows and boundary
 * columns of interior rows stored zeros, as on assembled levels.  D^-1 and
 * the Gershgorin bound of every level are formed by a pass over the matrix
 * the cycle runs on, then the coarsest inverse.  No KL input is needed:
 * the coarse levels see the coefficient only through the fine matrix.
 * Buffer built by ens_mg_build; graph the N^3 mesh's; arguments and errors
 * otherwise as for ens_mg_setup.  Stream ordered. */
ens_status ens_mg_setup_galerkin(const ens_mg* mg, const ens_graph* graph, const double* values,
                                 const float* values32, hipStream_t stream);
/* ens_mg_assemble_setup with Galerkin coarse levels (ens_mg_setup_galerkin):
 * the fine matrix assembled into values (required), values32 and rhs, the
 * fine level's D^-1 and bound formed by the assembly, then the Galerkin
 * products.  Arguments and errors as for ens_mg_assemble_setup, except
 * that values may not be NULL. */
ens_status ens_mg_assemble_setup_galerkin(const ens_mg* mg, const ens_graph* graph, const void* kl,
                                          const ens_problem* problem, const double* xi, double* values,
                                          float* values32, double* rhs, hipStream_t stream);
/* Where coarse level `level` (1 .. levels-1; level 0 is the caller's fine
 * matrix) keeps its operator inside the hierarchy buffer: *N its mesh size,
 * *values its FP64 matrix [nnz(N)][s] on the graph of ens_graph_build(N),
 * *values32 its FP32 copy (NULL for an FP64 cycle).  Host only; device
 * pointers into mg->buffer, owned by the caller's buffer, valid as long as
 * it is; the contents are those of the last set-up.  For inspecting the
 * coarse operators (rediscretized or Galerkin).  ENS_E_ARG for a level out
 * of range. */
ens_status ens_mg_level_values(const ens_mg* mg, int32_t level, int32_t* N, const double** values,
                               const float** values32);
/* Forget the buffer's built / set-up record (host only, never fails on an
 * unknown buffer).  Call it before the buffer is freed: a later allocation
 * at the same address would otherwise pass as built. */
ens_status ens_mg_release(const ens_mg* mg);
/* CG with z = M r from the hierarchy, per-sample scalars and masks and the
 * stopping rule of ens_cg (opts->coupled and opts->compact must be 0).  opts->mixed = 0: FP64
 * CG with an FP64 cycle.  opts->mixed = 1: the FP32-in-FP64 refinement of
 * ens_cg whose FP32 inner CG (on values32) is preconditioned by an FP32
 * cycle.  Workspace from ens_cg_workspace_bytes(graph, s, opts).
 * Synchronises. */
ens_status ens_cg_mg(const ens_graph* graph, int32_t s, const double* values, const float* values32, const double* b,
                     double* x, const ens_cg_opts* opts, const ens_mg* mg, void* workspace, size_t ws_bytes,
                     ens_cg_stat* stats, hipStream_t stream);

/* ------------------------------------------------- nonlinear: GMRES, Newton */

/* Restarted GMRES(restart) with right preconditioning, per sample, for the
 * nonsymmetric Newton systems of the nonlinear problem (Eq. fenl_lin_sys
 * with alpha != 0): Arnoldi on A M with two classical Gram-Schmidt passes,
 * Givens rotations on each sample's Hessenberg matrix, the estimate
 * |g_{j+1}| <= rtol |b| tested after every step, at a cycle's end
 * x += M V y and the true residual recomputed; converged when the true
 * residual meets rtol |b|.  b = 0 gives x = 0.  Iterations count Arnoldi
 * steps (products with A) over all cycles. */
typedef struct {
  double rtol;
  int32_t restart;   /* 1..32 */
  int32_t max_iter;
} ens_gmres_opts;

ens_status ens_gmres_workspace_bytes(const ens_graph* graph, int32_t s, int32_t restart, size_t* bytes);
/* values [nnz][s] (the matrix), b and x [n][s] (x in: initial guess), all
 * device FP64.  Preconditioner M: mg == NULL -> Jacobi (the diagonal of
 * values); else the V-cycle of the set-up hierarchy `mg`, whose fine level
 * is the matrix mg_values [nnz][s] it was set up with (for the Newton
 * systems: the diffusion matrix of ens_mg_assemble_setup, or D + alpha C
 * of ens_mg_assemble_setup_adv), FP64 for an FP64 hierarchy and FP32
 * (values32) for an FP32 one.  An FP32 cycle takes its input rounded to
 * FP32 and its output is widened back; the Krylov basis, products and
 * updates stay FP64, and the true residual at each cycle's end decides
 * convergence.  With multigrid the workspace keeps each step's M v_j and a
 * cycle ends with x += sum_j y_j M v_j (no further cycle).  stats[e]: iters,
 * outer_iters = restart cycles, status, rel_res = the final relative
 * residual.  Synchronises. */
ens_status ens_gmres(const ens_graph* graph, int32_t s, const double* values, const double* b, double* x,
                     const ens_gmres_opts* opts, const ens_mg* mg, const void* mg_values, void* workspace,
                     size_t ws_bytes, ens_cg_stat* stats, hipStream_t stream);

/* Newton's method per sample on F(u) = 0 (Sec. 4, Eq. fenl_lin_sys):
 * at u_k assemble F and A = dF/du (ens_nl_assemble); stop the sample when
 * |F(u_k)| <= rtol |load| (|F(u_0)| if the load is zero), at non-finite
 * norms, or after max_newton steps; otherwise solve A d = F by ens_gmres to
 * the forcing term of the step (opts->forcing) from d = 0 and set
 * u_{k+1} = u_k - d.  The inner solve accepts a cycle's Arnoldi residual
 * estimate when it meets the forcing term (the true residual is formed only
 * before a further cycle; the next step's exact |F| is the check).  A
 * linear solve that breaks down or turns non-finite stops its sample with
 * that status. */
typedef struct {
  double rtol;
  int32_t max_newton;
  double lin_rtol;
  int32_t restart;       /* GMRES restart length, 1..32 */
  int32_t lin_max_iter;  /* GMRES iterations per Newton step */
  int32_t jac32;         /* 1: the Newton systems use the Jacobian rounded to
                            FP32 (read and widened by the FP64 GMRES); F, the
                            step and u stay FP64 and the FP64 |F| decides */
  int32_t forcing;       /* GMRES tolerance of step k: 0 -> lin_rtol; 1 ->
                            the second choice of Eisenstat and Walker (1996):
                            eta_k = 0.9 (|F_k|/|F_{k-1}|)^2, raised to
                            0.9 eta_{k-1}^2 when that exceeds 0.1, at most
                            lin_rtol (also eta_0), at least
                            0.5 rtol |load| / |F_k| */
} ens_newton_opts;

typedef struct {
  int32_t newton_iters;  /* Newton updates taken */
  int32_t lin_iters;     /* GMRES iterations over all steps */
  int32_t status;        /* ens_sample_status */
  int32_t reserved;
  double rel_res;        /* |F(u)| / |load| at exit */
} ens_newton_stat;

ens_status ens_newton_workspace_bytes(const ens_graph* graph, int32_t s, const ens_newton_opts* opts,
                                      size_t* bytes);
/* u [n][s] (device, in: initial guess, out: solution); xi [s][M] (device);
 * kl from ens_kl_build(N, problem->M, problem->L); mg / mg_values as for
 * ens_gmres (NULL: Jacobi).  The workspace holds the Jacobian, F, the load,
 * the step and the GMRES workspace.  Synchronises. */
ens_status ens_newton(int32_t N, const ens_graph* graph, const void* kl, const ens_nl_problem* problem, int32_t s,
                      const double* xi, double* u, const ens_newton_opts* opts, const ens_mg* mg,
                      const void* mg_values, void* workspace, size_t ws_bytes, ens_newton_stat* stats,
                      hipStream_t stream);

/* The one-sample baseline with up to `streams` (1..32) solves in flight at
 * once, each on its own library stream (default priority) with its own
 * workspace slice, so that independent solves overlap on the device as they
 * would when run side by side.  Same arguments, layouts and per-sample
 * results as ens_scalar_cg; workspace from
 * ens_scalar_cg_concurrent_workspace_bytes.  Ordered after earlier work on
 * `stream` and before later work on it; synchronises. */
ens_status ens_scalar_cg_concurrent_workspace_bytes(const ens_graph* graph, int32_t streams, size_t* bytes);
ens_status ens_scalar_cg_concurrent(const ens_graph* graph, int32_t s, const double* values, const double* b,
                                    double* x, const ens_cg_opts* opts, int32_t lanes_per_row, int32_t streams,
                                    void* workspace, size_t ws_bytes, ens_cg_stat* stats, hipStream_t stream);

/* Layout change between the commuted [rows][s] and the sample-major
 * [s][rows] arrangement (Eqs. kron_sys_commuted and kron_sys), FP64,
 * out-of-place.  to_sample_major = 1: src [rows][s] -> dst [s][rows]. */
ens_status ens_relayout(const double* src, double* dst, int64_t rows, int32_t s, int32_t to_sample_major,
                        hipStream_t stream);

/* ------------------------------------------------- learned initial guess */

/* A reduced basis and a small network predict an initial guess for CG from
 * the KL inputs y of a sample; CG remains the solver and decides the
 * error (an extension of the method; the paper solves from zero).
 *
 * Network: 10 -> 256 -> 256 -> 32, GELU (exact erf form) after the two
 * hidden layers, linear output.  Parameters are one FP32 array of
 * ens_mlp_param_count() = 76,832 floats:
 *   W1 [256][10] | b1 [256] | W2 [256][256] | b2 [256] | W3 [32][256] | b3 [32]
 * Products run on the matrix cores with BF16 operands (inputs, weights and
 * activations rounded to nearest even) and FP32 accumulation; bias, GELU,
 * loss and Adam are FP32.  `batch` must be a multiple of 32 in [32, 65536].
 * Workspace (device, 256-byte aligned) from ens_mlp_workspace_bytes. */
int64_t ens_mlp_param_count(void);
ens_status ens_mlp_workspace_bytes(int32_t batch, size_t* bytes);

/* out [batch][32] (device) = network(xi [batch][10] (device)). */
ens_status ens_mlp_forward(const float* params, int32_t batch, const float* xi, float* out, void* workspace,
                           size_t ws_bytes, hipStream_t stream);

/* One forward and backward pass of the mean squared error
 * L = mean over batch and outputs of (out - target)^2: grad [76832] and
 * loss [1] (device) out; out [batch][32] optional. */
ens_status ens_mlp_grad(const float* params, int32_t batch, const float* xi, const float* target, float* out,
                        float* grad, float* loss, void* workspace, size_t ws_bytes, hipStream_t stream);

/* `steps` Adam steps (lr, beta = (0.9, 0.999), eps = 1e-8) on mini-batches
 * of the training set xi [count][10], target [count][32] (device): step s
 * uses the rows batch_idx[s*batch .. s*batch+batch-1] (device int32, the
 * caller's shuffle).  params, adam_m, adam_v [76832] are updated in place;
 * step0 = number of Adam steps already taken (bias correction); loss
 * [steps] (device, nullable) receives each step's batch loss. */
ens_status ens_mlp_train(float* params, float* adam_m, float* adam_v, int32_t step0, const float* xi,
                         const float* target, int32_t count, int32_t batch, int32_t steps, const int32_t* batch_idx,
                         float lr, float* loss, void* workspace, size_t ws_bytes, hipStream_t stream);

/* One Adam step (Kingma and Ba, ICLR 2015, Algorithm 1; the optimiser of
 * ens_mlp_train, which runs this same kernel after each gradient) on `count`
 * FP32 elements (device): with b1 = 0.9, b2 = 0.999, eps = 1e-8 and t = step
 * (1-based, the bias correction),
 *   m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
 *   params -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * params, adam_m, adam_v updated in place, grad read; none may alias another.
 * ENS_E_ARG for null pointers, count outside [0, INT32_MAX], step < 1 or
 * lr <= 0.  Stream-ordered, no synchronisation. */
ens_status ens_mlp_adam(float* params, const float* grad, float* adam_m, float* adam_v, int64_t count, int32_t step,
                        float lr, hipStream_t stream);

/* POD by the method of snapshots, FP64.  S [n][m] (device) holds one
 * solution per column.
 * ens_pod_collect: S[i][col0 + e] = x[i][e] for an ensemble x [n][s].
 * ens_pod_gram:    G [m][m] = S^T S (split-K workspace of
 *                  ens_pod_gram_workspace_bytes).
 * ens_pod_eig:     top-r eigenpairs of G by `iters` steps of block subspace
 *                  iteration on k >= r columns from the seeded start block
 *                  start [m][k], then Rayleigh-Ritz (Jacobi on k x k);
 *                  V [m][r] orthonormal, lambda [r] descending (device).
 * ens_pod_basis:   Phi [n][r] = S V diag(lambda)^(-1/2), each column's
 *                  largest-magnitude entry made positive.
 * ens_pod_project: C [s][r] = X^T Phi for an ensemble X [n][s].
 * ens_pod_standardize: per-coefficient mean mu [r] over the m rows of
 *                  C [m][r] (r <= 1024), a scale sd [r] and the network
 *                  targets T [m][r] = (C - mu) / sd in FP32; common = 0:
 *                  sd[j] the standard deviation of coefficient j;
 *                  common = 1: every sd[j] the largest of those
 *                  deviations, so the targets keep the coefficients'
 *                  relative sizes and a network's squared error on them is
 *                  the squared error of the reconstructed guess (Phi is
 *                  orthonormal).
 * ens_pod_reconstruct: x0 [n][s] = Phi (mu + sd c)^T for network outputs
 *                  c [s][r] (FP32; mu, sd nullable for raw coefficients),
 *                  written in the ensemble layout ready for ens_cg;
 *                  s * r <= 8192 (ENS_E_ARG otherwise). */
ens_status ens_pod_collect(const double* x, int64_t n, int32_t s, double* S, int32_t m, int32_t col0,
                           hipStream_t stream);
ens_status ens_pod_gram_workspace_bytes(int64_t n, int32_t m, size_t* bytes);
ens_status ens_pod_gram(const double* S, int64_t n, int32_t m, double* G, void* workspace, size_t ws_bytes,
                        hipStream_t stream);
ens_status ens_pod_eig_workspace_bytes(int32_t m, int32_t k, size_t* bytes);
ens_status ens_pod_eig(const double* G, int32_t m, int32_t k, int32_t r, const double* start, int32_t iters,
                       double* V, double* lambda, void* workspace, size_t ws_bytes, hipStream_t stream);
ens_status ens_pod_basis(const double* S, int64_t n, int32_t m, const double* V, const double* lambda, int32_t r,
                         double* Phi, hipStream_t stream);
ens_status ens_pod_project_workspace_bytes(int64_t n, int32_t r, int32_t s, size_t* bytes);
ens_status ens_pod_project(const double* Phi, const double* X, int64_t n, int32_t r, int32_t s, double* C,
                           void* workspace, size_t ws_bytes, hipStream_t stream);
ens_status ens_pod_standardize(const double* C, int32_t m, int32_t r, int32_t common, double* mu, double* sd,
                               float* T, hipStream_t stream);
ens_status ens_pod_reconstruct(const double* Phi, int64_t n, int32_t r, const float* c, const double* mu,
                               const double* sd, int32_t s, double* x0, hipStream_t stream);

/* ----------------------------------------------------------- measurement */

/* Plain device copy of `bytes` bytes (multiple of 16), used to calibrate
 * hardware traffic counters against a kernel of known traffic, and the
 * STREAM-style triad a[i] = b[i] + q c[i] in FP64 (the bandwidth the paper
 * bounds its SpMV with, Sec. 4).  Never synchronise. */
ens_status ens_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t stream);
ens_status ens_stream_triad(double* a, const double* b, const double* c, double q, int64_t n,
                            hipStream_t stream);
/* Pure read stream of `bytes` bytes (multiple of 16, 16-byte aligned src),
 * the read-only bandwidth ceiling next to the copy and the triad: every
 * 16-byte chunk is read once, and the chunks of each ENS_STREAM_READ_CHUNK_BYTES
 * piece are folded by XOR into one word, out (device)
 * [ceil(bytes / ENS_STREAM_READ_CHUNK_BYTES)] uint32.  ENS_E_RANGE above
 * 128 GiB.  Never synchronises. */
#define ENS_STREAM_READ_CHUNK_BYTES 16384
ens_status ens_stream_read(const void* src, size_t bytes, uint32_t* out, hipStream_t stream);
/* Pure write stream: dst (device, 16-byte aligned) [bytes / 16] 16-byte
 * chunks set to (value, value ^ 1, value ^ 2, value ^ 3) with ordinary
 * stores, as the assemblies write their values; the write-only bandwidth
 * ceiling.  bytes a multiple of 16.  Never synchronises. */
ens_status ens_stream_write(void* dst, size_t bytes, uint32_t value, hipStream_t stream);

/* Kernel timing with HIP events recorded on the launch stream around every
 * launch of the listed kernels while enabled.  Enabling creates a pool of
 * events up front (outside any region the caller times). */
enum {
  ENS_K_SPMV_F64 = 0,   /* ensemble SpMV (standalone and inside CG), FP64 */
  ENS_K_SPMV_F32 = 1,   /* ensemble SpMV, FP32 (refinement inner loop)   */
  ENS_K_ASSEMBLE = 2,
  ENS_K_SCALAR_SPMV = 3,
  ENS_K_MG_ROW = 4,     /* fine-level row passes of the multigrid cycle   */
  ENS_K_NL_ASSEMBLE = 5,/* nonlinear residual and Jacobian                  */
  ENS_K_GM_SPMV = 6,    /* the product w = A z of a GMRES step (FP64)       */
  ENS_K_GM_ORTH = 7,    /* GMRES Gram-Schmidt passes over the basis          */
  ENS_K_COUNT = 8
};
ens_status ens_prof_enable(int32_t on);
ens_status ens_prof_reset(void);
/* Totals since the last reset over the working launches of a kernel:
 * summed event durations (ms), launch count, and algorithmic bytes (the
 * kernel's byte model, summed per launch).  Launches shorter than 5 % of
 * the longest one -- solver kernels that found no active sample and
 * returned at once -- are left out. */
ens_status ens_prof_query(int32_t kernel_id, double* total_ms, int64_t* launches, double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* ENS_H */
