// Batched solve of many sample groups: every group is an ensemble of S
// samples on its own Q1 mesh (meshes of different sizes in one batch), and
// every CG phase runs for all groups in one launch.
//
// The work of a phase is a flat list of blocks: group g owns a contiguous
// range of row tiles (products) or of chunk blocks (vector updates), and a
// table maps each block to its group.  Block partials of the reductions are
// summed per group in two fixed-order stages (the first over chunks of at
// most kSegRows partial rows, the second one workgroup per group), and the
// second stage updates that group's per-sample state, so groups converge and
// stop independently: a finished group's blocks return at once.  A chunk of
// iterations is captured once into a HIP graph and replayed until every
// group has finished; the host reads one active count per replay.
//
// Why not one persistent kernel with in-kernel barriers between the phases:
// on this part a device-scope release/acquire fence writes back and
// invalidates the XCD's L2, and with one fence per block per phase the
// measured cost exceeds the launches a graph replays.
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "cgcore.hpp"
#include "mg.hpp"

namespace ens {

constexpr int kSegRows = 256;

struct GroupDev {
  int32_t n;
  int32_t nred, nredv;  // stage-1 rows of the row / vector reductions
  int64_t nnz;
  const int32_t* rp;
  const int32_t* ci;
  const double* vals;
  const double* b;
  double* x;
  double *r, *p, *q, *dinv;
  Ctl* ctl;
  int64_t row0, nrowb;  // flat row-tile blocks
  int64_t vec0, nvecb;  // flat chunk blocks
  int64_t red0, redv0;  // first stage-1 row
};

struct BatchDev {
  const GroupDev* groups;
  const int32_t* row_grp;   // [row blocks]
  const int32_t* vec_grp;   // [vector blocks]
  const int32_t* red_grp;   // [stage-1 rows of row reductions]
  const int32_t* redv_grp;  // [stage-1 rows of vector reductions]
  double* part;             // [max(row, vector blocks)][2S]
  double* out1;             // [max(stage-1 rows)][2S]
};

template <int S, int NW>
__global__ __launch_bounds__(NW * 64) void kb_spmv_dot(BatchDev bd) {
  const int64_t blk = blockIdx.x;
  const GroupDev& g = bd.groups[bd.row_grp[blk]];
  if (g.ctl->n_active == 0) return;
  spmv_dot_body<double, S, NW>(g.n, g.rp, g.ci, g.vals, g.p, g.q, blk - g.row0, bd.part + blk * S);
}

template <int S, int NW>
__global__ __launch_bounds__(NW * 64) void kb_residual(BatchDev bd, int store_r) {
  const int64_t blk = blockIdx.x;
  const GroupDev& g = bd.groups[bd.row_grp[blk]];
  residual_body<S, double, NW>(g.n, g.rp, g.ci, g.vals, g.x, g.b, store_r ? g.r : (double*)nullptr, blk - g.row0,
                               bd.part + blk * 2 * S);
}

template <int S>
__global__ __launch_bounds__(256) void kb_update(BatchDev bd) {
  const int64_t blk = blockIdx.x;
  const GroupDev& g = bd.groups[bd.vec_grp[blk]];
  if (g.ctl->n_active == 0) return;
  const int64_t nchunks = (int64_t)g.n * S / VecMap<double, S>::V;
  update_body<double, S>(nchunks, g.x, g.p, g.q, g.r, g.dinv, g.ctl, blk - g.vec0, bd.part + blk * 2 * S);
}

template <int S>
__global__ __launch_bounds__(256) void kb_pupdate(BatchDev bd) {
  const int64_t blk = blockIdx.x;
  const GroupDev& g = bd.groups[bd.vec_grp[blk]];
  if (g.ctl->n_active == 0) return;
  const int64_t nchunks = (int64_t)g.n * S / VecMap<double, S>::V;
  pupdate_body<double, S>(nchunks, g.r, g.dinv, g.p, g.ctl, blk - g.vec0);
}

template <int S>
__global__ __launch_bounds__(256) void kb_cg_start(BatchDev bd) {
  const int64_t blk = blockIdx.x;
  const GroupDev& g = bd.groups[bd.vec_grp[blk]];
  const int64_t nchunks = (int64_t)g.n * S / VecMap<double, S>::V;
  cg_start_body<double, S>(nchunks, g.r, g.dinv, g.p, (double*)nullptr, blk - g.vec0, bd.part + blk * 2 * S);
}

// Stage 1: stage-1 row c of group g sums partial rows
// [first + j kSegRows, first + (j+1) kSegRows) of that group, j = c - red0.
template <int P, int VEC>
__global__ __launch_bounds__(256) void kb_stage1(BatchDev bd, int gate) {
  const int64_t c = blockIdx.x;
  const GroupDev& g = bd.groups[(VEC ? bd.redv_grp : bd.red_grp)[c]];
  if (gate && g.ctl->n_active == 0) return;
  const int64_t first = VEC ? g.vec0 : g.row0;
  const int64_t count = VEC ? g.nvecb : g.nrowb;
  const int64_t j = c - (VEC ? g.redv0 : g.red0);
  const int64_t r0 = j * kSegRows;
  const int64_t r1 = r0 + kSegRows < count ? r0 + kSegRows : count;
  sum_rows<P>(bd.part + (first + r0) * P, r1 - r0, bd.out1 + c * P);
}

// Stage 2: workgroup g sums its stage-1 rows and updates its state.
template <int S, int NQ, int VEC>
__global__ __launch_bounds__(256) void kb_final(BatchDev bd, int op, int arg, int gate) {
  const GroupDev& g = bd.groups[blockIdx.x];
  Ctl* c = g.ctl;
  if (gate && c->n_active == 0) return;
  sum_rows<NQ * S>(bd.out1 + (VEC ? g.redv0 : g.red0) * NQ * S, VEC ? g.nredv : g.nred, c->tot);
  if (NQ == 1 && threadIdx.x < S) c->tot[S + threadIdx.x] = 0.0;
  __syncthreads();
  finalize<S>(c, op, arg);
}

// Per-group active counts summed into one word the host polls.
__global__ void kb_count(BatchDev bd, int ngroups, int32_t* out) {
  __shared__ int32_t red[256];
  int32_t a = 0;
  for (int g = threadIdx.x; g < ngroups; g += blockDim.x) a += bd.groups[g].ctl->n_active;
  red[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

template <int S>
__global__ __launch_bounds__(256) void kb_diag_inv(BatchDev bd, int ngroups) {
  // grid-stride over all groups' (row, sample) pairs, one group at a time
  for (int gi = 0; gi < ngroups; ++gi) {
    const GroupDev& g = bd.groups[gi];
    const int64_t total = (int64_t)g.n * S;
    for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x; t0 < total; t0 += (int64_t)gridDim.x * blockDim.x)
      diag_inv_body<double, S>(g.n, g.rp, g.ci, g.vals, g.dinv, t0 / blockDim.x);
  }
}

template <int S>
__global__ __launch_bounds__(256) void kb_zero_where(BatchDev bd, int ngroups) {
  for (int gi = 0; gi < ngroups; ++gi) {
    const GroupDev& g = bd.groups[gi];
    zero_where_body<S>((int64_t)g.n * S, g.x, g.ctl, (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                       (int64_t)gridDim.x * blockDim.x);
  }
}

static __global__ void kb_ctl_init(BatchDev bd, int ngroups, double rtol, int max_iter) {
  for (int gi = blockIdx.x; gi < ngroups; gi += gridDim.x) {
    Ctl* c = bd.groups[gi].ctl;
    if (threadIdx.x == 0) {
      c->rtol = rtol;
      c->inner_rtol = 0.0;
      c->max_iter = max_iter;
      c->inner_max_iter = max_iter;
      c->max_outer = 0;
      c->mixed = 0;
      c->coupled = 0;
      c->xnz = 1;
      c->n_active = 0;
      c->n_oactive = 0;
    }
    if (threadIdx.x < kMaxS) {
      const int e = threadIdx.x;
      c->active[e] = 0;
      c->oactive[e] = 0;
      c->iters[e] = 0;
      c->oiters[e] = 0;
      c->kiter[e] = 0;
      c->status[e] = ENS_SAMPLE_MAXITER;
      c->zero_b[e] = 0;
      c->rel_res[e] = 0.0;
    }
  }
}

// ------------------------------------------------------------ host side ---

static size_t r256(size_t b) { return (b + 255) & ~(size_t)255; }

template <int S, int NW>
struct Plan {
  static constexpr int RB = NW * EnsMap<double, S>::RPW;  // rows per row tile
  static constexpr int VB = kBlock * kU;                  // chunks per vector block
};

struct Layout {
  std::vector<GroupDev> g;
  std::vector<int32_t> row_grp, vec_grp, red_grp, redv_grp;
  int64_t row_blocks = 0, vec_blocks = 0, red_rows = 0, redv_rows = 0;
  size_t bytes = 0;
  size_t off_groups, off_tables, off_part, off_out1, off_ctl, off_vec, off_count;
};

template <int S, int NW>
static ens_status plan(const ens_group* groups, int ng, Layout& L) {
  using PL = Plan<S, NW>;
  L.g.resize(ng);
  L.row_blocks = L.vec_blocks = L.red_rows = L.redv_rows = 0;
  size_t vec_bytes = 0;
  for (int i = 0; i < ng; ++i) {
    const ens_group& gr = groups[i];
    ENS_ARG_CHECK(gr.graph && gr.values && gr.b && gr.x && gr.stats, "null group pointer");
    ENS_ARG_CHECK(gr.graph->n > 0 && gr.graph->row_ptr && gr.graph->col_idx, "empty group graph");
    ENS_ARG_CHECK(aligned16(gr.values) && aligned16(gr.b) && aligned16(gr.x), "group buffers must be 16-byte aligned");
    GroupDev& d = L.g[i];
    memset(&d, 0, sizeof(d));
    d.n = gr.graph->n;
    d.nnz = gr.graph->nnz;
    d.rp = gr.graph->row_ptr;
    d.ci = gr.graph->col_idx;
    d.vals = gr.values;
    d.b = gr.b;
    d.x = gr.x;
    d.nrowb = (d.n + PL::RB - 1) / PL::RB;
    const int64_t nchunks = (int64_t)d.n * S / VecMap<double, S>::V;
    d.nvecb = (nchunks + PL::VB - 1) / PL::VB;
    d.row0 = L.row_blocks;
    d.vec0 = L.vec_blocks;
    L.row_blocks += d.nrowb;
    L.vec_blocks += d.nvecb;
    d.nred = (int32_t)((d.nrowb + kSegRows - 1) / kSegRows);
    d.nredv = (int32_t)((d.nvecb + kSegRows - 1) / kSegRows);
    d.red0 = L.red_rows;
    d.redv0 = L.redv_rows;
    L.red_rows += d.nred;
    L.redv_rows += d.nredv;
    vec_bytes += 4 * r256((size_t)d.n * S * sizeof(double));
  }
  L.row_grp.resize(L.row_blocks);
  L.vec_grp.resize(L.vec_blocks);
  L.red_grp.resize(L.red_rows);
  L.redv_grp.resize(L.redv_rows);
  for (int i = 0; i < ng; ++i) {
    const GroupDev& d = L.g[i];
    for (int64_t b = 0; b < d.nrowb; ++b) L.row_grp[d.row0 + b] = i;
    for (int64_t b = 0; b < d.nvecb; ++b) L.vec_grp[d.vec0 + b] = i;
    for (int64_t b = 0; b < d.nred; ++b) L.red_grp[d.red0 + b] = i;
    for (int64_t b = 0; b < d.nredv; ++b) L.redv_grp[d.redv0 + b] = i;
  }
  size_t off = 0;
  L.off_groups = off;
  off += r256(sizeof(GroupDev) * ng);
  L.off_tables = off;
  off += r256(sizeof(int32_t) * (L.row_blocks + L.vec_blocks + L.red_rows + L.redv_rows));
  L.off_part = off;
  off += r256(sizeof(double) * 2 * S * (size_t)(L.row_blocks > L.vec_blocks ? L.row_blocks : L.vec_blocks));
  L.off_out1 = off;
  off += r256(sizeof(double) * 2 * S * (size_t)(L.red_rows > L.redv_rows ? L.red_rows : L.redv_rows));
  L.off_ctl = off;
  off += r256(sizeof(Ctl) * ng);
  L.off_count = off;
  off += 256;
  L.off_vec = off;
  off += vec_bytes;
  L.bytes = off;
  return ENS_OK;
}

static BatchDev bind(Layout& L, char* ws, int ng, int S) {
  BatchDev bd;
  int32_t* tables = (int32_t*)(ws + L.off_tables);
  bd.groups = (const GroupDev*)(ws + L.off_groups);
  bd.row_grp = tables;
  bd.vec_grp = tables + L.row_blocks;
  bd.red_grp = tables + L.row_blocks + L.vec_blocks;
  bd.redv_grp = tables + L.row_blocks + L.vec_blocks + L.red_rows;
  bd.part = (double*)(ws + L.off_part);
  bd.out1 = (double*)(ws + L.off_out1);
  char* vp = ws + L.off_vec;
  Ctl* ctl = (Ctl*)(ws + L.off_ctl);
  for (int i = 0; i < ng; ++i) {
    GroupDev& d = L.g[i];
    const size_t vb = r256((size_t)d.n * S * sizeof(double));
    d.r = (double*)vp;
    d.p = (double*)(vp + vb);
    d.q = (double*)(vp + 2 * vb);
    d.dinv = (double*)(vp + 3 * vb);
    vp += 4 * vb;
    d.ctl = ctl + i;
  }
  return bd;
}

template <int S, int NW>
static void batch_iteration(const BatchDev& bd, const Layout& L, int ng, hipStream_t st) {
  hipLaunchKernelGGL((kb_spmv_dot<S, NW>), dim3((unsigned)L.row_blocks), dim3(NW * 64), 0, st, bd);
  hipLaunchKernelGGL((kb_stage1<S, 0>), dim3((unsigned)L.red_rows), dim3(256), 0, st, bd, 1);
  hipLaunchKernelGGL((kb_final<S, 1, 0>), dim3((unsigned)ng), dim3(256), 0, st, bd, (int)OP_ALPHA, 0, 1);
  hipLaunchKernelGGL(kb_update<S>, dim3((unsigned)L.vec_blocks), dim3(256), 0, st, bd);
  hipLaunchKernelGGL((kb_stage1<2 * S, 1>), dim3((unsigned)L.redv_rows), dim3(256), 0, st, bd, 1);
  hipLaunchKernelGGL((kb_final<S, 2, 1>), dim3((unsigned)ng), dim3(256), 0, st, bd, (int)OP_UPDATE, 0, 1);
  hipLaunchKernelGGL(kb_pupdate<S>, dim3((unsigned)L.vec_blocks), dim3(256), 0, st, bd);
}

static ens_status poll(int32_t* dev_count, hipStream_t st, int32_t* out) {
  DeviceCtx* cx = device_ctx();
  if (!cx) {
    set_error("device context unavailable");
    return ENS_E_HIP;
  }
  ENS_HIP_TRY(hipMemcpyAsync(cx->host_flag, dev_count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  ENS_HIP_TRY(hipStreamSynchronize(st));
  *out = *cx->host_flag;
  return ENS_OK;
}

// Optional first work of a batch solve, enqueued on the solve's stream
// before the CG set-up (the assembly of ens_assemble_solve_batch).
struct Prologue {
  const AsmGroupDev* groups = nullptr;  // device
  const int32_t* blk_grp = nullptr;     // device
  int64_t blocks = 0;
  const ens_problem* prob = nullptr;
};

// The CG set-up of all groups: control blocks, D^-1, r = b - A x and its
// norms, x zeroed where b is, the first direction and rho.
template <int S, int NW>
static void batch_setup(const BatchDev& bd, const Layout& L, int ng, double rtol, int max_iter, hipStream_t st) {
  hipLaunchKernelGGL(kb_ctl_init, dim3((unsigned)(ng < 1024 ? ng : 1024)), dim3(64), 0, st, bd, ng, rtol, max_iter);
  hipLaunchKernelGGL(kb_diag_inv<S>, dim3(2048), dim3(256), 0, st, bd, ng);
  hipLaunchKernelGGL((kb_residual<S, NW>), dim3((unsigned)L.row_blocks), dim3(NW * 64), 0, st, bd, 1);
  hipLaunchKernelGGL((kb_stage1<2 * S, 0>), dim3((unsigned)L.red_rows), dim3(256), 0, st, bd, 0);
  hipLaunchKernelGGL((kb_final<S, 2, 0>), dim3((unsigned)ng), dim3(256), 0, st, bd, (int)OP_START, 0, 0);
  hipLaunchKernelGGL(kb_zero_where<S>, dim3(1024), dim3(256), 0, st, bd, ng);
  hipLaunchKernelGGL(kb_cg_start<S>, dim3((unsigned)L.vec_blocks), dim3(256), 0, st, bd);
  hipLaunchKernelGGL((kb_stage1<2 * S, 1>), dim3((unsigned)L.redv_rows), dim3(256), 0, st, bd, 0);
  hipLaunchKernelGGL((kb_final<S, 2, 1>), dim3((unsigned)ng), dim3(256), 0, st, bd, (int)OP_RHO, 0, 0);
}

// Capture `enqueue` on st into an executable graph.
template <typename F>
static ens_status capture(hipStream_t st, F&& enqueue, hipGraph_t* graph, hipGraphExec_t* exec) {
  ENS_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  ens_status rc = enqueue();
  hipError_t e1 = hipGetLastError();
  hipError_t e2 = hipStreamEndCapture(st, graph);
  if (rc != ENS_OK || e1 != hipSuccess || e2 != hipSuccess) {
    if (*graph) (void)hipGraphDestroy(*graph);
    *graph = nullptr;
    if (rc == ENS_OK) set_error("graph capture failed: %s / %s", hipGetErrorString(e1), hipGetErrorString(e2));
    return rc != ENS_OK ? rc : ENS_E_HIP;
  }
  hipError_t e3 = hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0);
  if (e3 != hipSuccess) {
    (void)hipGraphDestroy(*graph);
    *graph = nullptr;
    set_error("graph instantiation failed: %s", hipGetErrorString(e3));
    return ENS_E_HIP;
  }
  return ENS_OK;
}

template <int S, int NW>
static ens_status solve_batch(const ens_group* groups, int ng, const ens_batch_opts& o, void* ws, size_t ws_bytes,
                              hipStream_t user, const Prologue* pro = nullptr) {
  Layout L;
  ens_status rc = plan<S, NW>(groups, ng, L);
  if (rc != ENS_OK) return rc;
  if (ws_bytes < L.bytes) {
    set_error("batch workspace of %zu bytes is smaller than the %zu required", ws_bytes, L.bytes);
    return ENS_E_NOMEM;
  }
  char* w = (char*)ws;
  BatchDev bd = bind(L, w, ng, S);
  int32_t* dcount = (int32_t*)(w + L.off_count);
  DeviceCtx* cx = device_ctx();
  if (!cx) {
    set_error("device context unavailable");
    return ENS_E_HIP;
  }
  // all work runs on the library's own stream, ordered after and before the
  // caller's stream by events (graph capture needs a non-default stream)
  hipStream_t st = cx->work_stream;
  ENS_HIP_TRY(hipEventRecord(cx->ev_in, user));
  ENS_HIP_TRY(hipStreamWaitEvent(st, cx->ev_in, 0));
  ENS_HIP_TRY(hipMemcpyAsync(w + L.off_groups, L.g.data(), sizeof(GroupDev) * ng, hipMemcpyHostToDevice, st));
  std::vector<int32_t> tables;
  tables.insert(tables.end(), L.row_grp.begin(), L.row_grp.end());
  tables.insert(tables.end(), L.vec_grp.begin(), L.vec_grp.end());
  tables.insert(tables.end(), L.red_grp.begin(), L.red_grp.end());
  tables.insert(tables.end(), L.redv_grp.begin(), L.redv_grp.end());
  ENS_HIP_TRY(hipMemcpyAsync(w + L.off_tables, tables.data(), sizeof(int32_t) * tables.size(),
                             hipMemcpyHostToDevice, st));
  const int max_iter = o.max_iter > 0 ? o.max_iter : 10000;
  const int chunk = o.check_every > 0 ? o.check_every : 16;
  // first: [assembly,] set-up, one chunk of iterations, the active count;
  // then: one chunk and the count, repeated until no sample is active
  auto first = [&]() -> ens_status {
    if (pro) {
      ens_status r2 = batch_assemble_launch(S, pro->groups, pro->blk_grp, pro->blocks, *pro->prob, st);
      if (r2 != ENS_OK) return r2;
    }
    batch_setup<S, NW>(bd, L, ng, o.rtol, max_iter, st);
    for (int k = 0; k < chunk; ++k) batch_iteration<S, NW>(bd, L, ng, st);
    hipLaunchKernelGGL(kb_count, dim3(1), dim3(256), 0, st, bd, ng, dcount);
    return ENS_OK;
  };
  auto next = [&]() -> ens_status {
    for (int k = 0; k < chunk; ++k) batch_iteration<S, NW>(bd, L, ng, st);
    hipLaunchKernelGGL(kb_count, dim3(1), dim3(256), 0, st, bd, ng, dcount);
    return ENS_OK;
  };
  hipGraph_t g_first = nullptr, g_next = nullptr;
  hipGraphExec_t x_first = nullptr, x_next = nullptr;
  auto release = [&]() {
    if (x_first) (void)hipGraphExecDestroy(x_first);
    if (g_first) (void)hipGraphDestroy(g_first);
    if (x_next) (void)hipGraphExecDestroy(x_next);
    if (g_next) (void)hipGraphDestroy(g_next);
  };
  if (o.use_graph) {
    rc = capture(st, first, &g_first, &x_first);
    if (rc == ENS_OK) rc = capture(st, next, &g_next, &x_next);
    if (rc != ENS_OK) {
      release();
      return rc;
    }
  }
  ens_status out = ENS_OK;
  for (int k0 = 0; k0 < max_iter; k0 += chunk) {
    if (o.use_graph) {
      hipError_t e = hipGraphLaunch(k0 == 0 ? x_first : x_next, st);
      if (e != hipSuccess) {
        set_error("graph launch failed: %s", hipGetErrorString(e));
        out = ENS_E_HIP;
        break;
      }
    } else {
      out = k0 == 0 ? first() : next();
      hipError_t e = hipGetLastError();
      if (out == ENS_OK && e != hipSuccess) {
        set_error("launch failed: %s", hipGetErrorString(e));
        out = ENS_E_HIP;
      }
      if (out != ENS_OK) break;
    }
    int32_t act = 0;
    out = poll(dcount, st, &act);
    if (out != ENS_OK || act == 0) break;
  }
  release();
  if (out != ENS_OK) return out;
  // true residuals
  hipLaunchKernelGGL((kb_residual<S, NW>), dim3((unsigned)L.row_blocks), dim3(NW * 64), 0, st, bd, 0);
  hipLaunchKernelGGL((kb_stage1<2 * S, 0>), dim3((unsigned)L.red_rows), dim3(256), 0, st, bd, 0);
  hipLaunchKernelGGL((kb_final<S, 2, 0>), dim3((unsigned)ng), dim3(256), 0, st, bd, (int)OP_TRUE, 0, 0);
  ENS_LAUNCH_CHECK();
  std::vector<Ctl> h(ng);
  ENS_HIP_TRY(hipMemcpyAsync(h.data(), w + L.off_ctl, sizeof(Ctl) * ng, hipMemcpyDeviceToHost, st));
  ENS_HIP_TRY(hipStreamSynchronize(st));
  ENS_HIP_TRY(hipEventRecord(cx->ev_out, st));
  ENS_HIP_TRY(hipStreamWaitEvent(user, cx->ev_out, 0));
  ens_status agg = ENS_OK;
  for (int i = 0; i < ng; ++i)
    for (int e = 0; e < S; ++e) {
      ens_cg_stat& s = groups[i].stats[e];
      s.iters = h[i].iters[e];
      s.outer_iters = 0;
      s.status = h[i].status[e];
      s.compacted = 0;
      s.rel_res = h[i].rel_res[e];
      if (s.status != ENS_SAMPLE_CONVERGED) agg = ENS_W_NOT_CONVERGED;
    }
  return agg;
}

// ens_assemble_solve_batch: the groups' assembly descriptors and the
// workgroup -> group table of the flat assembly launch follow the solver's
// workspace; need != nullptr: sizes only.
template <int S, int NW>
static ens_status assemble_solve(const ens_group* groups, const ens_group_input* in, int ng, const ens_problem& prob,
                                 const ens_batch_opts& o, void* ws, size_t ws_bytes, hipStream_t user, size_t* need) {
  Layout L;
  ens_status rc = plan<S, NW>(groups, ng, L);
  if (rc != ENS_OK) return rc;
  std::vector<AsmGroupDev> ag(ng);
  std::vector<int32_t> bg;
  int64_t blocks = 0;
  for (int i = 0; i < ng; ++i) {
    ENS_ARG_CHECK(in[i].kl && in[i].xi, "null assembly input");
    int64_t n = 0, nnz = 0;
    rc = ens_mesh_sizes(in[i].N, &n, &nnz, nullptr);
    if (rc != ENS_OK) return rc;
    ENS_ARG_CHECK(groups[i].graph->n == n && groups[i].graph->nnz == nnz, "group graph is not its mesh's graph");
    AsmGroupDev& d = ag[i];
    d.N = in[i].N;
    d.tile0 = blocks;
    kl_parts(in[i].kl, prob.M, &d.sq, &d.tr, &d.phi);
    d.xi = in[i].xi;
    d.rp = groups[i].graph->row_ptr;
    d.values = const_cast<double*>(groups[i].values);
    d.rhs = const_cast<double*>(groups[i].b);
    d.x = groups[i].x;
    const int64_t t = asm_tiles(in[i].N, S);
    bg.insert(bg.end(), (size_t)t, i);
    blocks += t;
  }
  const size_t off_ag = r256(L.bytes), off_bg = off_ag + r256(sizeof(AsmGroupDev) * ng);
  const size_t total = off_bg + r256(sizeof(int32_t) * (size_t)blocks);
  if (need) {
    *need = total;
    return ENS_OK;
  }
  if (ws_bytes < total) {
    set_error("batch workspace of %zu bytes is smaller than the %zu required", ws_bytes, total);
    return ENS_E_NOMEM;
  }
  char* w = (char*)ws;
  ENS_HIP_TRY(hipMemcpyAsync(w + off_ag, ag.data(), sizeof(AsmGroupDev) * ng, hipMemcpyHostToDevice, user));
  ENS_HIP_TRY(hipMemcpyAsync(w + off_bg, bg.data(), sizeof(int32_t) * bg.size(), hipMemcpyHostToDevice, user));
  Prologue pro;
  pro.groups = (const AsmGroupDev*)(w + off_ag);
  pro.blk_grp = (const int32_t*)(w + off_bg);
  pro.blocks = blocks;
  pro.prob = &prob;
  // the host tables stay alive until solve_batch has synchronised
  return solve_batch<S, NW>(groups, ng, o, ws, ws_bytes, user, &pro);
}

static bool tile_ok(int t) { return t == 2 || t == 4 || t == 8; }

template <int S>
static ens_status dispatch_tile(const ens_group* g, int ng, const ens_batch_opts& o, void* ws, size_t b,
                                hipStream_t st, size_t* need) {
  Layout L;
  ens_status rc;
  switch (o.tile) {
    case 2: rc = need ? plan<S, 2>(g, ng, L) : solve_batch<S, 2>(g, ng, o, ws, b, st); break;
    case 4: rc = need ? plan<S, 4>(g, ng, L) : solve_batch<S, 4>(g, ng, o, ws, b, st); break;
    default: rc = need ? plan<S, 8>(g, ng, L) : solve_batch<S, 8>(g, ng, o, ws, b, st); break;
  }
  if (need && rc == ENS_OK) *need = L.bytes;
  return rc;
}

static ens_status dispatch(const ens_group* g, int ng, int32_t s, const ens_batch_opts& o, void* ws, size_t b,
                           hipStream_t st, size_t* need) {
  switch (s) {
    case 8: return dispatch_tile<8>(g, ng, o, ws, b, st, need);
    case 16: return dispatch_tile<16>(g, ng, o, ws, b, st, need);
    case 32: return dispatch_tile<32>(g, ng, o, ws, b, st, need);
    default: set_error("batch ensemble size %d not compiled in (8, 16, 32)", s); return ENS_E_UNSUPPORTED;
  }
}

template <int S>
static ens_status dispatch_asm_tile(const ens_group* g, const ens_group_input* in, int ng, const ens_problem& pr,
                                    const ens_batch_opts& o, void* ws, size_t b, hipStream_t st, size_t* need) {
  switch (o.tile) {
    case 2: return assemble_solve<S, 2>(g, in, ng, pr, o, ws, b, st, need);
    case 4: return assemble_solve<S, 4>(g, in, ng, pr, o, ws, b, st, need);
    default: return assemble_solve<S, 8>(g, in, ng, pr, o, ws, b, st, need);
  }
}

static ens_status dispatch_asm(const ens_group* g, const ens_group_input* in, int ng, int32_t s,
                               const ens_problem& pr, const ens_batch_opts& o, void* ws, size_t b, hipStream_t st,
                               size_t* need) {
  switch (s) {
    case 8: return dispatch_asm_tile<8>(g, in, ng, pr, o, ws, b, st, need);
    case 16: return dispatch_asm_tile<16>(g, in, ng, pr, o, ws, b, st, need);
    case 32: return dispatch_asm_tile<32>(g, in, ng, pr, o, ws, b, st, need);
    default: set_error("batch ensemble size %d not compiled in (8, 16, 32)", s); return ENS_E_UNSUPPORTED;
  }
}

}  // namespace ens

using namespace ens;

extern "C" {

ens_status ens_assemble_solve_batch_workspace_bytes(const ens_group* groups, const ens_group_input* inputs,
                                                    int32_t n_groups, int32_t s, const ens_problem* problem,
                                                    const ens_batch_opts* opts, size_t* bytes) {
  ENS_ARG_CHECK(groups && inputs && n_groups >= 1 && problem && opts && bytes, "bad batch arguments");
  ENS_ARG_CHECK(tile_ok(opts->tile), "tile must be 2, 4 or 8 wavefronts");
  ENS_ARG_CHECK(problem->M >= 0 && problem->M <= 16, "problem->M out of range");
  return dispatch_asm(groups, inputs, n_groups, s, *problem, *opts, nullptr, 0, nullptr, bytes);
}

ens_status ens_assemble_solve_batch(const ens_group* groups, const ens_group_input* inputs, int32_t n_groups,
                                    int32_t s, const ens_problem* problem, const ens_batch_opts* opts,
                                    void* workspace, size_t ws_bytes, hipStream_t stream) {
  ENS_ARG_CHECK(groups && inputs && n_groups >= 1 && problem && opts && workspace, "bad batch arguments");
  ENS_ARG_CHECK(((uintptr_t)workspace & 255u) == 0, "workspace must be 256-byte aligned");
  ENS_ARG_CHECK(tile_ok(opts->tile), "tile must be 2, 4 or 8 wavefronts");
  ENS_ARG_CHECK(opts->rtol >= 0.0, "rtol must be >= 0");
  ENS_ARG_CHECK(problem->M >= 0 && problem->M <= 16, "problem->M out of range");
  return dispatch_asm(groups, inputs, n_groups, s, *problem, *opts, workspace, ws_bytes, stream, nullptr);
}

ens_status ens_batch_workspace_bytes(const ens_group* groups, int32_t n_groups, int32_t s, const ens_batch_opts* opts,
                                     size_t* bytes) {
  ENS_ARG_CHECK(groups && n_groups >= 1 && opts && bytes, "bad batch arguments");
  ENS_ARG_CHECK(tile_ok(opts->tile), "tile must be 2, 4 or 8 wavefronts");
  return dispatch(groups, n_groups, s, *opts, nullptr, 0, nullptr, bytes);
}

ens_status ens_solve_batch(const ens_group* groups, int32_t n_groups, int32_t s, const ens_batch_opts* opts,
                           void* workspace, size_t ws_bytes, hipStream_t stream) {
  ENS_ARG_CHECK(groups && n_groups >= 1 && opts && workspace, "bad batch arguments");
  ENS_ARG_CHECK(((uintptr_t)workspace & 255u) == 0, "workspace must be 256-byte aligned");
  ENS_ARG_CHECK(tile_ok(opts->tile), "tile must be 2, 4 or 8 wavefronts");
  ENS_ARG_CHECK(opts->rtol >= 0.0, "rtol must be >= 0");
  return dispatch(groups, n_groups, s, *opts, workspace, ws_bytes, stream, nullptr);
}

}  // extern "C"

// ------------------------------------------------------------- autotuner ---

namespace ens {

static std::string tune_key(const int32_t* meshes, int nm, const ens_problem& pr, const ens_batch_opts& o) {
  char buf[160];
  std::string k = "gfx950:N";
  for (int i = 0; i < nm; ++i) k += "_" + std::to_string(meshes[i]);
  snprintf(buf, sizeof(buf), ":M%d:sig%.4g:L%.4g:rtol%.3g:ce%d", pr.M, pr.sigma, pr.L, o.rtol, o.check_every);
  return k + buf;
}

static bool cache_lookup(const char* path, const std::string& key, int* s, int* tile) {
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char kb[512];
  int a = 0, b = 0;
  bool found = false;
  while (fscanf(f, "%511s %d %d", kb, &a, &b) == 3)
    if (key == kb) {  // the last entry for a key wins
      *s = a;
      *tile = b;
      found = true;
    }
  fclose(f);
  return found;
}

static void cache_store(const char* path, const std::string& key, int s, int tile) {
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d %d\n", key.c_str(), s, tile);
  fclose(f);
}

// Trial buffers of one mesh: graph, KL table, and 32 samples' values, b and
// x, carved into 32/s groups of s samples for a candidate s.
struct TrialMesh {
  int N = 0;
  int64_t n = 0, nnz = 0;
  int32_t *rp = nullptr, *ci = nullptr;
  void* kl = nullptr;
  double *xi = nullptr, *vals = nullptr, *b = nullptr, *x = nullptr;
  ens_graph g{};
};

constexpr int kTrial = 32;  // samples per mesh in every trial

// The autotuner's caller-owned workspace: each mesh's trial buffers at
// 256-byte aligned offsets from `base`, then the largest batch-solver
// workspace any candidate needs.  With base == nullptr only the sizes are
// formed (the solver's need depends on the shapes alone, so its plan runs
// on the offsets themselves).
static ens_status tune_layout(char* base, const int32_t* meshes, int nm, const ens_problem& pr,
                              const int32_t* s_cand, int ns, const int32_t* tile_cand, int nt,
                              const ens_batch_opts& o0, std::vector<TrialMesh>& t, char** ws, size_t* ws_need,
                              size_t* total) {
  // a non-null stand-in address keeps the plan's pointer checks meaningful
  // when only sizes are wanted; nothing is dereferenced then
  char* b0 = base ? base : (char*)(uintptr_t)256;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = b0 + off;
    off += r256(bytes);
    return p;
  };
  const int M = pr.M;
  t.assign(nm, TrialMesh{});
  for (int i = 0; i < nm; ++i) {
    TrialMesh& m = t[i];
    m.N = meshes[i];
    ens_status rc = ens_mesh_sizes(m.N, &m.n, &m.nnz, nullptr);
    if (rc != ENS_OK) return rc;
    size_t klb = 0;
    rc = ens_kl_bytes(m.N, M, &klb);
    if (rc != ENS_OK) return rc;
    m.rp = (int32_t*)take(sizeof(int32_t) * (m.n + 1));
    m.ci = (int32_t*)take(sizeof(int32_t) * m.nnz);
    m.kl = take(klb);
    m.xi = (double*)take(sizeof(double) * kTrial * (M > 0 ? M : 1));
    m.vals = (double*)take(sizeof(double) * kTrial * m.nnz);
    m.b = (double*)take(sizeof(double) * kTrial * m.n);
    m.x = (double*)take(sizeof(double) * kTrial * m.n);
    m.g = ens_graph{(int32_t)m.n, m.nnz, m.rp, m.ci};
  }
  size_t need = 0;
  std::vector<ens_cg_stat> stats((size_t)kTrial);
  for (int a = 0; a < ns; ++a) {
    const int s = s_cand[a];
    std::vector<ens_group> gr;
    for (int i = 0; i < nm; ++i)
      for (int j = 0; j < kTrial / s; ++j)
        gr.push_back(ens_group{&t[i].g, t[i].vals, t[i].b, t[i].x, stats.data()});
    for (int c = 0; c < nt; ++c) {
      ens_batch_opts o = o0;
      o.tile = tile_cand[c];
      size_t nb = 0;
      ens_status rc = ens_batch_workspace_bytes(gr.data(), (int)gr.size(), s, &o, &nb);
      if (rc != ENS_OK) return rc;
      need = nb > need ? nb : need;
    }
  }
  *ws = take(need);
  *ws_need = need;
  *total = off;
  return ENS_OK;
}

static ens_status tune_check(const int32_t* meshes, int32_t nm, const ens_problem* prob, const int32_t* s_cand,
                             int32_t ns, const int32_t* tile_cand, int32_t nt, const ens_batch_opts* base) {
  ENS_ARG_CHECK(meshes && nm >= 1 && prob && s_cand && ns >= 1 && tile_cand && nt >= 1 && base, "bad arguments");
  ENS_ARG_CHECK(base->rtol >= 0.0, "rtol must be >= 0");
  for (int i = 0; i < nm; ++i) ENS_ARG_CHECK(meshes[i] >= 1, "mesh sizes must be >= 1");
  for (int i = 0; i < ns; ++i)
    if (s_cand[i] != 8 && s_cand[i] != 16 && s_cand[i] != 32) {
      set_error("candidate ensemble size %d not compiled in (8, 16, 32)", s_cand[i]);
      return ENS_E_UNSUPPORTED;
    }
  for (int i = 0; i < nt; ++i) ENS_ARG_CHECK(tile_ok(tile_cand[i]), "tile must be 2, 4 or 8");
  return ENS_OK;
}

}  // namespace ens

extern "C" ens_status ens_batch_autotune_workspace_bytes(const int32_t* meshes, int32_t nm,
                                                         const ens_problem* prob, const int32_t* s_cand,
                                                         int32_t ns, const int32_t* tile_cand, int32_t nt,
                                                         const ens_batch_opts* base, size_t* bytes) {
  ENS_ARG_CHECK(bytes, "bad arguments");
  ens_status rc = tune_check(meshes, nm, prob, s_cand, ns, tile_cand, nt, base);
  if (rc != ENS_OK) return rc;
  std::vector<TrialMesh> t;
  char* ws = nullptr;
  size_t need = 0;
  return tune_layout(nullptr, meshes, nm, *prob, s_cand, ns, tile_cand, nt, *base, t, &ws, &need, bytes);
}

extern "C" ens_status ens_batch_autotune(const int32_t* meshes, int32_t nm, const ens_problem* prob,
                                         const double* xi_host, const int32_t* s_cand, int32_t ns,
                                         const int32_t* tile_cand, int32_t nt, const ens_batch_opts* base,
                                         const char* cache_path, int32_t* best_s, int32_t* best_tile,
                                         double* scores, void* workspace, size_t ws_bytes, hipStream_t stream) {
  ens_status rc = tune_check(meshes, nm, prob, s_cand, ns, tile_cand, nt, base);
  if (rc != ENS_OK) return rc;
  ENS_ARG_CHECK(xi_host && best_s && best_tile, "bad arguments");
  const std::string key = tune_key(meshes, nm, *prob, *base);
  int cs = 0, ct = 0;
  if (!scores && cache_lookup(cache_path, key, &cs, &ct)) {
    *best_s = cs;
    *best_tile = ct;
    return ENS_OK;
  }
  ENS_ARG_CHECK(workspace, "the trials need a workspace (ens_batch_autotune_workspace_bytes)");
  ENS_ARG_CHECK(((uintptr_t)workspace & 255u) == 0, "workspace must be 256-byte aligned");
  const int M = prob->M;
  std::vector<TrialMesh> t;
  char* ws = nullptr;
  size_t ws_need = 0, total = 0;
  rc = tune_layout((char*)workspace, meshes, nm, *prob, s_cand, ns, tile_cand, nt, *base, t, &ws, &ws_need, &total);
  if (rc != ENS_OK) return rc;
  if (ws_bytes < total) {
    set_error("autotune workspace too small: %zu < %zu bytes", ws_bytes, total);
    return ENS_E_ARG;
  }
  std::vector<ens_cg_stat> stats((size_t)nm * kTrial);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double best = -1.0;
#define TUNE_TRY(expr)                                             \
  do {                                                             \
    hipError_t _e = (expr);                                        \
    if (_e != hipSuccess) {                                        \
      set_error("autotune: %s: %s", #expr, hipGetErrorString(_e)); \
      rc = ENS_E_HIP;                                              \
      goto done;                                                   \
    }                                                              \
  } while (0)
  TUNE_TRY(hipEventCreate(&e0));
  TUNE_TRY(hipEventCreate(&e1));
  for (int i = 0; i < nm; ++i) {
    TrialMesh& m = t[i];
    if (M > 0)
      TUNE_TRY(hipMemcpyAsync(m.xi, xi_host + (size_t)i * kTrial * M, sizeof(double) * kTrial * M,
                              hipMemcpyHostToDevice, stream));
    rc = ens_graph_build(m.N, m.rp, m.ci, stream);
    if (rc == ENS_OK) rc = ens_kl_build(m.N, M, prob->L, m.kl, stream);
    if (rc != ENS_OK) goto done;
  }
  for (int a = 0; a < ns; ++a) {
    const int s = s_cand[a];
    const int per = kTrial / s;  // groups per mesh
    std::vector<ens_group> gr;
    for (int i = 0; i < nm; ++i)
      for (int j = 0; j < per; ++j) {
        TrialMesh& m = t[i];
        double* v = m.vals + (size_t)j * s * m.nnz;
        double* b = m.b + (size_t)j * s * m.n;
        double* x = m.x + (size_t)j * s * m.n;
        rc = ens_assemble(m.N, &m.g, m.kl, prob, s, m.xi + (size_t)j * s * M, v, nullptr, b, stream);
        if (rc != ENS_OK) goto done;
        gr.push_back(ens_group{&m.g, v, b, x, stats.data() + ((size_t)i * kTrial + (size_t)j * s)});
      }
    for (int c = 0; c < nt; ++c) {
      ens_batch_opts o = *base;
      o.tile = tile_cand[c];
      float ms = 0.f;
      const int reps = (a == 0 && c == 0) ? 2 : 1;  // the very first solve also warms up
      for (int rep = 0; rep < reps; ++rep) {
        for (int i = 0; i < nm; ++i) TUNE_TRY(hipMemsetAsync(t[i].x, 0, sizeof(double) * kTrial * t[i].n, stream));
        TUNE_TRY(hipEventRecord(e0, stream));
        rc = ens_solve_batch(gr.data(), (int)gr.size(), s, &o, ws, ws_need, stream);
        if (rc != ENS_OK && rc != ENS_W_NOT_CONVERGED) goto done;
        TUNE_TRY(hipEventRecord(e1, stream));
        TUNE_TRY(hipEventSynchronize(e1));
        TUNE_TRY(hipEventElapsedTime(&ms, e0, e1));
      }
      rc = ENS_OK;
      const double score = (double)nm * kTrial / (ms * 1e-3);  // solved samples per second
      if (scores) scores[a * nt + c] = score;
      if (score > best) {
        best = score;
        *best_s = s;
        *best_tile = tile_cand[c];
      }
    }
  }
  cache_store(cache_path, key, *best_s, *best_tile);
done:
#undef TUNE_TRY
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc != ENS_OK) (void)hipStreamSynchronize(stream);  // no trial work left in flight on the caller's buffer
  return rc;
}
