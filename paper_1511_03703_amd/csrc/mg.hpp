// Geometric multigrid hierarchy of the ensemble Q1 problem (Sec. 3.5,
// Alg. vcycle): the nested meshes N, N/2, ... (halved while even and above
// 4), each level's ensemble matrix assembled on its own mesh with the
// samples' KL coefficients, trilinear prolongation onto interior nodes with
// its transpose as restriction, order-2 Chebyshev smoothing in D^-1 A on
// [lmax/4, lmax] per sample (lmax the Gershgorin bound), and an exact
// solve of the coarsest interior block (per-sample dense inverse).
#pragma once

#include "common.hpp"

namespace ens {

struct Ctl;

constexpr int kMgMaxLevels = 16;
constexpr double kMgRatio = 4.0;
constexpr int64_t kMgMaxCoarse = 512;  // interior unknowns of the coarsest level

struct MgLevel {
  int N = 0;
  int64_t n = 0, nnz = 0;
  const int32_t* rp = nullptr;  // level 0: the caller's graph
  const int32_t* ci = nullptr;
  const double* vals = nullptr;   // FP64 matrix (level 0: the caller's)
  const float* vals32 = nullptr;  // FP32 matrix of an FP32 cycle (level 0: the caller's)
  int32_t *own_rp = nullptr, *own_ci = nullptr;
  double* own_vals = nullptr;
  float* own_vals32 = nullptr;
  void* kl = nullptr;
  void* dinv = nullptr;  // cycle precision
  double* lmax = nullptr;
  void *b = nullptr, *xa = nullptr, *xb = nullptr, *r = nullptr, *d = nullptr;  // cycle precision
  int64_t m = 0;           // coarsest level: interior unknowns
  double* ainv = nullptr;  // coarsest level: [S][m][m]
  double* tpart = nullptr; // [tiles][S] bound maxima per assembly tile
};

struct MgPlan {
  int levels = 0;
  int fp32 = 0;  // cycle in FP32 (vectors, D^-1 and matrices)
  MgLevel lv[kMgMaxLevels];
  double* part = nullptr;  // [kMgPartRows][S] scratch of the bound reduction
  size_t bytes = 0;
};

// The tiled assembly (assemble.hip): tiles of the N^3 mesh for s samples
// (the rows of a fused bound's partial array), the launcher with an optional
// fused D^-1 and bound (bnd 1: FP32, 2: FP64; dinv of that type, bpart
// [tiles][s]; adv: {alpha, vx, vy, vz} of an advection term alpha v.grad u,
// with a fused bound only; nullptr or alpha = 0: diffusion alone), and the
// parts of a KL table.
int64_t asm_tiles(int N, int S);
ens_status assemble_launch(int N, const ens_graph* graph, const double* sq, const int32_t* tr, const double* phi,
                           const ens_problem* prob, int s, const double* xi, double* values, float* values32,
                           double* rhs, int bnd, void* dinv, double* bpart, hipStream_t stream,
                           const double* adv = nullptr);
void kl_parts(const void* kl, int M, const double** sq, const int32_t** tr, const double** phi);

// One group of a batched assembly: its mesh, KL table parts, KL inputs
// [s][M], graph, and the buffers it fills (FP64 values, load vector, the
// solution set to zero); tile0 is its first workgroup in the flat launch.
struct AsmGroupDev {
  int32_t N;
  int64_t tile0;
  const double *sq, *phi;
  const int32_t* tr;
  const double* xi;
  const int32_t* rp;
  double *values, *rhs, *x;
};
// The assemblies of a batch's groups in one launch of `blocks` workgroups
// (the groups' asm_tiles summed); blk_grp [blocks] maps workgroup -> group.
ens_status batch_assemble_launch(int S, const AsmGroupDev* groups, const int32_t* blk_grp, int64_t blocks,
                                 const ens_problem& prob, hipStream_t st);

int mg_levels(int N, int* Ns);
// 0: buffer unknown; 1: built (ens_mg_build); 2: set up (ens_mg_setup).
int mg_stage(const ens_mg* mg);
// 1 if the buffer is set up for the (nonsymmetric) advection-diffusion
// operator (ens_mg_assemble_setup_adv).
int mg_nonsym(const ens_mg* mg);
// Carve the hierarchy buffer (base nullable: sizes only).  Returns false if
// the coarsest level is too large for its dense solve.
bool mg_plan(int N, int M, int S, int fp32, char* base, MgPlan* plan);
// Attach the fine level's graph and matrices (vals32 only for FP32 cycles).
void mg_attach_fine(MgPlan* plan, const int32_t* rp, const int32_t* ci, const double* vals, const float* vals32);
// z = M r for all samples in the cycle precision T; every kernel returns at
// once when the control block (nullable) reports no active sample.  With
// dot (nullable), the last fine-level pass also writes the per-sample
// partials of r . z, one row of S doubles per row tile of 4 wavefronts
// (ceil(n / (4 * rows per wavefront)) rows).
template <typename T, int S>
void mg_vcycle(const MgPlan& plan, const T* r, T* z, const Ctl* gate, hipStream_t st, double* dot = nullptr);

}  // namespace ens
