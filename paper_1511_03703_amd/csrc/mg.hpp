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
  const double* vals = nullptr;  // level 0: the caller's values
  int32_t *own_rp = nullptr, *own_ci = nullptr;
  double* own_vals = nullptr;
  void* kl = nullptr;
  double *dinv = nullptr, *lmax = nullptr;
  double *b = nullptr, *xa = nullptr, *xb = nullptr, *r = nullptr, *d = nullptr;
  int64_t m = 0;           // coarsest level: interior unknowns
  double* ainv = nullptr;  // coarsest level: [S][m][m]
};

struct MgPlan {
  int levels = 0;
  MgLevel lv[kMgMaxLevels];
  double* part = nullptr;  // [kMgPartRows][S] scratch of the bound reduction
  size_t bytes = 0;
};

int mg_levels(int N, int* Ns);
// Carve the hierarchy buffer (base nullable: sizes only).  Returns false if
// the coarsest level is too large for its dense solve.
bool mg_plan(int N, int M, int S, char* base, MgPlan* plan);
// Attach the fine level's graph and values.
void mg_attach_fine(MgPlan* plan, const int32_t* rp, const int32_t* ci, const double* vals);
// z = M r for all samples; every kernel returns at once when the control
// block (nullable) reports no active sample.
template <int S>
void mg_vcycle(const MgPlan& plan, const double* r, double* z, const Ctl* gate, hipStream_t st);

}  // namespace ens
