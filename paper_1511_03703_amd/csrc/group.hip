// Grouping of samples into ensembles (Sec. 3.7): an ensemble runs as long
// as its slowest sample, so samples expected to need similar iteration
// counts belong together.  The paper names the variation of a sample's
// parameters over the domain as a predictor of its count; the device side
// of that predictor is ens_kl_extrema (assemble.hip), and this host step
// turns any per-sample key into an order whose consecutive runs are the
// ensembles.
#include <cmath>

#include <algorithm>
#include <numeric>
#include <vector>

#include "common.hpp"

using namespace ens;

extern "C" ens_status ens_group_order(int64_t count, const double* key, int32_t* perm) {
  ENS_ARG_CHECK(count >= 0 && count <= INT32_MAX, "count out of range");
  ENS_ARG_CHECK(count == 0 || (key && perm), "null key or perm");
  std::vector<int32_t> idx((size_t)count);
  std::iota(idx.begin(), idx.end(), 0);
  // ascending key, equal keys in index order, non-finite keys last (in
  // index order): a strict weak order, so the stable sort is deterministic
  std::stable_sort(idx.begin(), idx.end(), [key](int32_t a, int32_t b) {
    const bool fa = std::isfinite(key[a]), fb = std::isfinite(key[b]);
    if (fa != fb) return fa;
    return fa && key[a] < key[b];
  });
  std::copy(idx.begin(), idx.end(), perm);
  return ENS_OK;
}
