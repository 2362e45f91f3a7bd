// The truncation rule of a two-site update (Chen & Stoudenmire,
// arXiv:1910.09142, Results section: at most chi_max singular values, and
// a discarded weight relative to ||theta'||^2 at most the cutoff), shared
// by the dense truncation (update.hip) and the merge of the charge blocks
// of a U(1) update (u1.hip).
#pragma once
#include "hmps_internal.h"

namespace hmps {

struct TruncResult {
  int k;         // values kept
  double total;  // sum of all squared values (plus the unresolved tail)
  double kept;   // sum of the kept squared values
};

// key[0 .. N): singular values in descending order.  Keeps k = min(k_eps,
// chi_max), k_eps the smallest k >= 1 whose discarded tail
// sum_{j>=k} sigma_j^2 (plus `unres`, the part of ||theta'||^2 no value
// resolves) is <= cutoff * total; values at or below SIGMA_FLOOR sigma_0
// are numerically zero and always dropped.  No cut falls inside a run of
// ties (relative gaps <= TIE_TOL): when the target set the cut the whole
// run is kept (the discarded weight stays within the target), unless that
// passes chi_max; then, as when the cap sets the cut, the whole run is
// dropped unless it starts at sigma_0.  rr: unres = n2 - (sum of the
// squared values), the mixed path's unresolved tail; else 0.
__device__ inline TruncResult truncation_rule(const double *key, int N,
                                              bool rr, double n2,
                                              int chi_max, double cutoff) {
  double total = 0.0;
  for (int j = N - 1; j >= 0; --j) total += key[j] * key[j];
  const double unres = rr ? fmax(n2 - total, 0.0) : 0.0;
  total += unres;
  int kfloor = 0;
  while (kfloor < N && key[kfloor] > SIGMA_FLOOR * key[0]) ++kfloor;
  const double thr = cutoff * total;
  int k_eps = N;
  double tail = unres;
  for (int k = N; k >= 1; --k) {
    if (k < N) tail += key[k] * key[k];
    if (tail <= thr)
      k_eps = k;
    else
      break;
  }
  // the largest k allowed: the cap and the numerical floor
  int kcap = chi_max < kfloor ? chi_max : kfloor;
  if (kcap < 1) kcap = 1;
  int k = k_eps < kcap ? k_eps : kcap;
  if (k > N) k = N;
  auto tied = [&](int j) {
    return key[j - 1] - key[j] <= TIE_TOL * key[j - 1];
  };
  if (k >= 1 && k < N && tied(k)) {
    int end = k;
    while (end < N && tied(end)) ++end;
    if (k_eps <= kcap && end <= kcap) {
      k = end;
    } else {
      int i = k - 1;
      while (i > 0 && tied(i)) --i;
      if (i > 0) k = i;
    }
  }
  double kept = 0.0;
  for (int j = k - 1; j >= 0; --j) kept += key[j] * key[j];
  return {k, total, kept};
}

}  // namespace hmps
