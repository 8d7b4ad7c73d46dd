// Device tables shared by the pair-density kernels and their adjoints.
#pragma once

#include "internal.h"

namespace tdx {
namespace {

// Miller-index lookup box per k: lut[k][(m0+M0)(2M1+1)(2M2+1) + ...] = index
// of that plane wave in the basis of k, -1 (preset) if absent.
__global__ void k_lut(const int *miller, const int *npw, int npw_max, int nk, int M0, int M1,
                      int M2, int *lut, long box) {
  const int k = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk || i >= npw[k]) return;
  const int *m = miller + ((size_t)k * npw_max + i) * 3;
  const long idx = ((long)(m[0] + M0) * (2 * M1 + 1) + (m[1] + M1)) * (2 * M2 + 1) + (m[2] + M2);
  lut[(size_t)k * box + idx] = i;
}

// First and one-past-last transition of every (k, n) row (0, 0 if empty),
// over the first n_trans transitions of the list only.
__global__ void k_rows(const long long *koff, const int *tn, int nb_max, long long n_trans,
                       long long *rowbeg, long long *rowend) {
  const int k = blockIdx.x;
  const long long t0 = koff[k], t1 = koff[k + 1] < n_trans ? koff[k + 1] : n_trans;
  for (long long t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
    const int n = tn[t];
    if (t == t0 || tn[t - 1] != n) rowbeg[(size_t)k * nb_max + n] = t;
    if (t == t1 - 1 || tn[t + 1] != n) rowend[(size_t)k * nb_max + n] = t + 1;
  }
}

}  // namespace
}  // namespace tdx
