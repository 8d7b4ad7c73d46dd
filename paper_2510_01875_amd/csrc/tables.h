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

// Fill of a table (a kernel rather than a memset, so that the enqueueing
// call can be captured into a HIP graph).
template <class T>
__global__ void k_fill(T *p, long long n, T v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

// k_r + q = k_{r'} + G_s on the device: kp[k] = index of k', gs[3k..3k+2] =
// G_s, for q = sum_i qj_i / N_i b_i on the Monkhorst-Pack grid N.
__global__ void k_kq_map(int n0, int n1, int n2, int q0, int q1, int q2, int *kp, int *gs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n0 * n1 * n2) return;
  const int N[3] = {n0, n1, n2}, qj[3] = {q0, q1, q2};
  const int r[3] = {k / (n1 * n2), (k / n2) % n1, k % n2};
  int rp[3];
  for (int i = 0; i < 3; ++i) {
    const int s = r[i] + qj[i];
    const int m = ((s % N[i]) + N[i]) % N[i];
    rp[i] = m;
    gs[3 * k + i] = (s - m) / N[i];
  }
  kp[k] = (rp[0] * n1 + rp[1]) * n2 + rp[2];
}

// First and one-past-last transition of every (k, n) row (0, 0 if empty),
// over the transitions t_lo .. t_hi - 1 of the list only.
__global__ void k_rows(const long long *koff, const int *tn, int nb_max, long long t_lo,
                       long long t_hi, long long *rowbeg, long long *rowend) {
  const int k = blockIdx.x;
  const long long t0 = koff[k] > t_lo ? koff[k] : t_lo;
  const long long t1 = koff[k + 1] < t_hi ? koff[k + 1] : t_hi;
  for (long long t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
    const int n = tn[t];
    if (t == t0 || tn[t - 1] != n) rowbeg[(size_t)k * nb_max + n] = t;
    if (t == t1 - 1 || tn[t + 1] != n) rowend[(size_t)k * nb_max + n] = t + 1;
  }
}

}  // namespace
}  // namespace tdx
