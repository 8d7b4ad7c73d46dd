// Screened transition list T(q) = {(k,n,m): |f_nk - f_m,k+q| > thr}, CSR by k,
// ordered by k, then n, then m (two passes: count, then fill at prefix sums).
// In the paired form one transition of each time-reversal pair is kept: all
// of k when its partner -k-q has a larger index, n < m when k is its own
// partner, none otherwise.
#include <cmath>

#include "internal.h"

namespace tdx {
namespace {

constexpr int kThreads = 256;

// which transitions (k, n, m) of a k-point the list keeps: 0 none, 1 all,
// 2 those with n < m
__device__ inline int keep_mode(int k, const int *kt) {
  if (!kt) return 1;
  return kt[k] > k ? 1 : (kt[k] == k ? 2 : 0);
}

__global__ void __launch_bounds__(kThreads)
    k_trans_count(const double *occ, const int *nb, int nb_max, const int *kp, const int *kt,
                  double thr, int *rowcnt, long long *kcount) {
  const int k = blockIdx.x;
  const int j = kp[k];
  const int mode = keep_mode(k, kt);
  const int nbk = mode ? nb[k] : 0, nbj = nb[j];
  const double *fk = occ + (size_t)k * nb_max;
  const double *fj = occ + (size_t)j * nb_max;
  __shared__ long long sh[kThreads];
  long long local = 0;
  for (int n = threadIdx.x; n < nb_max; n += kThreads) {
    int c = 0;
    if (n < nbk) {
      const double fn = fk[n];
      for (int m = mode == 2 ? n + 1 : 0; m < nbj; ++m) c += fabs(fn - fj[m]) > thr;
    }
    rowcnt[(size_t)k * nb_max + n] = c;
    local += c;
  }
  sh[threadIdx.x] = local;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) kcount[k] = sh[0];
}

__global__ void __launch_bounds__(kThreads)
    k_trans_fill(const double *occ, const double *eps, const int *nb, int nb_max, const int *kp,
                 const int *kt, double thr, const int *rowcnt, const long long *koff, int *ok,
                 int *on, int *om, double *odelta, double *odf) {
  extern __shared__ long long rowoff[];  // [nb_max]
  const int k = blockIdx.x;
  const int j = kp[k];
  const int mode = keep_mode(k, kt);
  const int nbk = mode ? nb[k] : 0, nbj = nb[j];
  if (threadIdx.x == 0) {
    long long acc = koff[k];
    for (int n = 0; n < nb_max; ++n) {
      rowoff[n] = acc;
      acc += rowcnt[(size_t)k * nb_max + n];
    }
  }
  __syncthreads();
  const double *fk = occ + (size_t)k * nb_max, *fj = occ + (size_t)j * nb_max;
  const double *ek = eps + (size_t)k * nb_max, *ej = eps + (size_t)j * nb_max;
  for (int n = threadIdx.x; n < nbk; n += kThreads) {
    long long t = rowoff[n];
    const double fn = fk[n], en = ek[n];
    for (int m = mode == 2 ? n + 1 : 0; m < nbj; ++m) {
      const double df = fn - fj[m];
      if (fabs(df) > thr) {
        ok[t] = k;
        on[t] = n;
        om[t] = m;
        odelta[t] = ej[m] - en;
        odf[t] = df;
        ++t;
      }
    }
  }
}

}  // namespace
}  // namespace tdx

using namespace tdx;

extern "C" int tdx_transitions(tdx_ctx *ctx, const tdx_states *st, const int qj[3], double thr,
                               tdx_translist *tl, int64_t *count, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && st && qj && tl && count, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(std::isfinite(thr) && thr >= 0, TDX_ERR_INVALID_ARG, "bad threshold");
  TDX_REQUIRE(st->occ && st->eps && st->nb, TDX_ERR_INVALID_ARG, "states not built");
  TDX_TRY(check_device(ctx));
  hipStream_t s = as_stream(stream);
  const int nk = st->n_k, nb_max = st->nb_max;
  TDX_REQUIRE(st->kgrid[0] * st->kgrid[1] * st->kgrid[2] == nk, TDX_ERR_SHAPE,
              "states kgrid does not match n_k");
  TDX_REQUIRE(nb_max <= 16384, TDX_ERR_SHAPE, "nb_max %d above 16384", nb_max);
  TDX_REQUIRE(tl->paired == 0 || tl->paired == 1, TDX_ERR_INVALID_ARG, "paired must be 0 or 1");
  std::vector<int> kp, gs;
  kq_map(st->kgrid, qj, &kp, &gs);
  // time-reversal partner of each k: -k-q on the grid.  Monkhorst-Pack index
  // r maps to N-1-r under k -> -k.
  std::vector<int> kt(nk);
  for (int k = 0; k < nk; ++k) {
    int r[3];
    kindex_split(k, st->kgrid, r);
    int rt[3];
    for (int i = 0; i < 3; ++i) {
      const int N = st->kgrid[i];
      rt[i] = (((N - 1 - r[i] - qj[i]) % N) + N) % N;
    }
    kt[k] = (rt[0] * st->kgrid[1] + rt[1]) * st->kgrid[2] + rt[2];
  }
  void *w1, *w2;
  TDX_TRY(ws_get(ctx, WS_ROWS, sizeof(int) * (size_t)nk * nb_max, &w1));
  TDX_TRY(ws_get(ctx, WS_MISC, sizeof(long long) * (2 * (size_t)nk + 1) + 2 * sizeof(int) * nk,
                 &w2));
  int *d_rows = (int *)w1;
  long long *d_kcount = (long long *)w2;
  long long *d_koff = d_kcount + nk;
  int *d_kp = (int *)(d_koff + nk + 1);
  int *d_kt = d_kp + nk;
  TDX_HIP(hipMemcpyAsync(d_kp, kp.data(), sizeof(int) * nk, hipMemcpyHostToDevice, s));
  TDX_HIP(hipMemcpyAsync(d_kt, kt.data(), sizeof(int) * nk, hipMemcpyHostToDevice, s));
  const int *kt_arg = tl->paired ? d_kt : nullptr;
  hipLaunchKernelGGL(k_trans_count, dim3(nk), dim3(kThreads), 0, s, st->occ, st->nb, nb_max,
                     d_kp, kt_arg, thr, d_rows, d_kcount);
  TDX_HIP(hipGetLastError());
  std::vector<long long> kc(nk), off(nk + 1);
  TDX_HIP(hipMemcpyAsync(kc.data(), d_kcount, sizeof(long long) * nk, hipMemcpyDeviceToHost, s));
  TDX_HIP(hipStreamSynchronize(s));
  off[0] = 0;
  for (int k = 0; k < nk; ++k) off[k + 1] = off[k] + kc[k];
  *count = off[nk];
  if (tl->capacity < off[nk])
    return fail(TDX_ERR_SHAPE, "transition capacity %lld < %lld", (long long)tl->capacity,
                (long long)off[nk]);
  if (!tl->k && !tl->n && !tl->m && !tl->delta && !tl->df && !tl->k_offsets)
    return TDX_OK;  // a count query
  TDX_REQUIRE(tl->k_offsets && (off[nk] == 0 || (tl->k && tl->n && tl->m && tl->delta && tl->df)),
              TDX_ERR_INVALID_ARG, "a transition buffer is null");
  TDX_HIP(hipMemcpyAsync(d_koff, off.data(), sizeof(long long) * (nk + 1), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_trans_fill, dim3(nk), dim3(kThreads), sizeof(long long) * nb_max, s,
                     st->occ, st->eps, st->nb, nb_max, d_kp, kt_arg, thr, d_rows, d_koff, tl->k,
                     tl->n, tl->m, tl->delta, tl->df);
  TDX_HIP(hipGetLastError());
  TDX_HIP(hipMemcpyAsync(tl->k_offsets, off.data(), sizeof(int64_t) * (nk + 1),
                         hipMemcpyHostToDevice, s));
  TDX_HIP(hipStreamSynchronize(s));
  return TDX_OK;
}
