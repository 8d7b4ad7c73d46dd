// Kohn-Sham states of a local model potential on the Monkhorst-Pack grid.
//
// H_GG'(k) = 1/2 |k+G|^2 delta_GG' + V(G - G') on the plane-wave sphere,
// dense FP64 Hermitian eigensolve (rocSOLVER, divide and conquer) in batches
// of k, band count moved up to a multiplet end, chemical potential by
// bisection on the electron count, Fermi-Dirac occupations.
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace tdx {
namespace {

constexpr double kDegenTol = 1e-6;  // eigenvalue gap that separates multiplets

struct HostBasis {
  Lattice L;
  std::vector<std::vector<int>> m;  // per k, flattened triples
  int npw_max = 0;
  int mmax[3] = {0, 0, 0};          // max |Miller| per axis over all k
};

int validate(const tdx_model *md) {
  TDX_REQUIRE(md, TDX_ERR_INVALID_ARG, "model is null");
  for (int i = 0; i < 3; ++i)
    TDX_REQUIRE(md->kgrid[i] > 0 && md->kgrid[i] <= 1024, TDX_ERR_INVALID_ARG, "bad kgrid");
  TDX_REQUIRE(std::isfinite(md->ecut_wf) && md->ecut_wf > 0, TDX_ERR_INVALID_ARG, "bad ecut_wf");
  TDX_REQUIRE(md->n_bands >= 0, TDX_ERR_INVALID_ARG, "bad n_bands");
  TDX_REQUIRE(std::isfinite(md->n_electrons) && md->n_electrons > 0, TDX_ERR_INVALID_ARG,
              "bad n_electrons");
  TDX_REQUIRE(md->n_atoms >= 0 && (md->n_atoms == 0 || md->positions), TDX_ERR_INVALID_ARG,
              "bad positions");
  TDX_REQUIRE(md->n_shells >= 0 && md->n_shells <= 64 &&
                  (md->n_shells == 0 || (md->shell_n2 && md->shell_v)),
              TDX_ERR_INVALID_ARG, "bad shell table");
  for (int i = 0; i < 3 * md->n_atoms; ++i)
    TDX_REQUIRE(std::isfinite(md->positions[i]), TDX_ERR_INVALID_ARG, "non-finite position");
  for (int j = 0; j < md->n_shells; ++j)
    TDX_REQUIRE(std::isfinite(md->shell_v[j]), TDX_ERR_INVALID_ARG, "non-finite shell_v");
  return TDX_OK;
}

int host_basis(const tdx_model *md, HostBasis *hb) {
  TDX_TRY(make_lattice(md->cell, &hb->L));
  const int nk = md->kgrid[0] * md->kgrid[1] * md->kgrid[2];
  hb->m.resize(nk);
  for (int k = 0; k < nk; ++k) {
    int r[3];
    kindex_split(k, md->kgrid, r);
    double red[3];
    mp_point(md->kgrid, r[0], r[1], r[2], red);
    gsphere(hb->L, red, md->ecut_wf, &hb->m[k]);
    const int n = (int)hb->m[k].size() / 3;
    hb->npw_max = std::max(hb->npw_max, n);
    for (int i = 0; i < 3 * n; ++i)
      hb->mmax[i % 3] = std::max(hb->mmax[i % 3], std::abs(hb->m[k][i]));
  }
  return TDX_OK;
}

// V on the box of Miller differences |d_i| <= D_i, index
// ((d0 + D0) * (2 D1 + 1) + d1 + D1) * (2 D2 + 1) + d2 + D2.
__global__ void k_vtable(double2 *vt, int D0, int D1, int D2, double3 b0, double3 b1, double3 b2,
                         double volume, const double *pos, int n_atoms, const int *shell_n2,
                         const double *shell_v, int n_shells, double shell_unit, int gauss,
                         double z_ion, double sigma) {
  const int n1 = 2 * D1 + 1, n2 = 2 * D2 + 1;
  const long total = (long)(2 * D0 + 1) * n1 * n2;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x) {
    const int d2 = (int)(i % n2) - D2;
    const int d1 = (int)((i / n2) % n1) - D1;
    const int d0 = (int)(i / ((long)n1 * n2)) - D0;
    const double gx = d0 * b0.x + d1 * b1.x + d2 * b2.x;
    const double gy = d0 * b0.y + d1 * b1.y + d2 * b2.y;
    const double gz = d0 * b0.z + d1 * b1.z + d2 * b2.z;
    const double g2 = gx * gx + gy * gy + gz * gz;
    double v = 0.0;
    bool matched = false;
    for (int s = 0; s < n_shells; ++s) {
      const double s2 = shell_unit * shell_unit * shell_n2[s];
      if (fabs(g2 - s2) <= 1e-9 * s2) {
        v = shell_v[s];
        matched = true;
      }
    }
    if (!matched && gauss && g2 > 0)
      v = -4.0 * M_PI * z_ion * exp(-0.5 * sigma * sigma * g2) / (volume * g2);
    if (d0 == 0 && d1 == 0 && d2 == 0) v = 0.0;
    double sr = 0.0, si = 0.0;
    for (int a = 0; a < n_atoms; ++a) {
      const double ph = gx * pos[3 * a] + gy * pos[3 * a + 1] + gz * pos[3 * a + 2];
      double s, c;
      sincos(ph, &s, &c);
      sr += c;
      si -= s;
    }
    vt[i] = make_double2(v * sr, v * si);
  }
}

// Column-major Hamiltonians of a batch of k-points sharing the basis size
// n: A[kk][i + j*n] for k = klist[kk].
__global__ void k_build_h(double2 *A, int n, const int *klist, int nkb, const int *miller,
                          int npw_max, const double *kcart, const double2 *vt, int D0, int D1,
                          int D2, double3 b0, double3 b1, double3 b2) {
  const int i = blockIdx.x * 16 + threadIdx.x;
  const int j = blockIdx.y * 16 + threadIdx.y;
  const int kk = blockIdx.z;
  if (i >= n || j >= n || kk >= nkb) return;
  const int k = klist[kk];
  const int *mi = miller + ((size_t)k * npw_max + i) * 3;
  const int *mj = miller + ((size_t)k * npw_max + j) * 3;
  const int d0 = mi[0] - mj[0], d1 = mi[1] - mj[1], d2 = mi[2] - mj[2];
  const long idx = ((long)(d0 + D0) * (2 * D1 + 1) + (d1 + D1)) * (2 * D2 + 1) + (d2 + D2);
  double2 h = vt[idx];
  if (i == j) {
    const double *kc = kcart + 3 * k;
    const double px = kc[0] + mi[0] * b0.x + mi[1] * b1.x + mi[2] * b2.x;
    const double py = kc[1] + mi[0] * b0.y + mi[1] * b1.y + mi[2] * b2.y;
    const double pz = kc[2] + mi[0] * b0.z + mi[1] * b1.z + mi[2] * b2.z;
    h.x += 0.5 * (px * px + py * py + pz * pz);
    h.y = 0.0;
  }
  A[(size_t)kk * n * n + (size_t)j * n + i] = h;
}

// flag = 1 if any eigenvector entry of the batch is not finite
__global__ void k_finite(const double2 *A, size_t count, int *flag) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    if (!isfinite(A[i].x) || !isfinite(A[i].y)) atomicOr(flag, 1);
}

// Copy eigenpairs of a batch out as band rows, zero beyond n.
__global__ void k_extract(const double2 *A, const double *D, int n, const int *klist, int nkb,
                          int nb_max, int npw_max, double *eps, double2 *coef) {
  const int kk = blockIdx.y;
  const int nband = blockIdx.x;
  if (kk >= nkb || nband >= nb_max) return;
  const int k = klist[kk];
  double2 *dst = coef + ((size_t)k * nb_max + nband) * npw_max;
  if (nband >= n) {
    for (int i = threadIdx.x; i < npw_max; i += blockDim.x) dst[i] = make_double2(0.0, 0.0);
    if (threadIdx.x == 0) eps[(size_t)k * nb_max + nband] = INFINITY;
    return;
  }
  const double2 *src = A + (size_t)kk * n * n + (size_t)nband * n;
  for (int i = threadIdx.x; i < npw_max; i += blockDim.x)
    dst[i] = i < n ? src[i] : make_double2(0.0, 0.0);
  if (threadIdx.x == 0) eps[(size_t)k * nb_max + nband] = D[(size_t)kk * n + nband];
}

// Band count per k: n_bands moved up past any multiplet; flag if the
// capacity is exceeded.
__global__ void k_snap(const double *eps, const int *npw, int nk, int nb_max, int n_bands,
                       int *nb, int *flag) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  const int n = npw[k];
  int c = (n_bands <= 0 || n_bands >= n) ? n : n_bands;
  const double *e = eps + (size_t)k * nb_max;
  while (c < n) {
    if (c >= nb_max) {
      atomicOr(flag, 1);
      c = nb_max;
      break;
    }
    if (e[c] - e[c - 1] >= kDegenTol) break;
    ++c;
  }
  if (c > nb_max) {
    atomicOr(flag, 1);
    c = nb_max;
  }
  nb[k] = c;
}

__device__ inline double fermi(double x) {
  if (x > 0.0) {
    const double e = exp(-x);
    return e / (1.0 + e);
  }
  return 1.0 / (1.0 + exp(x));
}

constexpr int kMuThreads = 1024;

// Block reduction in a fixed order (deterministic).
__device__ double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kMuThreads / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ double block_min(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kMuThreads / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmin(sh[t], sh[t + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Chemical potential by bisection on (2/N_k) sum f = N_e, run by one block.
// out[0] = mu, out[1] = status (0 ok, 1 too few bands).
__global__ void __launch_bounds__(kMuThreads)
    k_find_mu(const double *eps, const int *nb, int nk, int nb_max, double T, double ne,
              double *out) {
  __shared__ double sh[kMuThreads];
  double lo_l = INFINITY, hi_l = -INFINITY, cnt_l = 0.0;
  for (long i = threadIdx.x; i < (long)nk * nb_max; i += kMuThreads) {
    const int k = (int)(i / nb_max), n = (int)(i % nb_max);
    if (n < nb[k]) {
      lo_l = fmin(lo_l, eps[i]);
      hi_l = fmax(hi_l, eps[i]);
      cnt_l += 1.0;
    }
  }
  const double emin = block_min(lo_l, sh);
  const double emax = -block_min(-hi_l, sh);
  const double nstates = block_sum(cnt_l, sh);
  if (2.0 * nstates / nk <= ne) {
    if (threadIdx.x == 0) {
      out[0] = 0.0;
      out[1] = 1.0;
    }
    return;
  }
  double lo = emin - 50.0 * T, hi = emax + 50.0 * T;
  for (int it = 0; it < 2000; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    double s = 0.0;
    for (long i = threadIdx.x; i < (long)nk * nb_max; i += kMuThreads) {
      const int k = (int)(i / nb_max), n = (int)(i % nb_max);
      if (n < nb[k]) s += fermi((eps[i] - mid) / T);
    }
    const double count = 2.0 / nk * block_sum(s, sh);
    if (count < ne)
      lo = mid;
    else
      hi = mid;
  }
  if (threadIdx.x == 0) {
    out[0] = 0.5 * (lo + hi);
    out[1] = 0.0;
  }
}

// Occupations at mu; top[k] = occupation of the highest kept band.
__global__ void k_occ(const double *eps, const int *nb, int nk, int nb_max, double T,
                      const double *mu_p, double *occ, double *top) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)nk * nb_max) return;
  const int k = (int)(i / nb_max), n = (int)(i % nb_max);
  const double mu = mu_p[0];
  const double f = n < nb[k] ? fermi((eps[i] - mu) / T) : 0.0;
  occ[i] = f;
  if (n == nb[k] - 1) top[k] = f;
}

int occupations_impl(tdx_ctx *ctx, tdx_states *st, double T, double ne, double f_trunc,
                     hipStream_t s) {
  TDX_REQUIRE(std::isfinite(T) && T > 0, TDX_ERR_INVALID_ARG, "temperature must be > 0");
  TDX_REQUIRE(std::isfinite(ne) && ne > 0, TDX_ERR_INVALID_ARG, "bad electron count");
  void *aux;
  TDX_TRY(ws_get(ctx, WS_MISC, sizeof(double) * (2 + st->n_k), &aux));
  double *d_out = (double *)aux;
  double *d_top = d_out + 2;
  hipLaunchKernelGGL(k_find_mu, dim3(1), dim3(kMuThreads), 0, s, st->eps, st->nb, st->n_k,
                     st->nb_max, T, ne, d_out);
  TDX_HIP(hipGetLastError());
  const long tot = (long)st->n_k * st->nb_max;
  hipLaunchKernelGGL(k_occ, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, st->eps,
                     st->nb, st->n_k, st->nb_max, T, d_out, st->occ, d_top);
  TDX_HIP(hipGetLastError());
  std::vector<double> h(2 + st->n_k);
  TDX_HIP(hipMemcpyAsync(h.data(), d_out, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
  TDX_HIP(hipStreamSynchronize(s));
  TDX_REQUIRE(h[1] == 0.0, TDX_ERR_NUMERIC, "too few bands for %g electrons", ne);
  double top = 0.0;
  for (int k = 0; k < st->n_k; ++k) top = std::max(top, h[2 + k]);
  TDX_REQUIRE(top < f_trunc, TDX_ERR_NUMERIC,
              "band set too small: highest kept band has occupation %.3e >= %.3e", top, f_trunc);
  st->mu = h[0];
  st->temperature = T;
  return TDX_OK;
}

}  // namespace
}  // namespace tdx

using namespace tdx;

extern "C" {

int tdx_states_query(const tdx_model *model, tdx_states_dims *out) {
  clear_error();
  TDX_TRY(validate(model));
  TDX_REQUIRE(out, TDX_ERR_INVALID_ARG, "out is null");
  HostBasis hb;
  TDX_TRY(host_basis(model, &hb));
  out->n_k = model->kgrid[0] * model->kgrid[1] * model->kgrid[2];
  out->npw_max = hb.npw_max;
  out->nb_max = model->n_bands <= 0 ? hb.npw_max : std::min(hb.npw_max, model->n_bands + 64);
  return TDX_OK;
}

int tdx_build_states(tdx_ctx *ctx, const tdx_model *md, double T, tdx_states *st,
                     tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && st, TDX_ERR_INVALID_ARG, "null argument");
  TDX_TRY(validate(md));
  TDX_REQUIRE(std::isfinite(T) && T > 0, TDX_ERR_INVALID_ARG, "temperature must be > 0");
  TDX_REQUIRE(st->npw && st->nb && st->miller && st->eps && st->occ && st->coef,
              TDX_ERR_INVALID_ARG, "a states buffer is null");
  TDX_TRY(check_device(ctx));
  hipStream_t s = as_stream(stream);
  HostBasis hb;
  TDX_TRY(host_basis(md, &hb));
  const int nk = md->kgrid[0] * md->kgrid[1] * md->kgrid[2];
  const int nb_need = md->n_bands <= 0 ? hb.npw_max : std::min(hb.npw_max, md->n_bands + 64);
  TDX_REQUIRE(st->n_k == nk && st->npw_max == hb.npw_max && st->nb_max == nb_need,
              TDX_ERR_SHAPE, "states dims (%d,%d,%d) differ from tdx_states_query (%d,%d,%d)",
              st->n_k, st->npw_max, st->nb_max, nk, hb.npw_max, nb_need);
  const Lattice &L = hb.L;
  st->omega_cell = L.volume;
  for (int i = 0; i < 3; ++i) {
    st->kgrid[i] = md->kgrid[i];
    st->mmax[i] = hb.mmax[i];
    for (int j = 0; j < 3; ++j) {
      st->cell[3 * i + j] = L.a[i][j];
      st->bvec[3 * i + j] = L.b[i][j];
    }
  }
  const int npw_max = hb.npw_max;

  // basis tables
  std::vector<int> npw(nk), mill((size_t)nk * npw_max * 3, 0);
  std::vector<double> kc(3 * (size_t)nk);
  for (int k = 0; k < nk; ++k) {
    npw[k] = (int)hb.m[k].size() / 3;
    std::copy(hb.m[k].begin(), hb.m[k].end(), mill.begin() + (size_t)k * npw_max * 3);
    int r[3];
    kindex_split(k, md->kgrid, r);
    double red[3];
    mp_point(md->kgrid, r[0], r[1], r[2], red);
    for (int j = 0; j < 3; ++j) kc[3 * k + j] = red[0] * L.b[0][j] + red[1] * L.b[1][j] + red[2] * L.b[2][j];
  }
  TDX_HIP(hipMemcpyAsync(st->npw, npw.data(), sizeof(int) * nk, hipMemcpyHostToDevice, s));
  TDX_HIP(hipMemcpyAsync(st->miller, mill.data(), sizeof(int) * mill.size(), hipMemcpyHostToDevice, s));

  // V(G) on the box of Miller differences
  const int D0 = 2 * hb.mmax[0], D1 = 2 * hb.mmax[1], D2 = 2 * hb.mmax[2];
  const size_t nvt = (size_t)(2 * D0 + 1) * (2 * D1 + 1) * (2 * D2 + 1);
  const size_t small_bytes = sizeof(double) * (3 * nk + 3 * std::max(md->n_atoms, 1) + 64) +
                             sizeof(int) * (64 + nk);
  void *tab;
  TDX_TRY(ws_get(ctx, WS_MISC2, nvt * sizeof(double2) + small_bytes, &tab));
  double2 *d_vt = (double2 *)tab;
  double *d_kc = (double *)(d_vt + nvt);
  double *d_pos = d_kc + 3 * nk;
  double *d_sv = d_pos + 3 * std::max(md->n_atoms, 1);
  int *d_sn = (int *)(d_sv + 64);
  int *d_klist = d_sn + 64;
  TDX_HIP(hipMemcpyAsync(d_kc, kc.data(), sizeof(double) * kc.size(), hipMemcpyHostToDevice, s));
  if (md->n_atoms)
    TDX_HIP(hipMemcpyAsync(d_pos, md->positions, sizeof(double) * 3 * md->n_atoms,
                           hipMemcpyHostToDevice, s));
  if (md->n_shells) {
    TDX_HIP(hipMemcpyAsync(d_sv, md->shell_v, sizeof(double) * md->n_shells, hipMemcpyHostToDevice, s));
    TDX_HIP(hipMemcpyAsync(d_sn, md->shell_n2, sizeof(int) * md->n_shells, hipMemcpyHostToDevice, s));
  }
  const double3 b0 = make_double3(L.b[0][0], L.b[0][1], L.b[0][2]);
  const double3 b1 = make_double3(L.b[1][0], L.b[1][1], L.b[1][2]);
  const double3 b2 = make_double3(L.b[2][0], L.b[2][1], L.b[2][2]);
  hipLaunchKernelGGL(k_vtable, dim3((unsigned)std::min<size_t>((nvt + 255) / 256, 65535)), dim3(256),
                     0, s, d_vt, D0, D1, D2, b0, b1, b2, L.volume, d_pos, md->n_atoms, d_sn,
                     d_sv, md->n_shells, md->shell_unit, md->gauss, md->z_ion, md->sigma);
  TDX_HIP(hipGetLastError());

  // k-points grouped by basis size: one unpadded batched eigensolve per size
  std::vector<int> order(nk);
  for (int k = 0; k < nk; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return npw[a] < npw[b]; });
  TDX_HIP(hipMemcpyAsync(d_klist, order.data(), sizeof(int) * nk, hipMemcpyHostToDevice, s));
  const size_t per_max = (size_t)npw_max * npw_max * sizeof(double2);
  const int kb_max = (int)std::max<size_t>(1, std::min<size_t>((size_t)nk, ((size_t)4 << 30) / per_max));
  void *wa, *wb;
  TDX_TRY(ws_get(ctx, WS_EIG, per_max * kb_max, &wa));
  TDX_TRY(ws_get(ctx, WS_EIG_AUX, ((size_t)2 * npw_max * sizeof(double) + sizeof(int)) * kb_max + 256, &wb));
  double2 *dA = (double2 *)wa;
  double *dD = (double *)wb;
  double *dE = dD + (size_t)npw_max * kb_max;
  int *dinfo = (int *)(dE + (size_t)npw_max * kb_max);
  int *d_flag = dinfo + kb_max;
  TDX_REQUIRE(rocblas_set_stream(ctx->blas, s) == rocblas_status_success, TDX_ERR_HIP,
              "rocblas_set_stream failed");
  std::vector<int> hinfo(kb_max + 1);
  for (int g0 = 0; g0 < nk;) {
    const int n = npw[order[g0]];
    int g1 = g0;
    while (g1 < nk && npw[order[g1]] == n && g1 - g0 < kb_max) ++g1;
    const int nkb = g1 - g0;
    for (int attempt = 0; attempt < 2; ++attempt) {
      dim3 g((n + 15) / 16, (n + 15) / 16, nkb);
      hipLaunchKernelGGL(k_build_h, g, dim3(16, 16), 0, s, dA, n, d_klist + g0, nkb, st->miller,
                         npw_max, d_kc, d_vt, D0, D1, D2, b0, b1, b2);
      TDX_HIP(hipGetLastError());
      // divide and conquer first; QR iteration if it returns non-finite vectors
      rocblas_status rs =
          attempt == 0
              ? rocsolver_zheevd_strided_batched(ctx->blas, rocblas_evect_original,
                                                 rocblas_fill_upper, n,
                                                 (rocblas_double_complex *)dA, n,
                                                 (rocblas_stride)n * n, dD, n, dE, n, dinfo, nkb)
              : rocsolver_zheev_strided_batched(ctx->blas, rocblas_evect_original,
                                                rocblas_fill_upper, n,
                                                (rocblas_double_complex *)dA, n,
                                                (rocblas_stride)n * n, dD, n, dE, n, dinfo, nkb);
      TDX_REQUIRE(rs == rocblas_status_success, TDX_ERR_HIP, "rocsolver eigensolver failed (%d)",
                  (int)rs);
      TDX_HIP(hipMemsetAsync(d_flag, 0, sizeof(int), s));
      const size_t cnt = (size_t)nkb * n * n;
      hipLaunchKernelGGL(k_finite, dim3((unsigned)std::min<size_t>((cnt + 255) / 256, 4096)),
                         dim3(256), 0, s, dA, cnt, d_flag);
      TDX_HIP(hipGetLastError());
      TDX_HIP(hipMemcpyAsync(hinfo.data(), dinfo, sizeof(int) * nkb, hipMemcpyDeviceToHost, s));
      TDX_HIP(hipMemcpyAsync(&hinfo[kb_max], d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
      TDX_HIP(hipStreamSynchronize(s));
      bool ok = hinfo[kb_max] == 0;
      for (int i = 0; i < nkb; ++i) ok = ok && hinfo[i] == 0;
      if (ok) break;
      TDX_REQUIRE(attempt == 0, TDX_ERR_NUMERIC, "eigensolver failed for basis size %d", n);
    }
    hipLaunchKernelGGL(k_extract, dim3(st->nb_max, nkb), dim3(256), 0, s, dA, dD, n,
                       d_klist + g0, nkb, st->nb_max, npw_max, st->eps, (double2 *)st->coef);
    TDX_HIP(hipGetLastError());
    g0 = g1;
  }

  // band counts
  TDX_HIP(hipMemsetAsync(d_flag, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_snap, dim3((nk + 127) / 128), dim3(128), 0, s, st->eps, st->npw, nk,
                     st->nb_max, md->n_bands, st->nb, d_flag);
  TDX_HIP(hipGetLastError());
  int flag = 0;
  TDX_HIP(hipMemcpyAsync(&flag, d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  TDX_HIP(hipStreamSynchronize(s));
  TDX_REQUIRE(flag == 0, TDX_ERR_SHAPE, "a multiplet straddles the band capacity %d", st->nb_max);
  return occupations_impl(ctx, st, T, md->n_electrons, md->f_trunc, s);
}

int tdx_occupations(tdx_ctx *ctx, tdx_states *st, double T, double ne, double f_trunc,
                    tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && st && st->eps && st->nb && st->occ, TDX_ERR_INVALID_ARG, "null argument");
  TDX_TRY(check_device(ctx));
  return occupations_impl(ctx, st, T, ne, f_trunc, as_stream(stream));
}

}  // extern "C"
