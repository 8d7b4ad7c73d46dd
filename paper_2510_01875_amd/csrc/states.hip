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
#include "tables.h"

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
  st->beta = 1.0 / T;
  st->n_electrons = ne;
  st->density = ne / st->omega_cell;
  st->chi0_pref = 2.0 / ((double)st->n_k * st->omega_cell);
  return TDX_OK;
}


// ---------------------------------------------------------------- adjoint
// Structure factors S(d) = sum_I exp(-i G(d).R_I) of the shell vectors.
__global__ void k_shell_sf(const int *d, int n_vec, double3 b0, double3 b1, double3 b2,
                           const double *pos, int n_atoms, double2 *sf) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_vec) return;
  const int d0 = d[3 * v], d1 = d[3 * v + 1], d2 = d[3 * v + 2];
  const double gx = d0 * b0.x + d1 * b1.x + d2 * b2.x;
  const double gy = d0 * b0.y + d1 * b1.y + d2 * b2.y;
  const double gz = d0 * b0.z + d1 * b1.z + d2 * b2.z;
  double sr = 0.0, si = 0.0;
  for (int a = 0; a < n_atoms; ++a) {
    double sn, cs;
    sincos(gx * pos[3 * a] + gy * pos[3 * a + 1] + gz * pos[3 * a + 2], &sn, &cs);
    sr += cs;
    si -= sn;
  }
  sf[v] = make_double2(sr, si);
}

// W_mn <- W_mn / (eps_n - eps_m) over all eigenpairs m of one k, zero for
// m in the multiplet of n (the loss is invariant under rotations inside a
// kept multiplet) and for columns n beyond the kept bands.  W is
// column-major n x nb_max (ld n).
__global__ void k_eig_scale(double2 *W, const double *D, int n, int nb_max, const int *nb, int k) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (m >= n || c >= nb_max) return;
  double2 &w = W[(size_t)c * n + m];
  if (c >= nb[k]) {
    w = make_double2(0.0, 0.0);
    return;
  }
  const double gap = D[c] - D[m];
  const double f = fabs(gap) > kDegenTol ? 1.0 / gap : 0.0;
  w = make_double2(w.x * f, w.y * f);
}

// Shell derivatives of one kept band n of one k:
//   part[k][n][s] = Re sum_G conj(x(G)) sum_{d on shell s} S(d) psi_n(G - d),
//   x = eps_bar_n psi_n + y_n  (dL = Re x^H dH psi_n, dH = sum_s dv_s M_s).
// One workgroup per (n, k of the batch).
__global__ void __launch_bounds__(256)
    k_shell_contract(const double2 *coef, const double *eps_bar, const int *npw, const int *nb,
                     const int *miller, int nb_max, int npw_max, const int *klist,
                     const double2 *Y, int n, const int *lut, long box, int M0, int M1, int M2,
                     const int *dvec, const int *dshell, const double2 *sf, int n_vec,
                     int n_shells, double *part) {
  __shared__ double sh[256];
  __shared__ double acc[64];
  const int band = blockIdx.x, kk = blockIdx.y;
  const int k = klist[kk];
  if (band >= nb[k]) return;
  const double2 *psi = coef + ((size_t)k * nb_max + band) * npw_max;
  const double2 *y = Y + ((size_t)kk * nb_max + band) * n;
  const double eb = eps_bar[(size_t)k * nb_max + band];
  const int *mk = miller + (size_t)k * npw_max * 3;
  const int *lutk = lut + (size_t)k * box;
  const int W1 = 2 * M1 + 1, W2 = 2 * M2 + 1;
  if (threadIdx.x < n_shells) acc[threadIdx.x] = 0.0;
  __syncthreads();
  for (int v = 0; v < n_vec; ++v) {
    const int d0 = dvec[3 * v], d1 = dvec[3 * v + 1], d2 = dvec[3 * v + 2];
    const double2 S = sf[v];
    double re = 0.0;
    for (int i = threadIdx.x; i < npw[k]; i += 256) {
      const int x0 = mk[3 * i] - d0 + M0, x1 = mk[3 * i + 1] - d1 + M1, x2 = mk[3 * i + 2] - d2 + M2;
      if (x0 < 0 || x0 > 2 * M0 || x1 < 0 || x1 >= W1 || x2 < 0 || x2 >= W2) continue;
      const int j = lutk[((long)x0 * W1 + x1) * W2 + x2];
      if (j < 0) continue;
      const double2 p = psi[i], yy = y[i], q = psi[j];
      const double xr = eb * p.x + yy.x, xi = eb * p.y + yy.y;
      const double sr = S.x * q.x - S.y * q.y, si = S.x * q.y + S.y * q.x;  // S(d) psi(G - d)
      re += xr * sr + xi * si;                                             // Re conj(x) (.)
    }
    sh[threadIdx.x] = re;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) acc[dshell[v]] += sh[0];
    __syncthreads();
  }
  if (threadIdx.x < n_shells)
    part[((size_t)k * nb_max + band) * n_shells + threadIdx.x] = acc[threadIdx.x];
}

// v_bar[s] = sum over (k, n) of part[k][n][s], fixed order.
__global__ void __launch_bounds__(256)
    k_shell_sum(const double *part, const int *nb, int nk, int nb_max, int n_shells,
                double *v_bar) {
  __shared__ double sh[256];
  const int s = blockIdx.x;
  double a = 0.0;
  for (long i = threadIdx.x; i < (long)nk * nb_max; i += 256)
    if ((int)(i % nb_max) < nb[i / nb_max]) a += part[(size_t)i * n_shells + s];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) v_bar[s] = sh[0];
}

// Hamiltonian tables shared by the states build and the potential adjoint:
// V on the box of Miller differences, k in Cartesian form, k-points grouped
// by basis size, eigensolver workspaces for up to kb_max k at a time.
struct HSetup {
  int D0 = 0, D1 = 0, D2 = 0;
  double3 b0, b1, b2;
  double2 *vt = nullptr;
  double *kc = nullptr, *pos = nullptr;
  int *klist = nullptr;
  std::vector<int> npw, order;
  int kb_max = 1;
  double2 *dA = nullptr;
  double *dD = nullptr, *dE = nullptr;
  int *dinfo = nullptr, *d_flag = nullptr;
};

int h_setup(tdx_ctx *ctx, const tdx_model *md, const HostBasis &hb, hipStream_t s, HSetup *h) {
  const Lattice &L = hb.L;
  const int nk = md->kgrid[0] * md->kgrid[1] * md->kgrid[2];
  const int npw_max = hb.npw_max;
  h->npw.resize(nk);
  std::vector<double> kc(3 * (size_t)nk);
  for (int k = 0; k < nk; ++k) {
    h->npw[k] = (int)hb.m[k].size() / 3;
    int r[3];
    kindex_split(k, md->kgrid, r);
    double red[3];
    mp_point(md->kgrid, r[0], r[1], r[2], red);
    for (int j = 0; j < 3; ++j)
      kc[3 * k + j] = red[0] * L.b[0][j] + red[1] * L.b[1][j] + red[2] * L.b[2][j];
  }
  h->D0 = 2 * hb.mmax[0];
  h->D1 = 2 * hb.mmax[1];
  h->D2 = 2 * hb.mmax[2];
  const size_t nvt = (size_t)(2 * h->D0 + 1) * (2 * h->D1 + 1) * (2 * h->D2 + 1);
  const size_t small_bytes = sizeof(double) * (3 * nk + 3 * std::max(md->n_atoms, 1) + 64) +
                             sizeof(int) * (64 + nk);
  void *tab;
  TDX_TRY(ws_get(ctx, WS_MISC2, nvt * sizeof(double2) + small_bytes, &tab));
  h->vt = (double2 *)tab;
  h->kc = (double *)(h->vt + nvt);
  double *d_pos = h->kc + 3 * nk;
  double *d_sv = d_pos + 3 * std::max(md->n_atoms, 1);
  int *d_sn = (int *)(d_sv + 64);
  h->klist = d_sn + 64;
  h->pos = d_pos;
  TDX_HIP(hipMemcpyAsync(h->kc, kc.data(), sizeof(double) * kc.size(), hipMemcpyHostToDevice, s));
  if (md->n_atoms)
    TDX_HIP(hipMemcpyAsync(d_pos, md->positions, sizeof(double) * 3 * md->n_atoms,
                           hipMemcpyHostToDevice, s));
  if (md->n_shells) {
    TDX_HIP(hipMemcpyAsync(d_sv, md->shell_v, sizeof(double) * md->n_shells, hipMemcpyHostToDevice, s));
    TDX_HIP(hipMemcpyAsync(d_sn, md->shell_n2, sizeof(int) * md->n_shells, hipMemcpyHostToDevice, s));
  }
  h->b0 = make_double3(L.b[0][0], L.b[0][1], L.b[0][2]);
  h->b1 = make_double3(L.b[1][0], L.b[1][1], L.b[1][2]);
  h->b2 = make_double3(L.b[2][0], L.b[2][1], L.b[2][2]);
  hipLaunchKernelGGL(k_vtable, dim3((unsigned)std::min<size_t>((nvt + 255) / 256, 65535)), dim3(256),
                     0, s, h->vt, h->D0, h->D1, h->D2, h->b0, h->b1, h->b2, L.volume, d_pos,
                     md->n_atoms, d_sn, d_sv, md->n_shells, md->shell_unit, md->gauss, md->z_ion,
                     md->sigma);
  TDX_HIP(hipGetLastError());
  h->order.resize(nk);
  for (int k = 0; k < nk; ++k) h->order[k] = k;
  std::stable_sort(h->order.begin(), h->order.end(),
                   [&](int a, int b) { return h->npw[a] < h->npw[b]; });
  TDX_HIP(hipMemcpyAsync(h->klist, h->order.data(), sizeof(int) * nk, hipMemcpyHostToDevice, s));
  const size_t per_max = (size_t)npw_max * npw_max * sizeof(double2);
  h->kb_max = (int)std::max<size_t>(1, std::min<size_t>((size_t)nk, ((size_t)4 << 30) / per_max));
  void *wa, *wb;
  TDX_TRY(ws_get(ctx, WS_EIG, per_max * h->kb_max, &wa));
  TDX_TRY(ws_get(ctx, WS_EIG_AUX,
                 ((size_t)2 * npw_max * sizeof(double) + sizeof(int)) * h->kb_max + 256, &wb));
  h->dA = (double2 *)wa;
  h->dD = (double *)wb;
  h->dE = h->dD + (size_t)npw_max * h->kb_max;
  h->dinfo = (int *)(h->dE + (size_t)npw_max * h->kb_max);
  h->d_flag = h->dinfo + h->kb_max;
  TDX_REQUIRE(rocblas_set_stream(ctx->blas, s) == rocblas_status_success, TDX_ERR_HIP,
              "rocblas_set_stream failed");
  // the host vectors above are released on return: wait for their copies
  TDX_HIP(hipStreamSynchronize(s));
  return TDX_OK;
}

// All eigenpairs of the nkb k-points order[g0 ...] (basis size n) into
// h.dA (column-major eigenvectors) and h.dD (ascending eigenvalues):
// divide and conquer, QR iteration if it returns non-finite vectors.
// Synchronises.
int eig_batch(tdx_ctx *ctx, const int *miller, int npw_max, HSetup &h, int g0, int nkb, int n,
              hipStream_t s) {
  std::vector<int> hinfo(nkb + 1);
  for (int attempt = 0; attempt < 2; ++attempt) {
    dim3 g((n + 15) / 16, (n + 15) / 16, nkb);
    hipLaunchKernelGGL(k_build_h, g, dim3(16, 16), 0, s, h.dA, n, h.klist + g0, nkb, miller,
                       npw_max, h.kc, h.vt, h.D0, h.D1, h.D2, h.b0, h.b1, h.b2);
    TDX_HIP(hipGetLastError());
    rocblas_status rs =
        attempt == 0
            ? rocsolver_zheevd_strided_batched(ctx->blas, rocblas_evect_original,
                                               rocblas_fill_upper, n,
                                               (rocblas_double_complex *)h.dA, n,
                                               (rocblas_stride)n * n, h.dD, n, h.dE, n, h.dinfo,
                                               nkb)
            : rocsolver_zheev_strided_batched(ctx->blas, rocblas_evect_original,
                                              rocblas_fill_upper, n,
                                              (rocblas_double_complex *)h.dA, n,
                                              (rocblas_stride)n * n, h.dD, n, h.dE, n, h.dinfo,
                                              nkb);
    TDX_REQUIRE(rs == rocblas_status_success, TDX_ERR_HIP, "rocsolver eigensolver failed (%d)",
                (int)rs);
    TDX_HIP(hipMemsetAsync(h.d_flag, 0, sizeof(int), s));
    const size_t cnt = (size_t)nkb * n * n;
    hipLaunchKernelGGL(k_finite, dim3((unsigned)std::min<size_t>((cnt + 255) / 256, 4096)),
                       dim3(256), 0, s, h.dA, cnt, h.d_flag);
    TDX_HIP(hipGetLastError());
    TDX_HIP(hipMemcpyAsync(hinfo.data(), h.dinfo, sizeof(int) * nkb, hipMemcpyDeviceToHost, s));
    TDX_HIP(hipMemcpyAsync(&hinfo[nkb], h.d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    TDX_HIP(hipStreamSynchronize(s));
    bool ok = hinfo[nkb] == 0;
    for (int i = 0; i < nkb; ++i) ok = ok && hinfo[i] == 0;
    if (ok) return TDX_OK;
    TDX_REQUIRE(attempt == 0, TDX_ERR_NUMERIC, "eigensolver failed for basis size %d", n);
  }
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
  HSetup h;
  TDX_TRY(h_setup(ctx, md, hb, s, &h));
  std::vector<int> mill((size_t)nk * npw_max * 3, 0);
  for (int k = 0; k < nk; ++k)
    std::copy(hb.m[k].begin(), hb.m[k].end(), mill.begin() + (size_t)k * npw_max * 3);
  TDX_HIP(hipMemcpyAsync(st->npw, h.npw.data(), sizeof(int) * nk, hipMemcpyHostToDevice, s));
  TDX_HIP(hipMemcpyAsync(st->miller, mill.data(), sizeof(int) * mill.size(), hipMemcpyHostToDevice, s));
  for (int g0 = 0; g0 < nk;) {
    const int n = h.npw[h.order[g0]];
    int g1 = g0;
    while (g1 < nk && h.npw[h.order[g1]] == n && g1 - g0 < h.kb_max) ++g1;
    const int nkb = g1 - g0;
    TDX_TRY(eig_batch(ctx, st->miller, npw_max, h, g0, nkb, n, s));
    hipLaunchKernelGGL(k_extract, dim3(st->nb_max, nkb), dim3(256), 0, s, h.dA, h.dD, n,
                       h.klist + g0, nkb, st->nb_max, npw_max, st->eps, (double2 *)st->coef);
    TDX_HIP(hipGetLastError());
    g0 = g1;
  }
  int *d_flag = h.d_flag;

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
  TDX_REQUIRE(std::isfinite(st->omega_cell) && st->omega_cell > 0, TDX_ERR_INVALID_ARG,
              "states without a cell volume (build them with tdx_build_states)");
  TDX_TRY(check_device(ctx));
  return occupations_impl(ctx, st, T, ne, f_trunc, as_stream(stream));
}

int tdx_potential_vjp(tdx_ctx *ctx, const tdx_model *md, const tdx_states *st,
                      const double *eps_bar, const double *coef_bar, double *v_bar,
                      tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && st && eps_bar && coef_bar && v_bar, TDX_ERR_INVALID_ARG, "null argument");
  TDX_TRY(validate(md));
  TDX_REQUIRE(md->n_shells > 0, TDX_ERR_INVALID_ARG, "the model has no tabulated shells");
  TDX_TRY(check_device(ctx));
  hipStream_t s = as_stream(stream);
  HostBasis hb;
  TDX_TRY(host_basis(md, &hb));
  const int nk = md->kgrid[0] * md->kgrid[1] * md->kgrid[2];
  TDX_REQUIRE(st->n_k == nk && st->npw_max == hb.npw_max, TDX_ERR_SHAPE,
              "states were not built from this model's basis");
  const int npw_max = st->npw_max, nb_max = st->nb_max, ns = md->n_shells;
  HSetup h;
  TDX_TRY(h_setup(ctx, md, hb, s, &h));
  // shell vectors on the box of Miller differences
  std::vector<int> dv, ds;
  const Lattice &L = hb.L;
  for (int d0 = -h.D0; d0 <= h.D0; ++d0)
    for (int d1 = -h.D1; d1 <= h.D1; ++d1)
      for (int d2 = -h.D2; d2 <= h.D2; ++d2) {
        if (!d0 && !d1 && !d2) continue;
        double g[3];
        for (int j = 0; j < 3; ++j) g[j] = d0 * L.b[0][j] + d1 * L.b[1][j] + d2 * L.b[2][j];
        const double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        int hit = -1;
        for (int j = 0; j < ns; ++j) {
          const double s2 = md->shell_unit * md->shell_unit * md->shell_n2[j];
          if (std::fabs(g2 - s2) <= 1e-9 * s2) hit = j;
        }
        if (hit < 0) continue;
        dv.push_back(d0);
        dv.push_back(d1);
        dv.push_back(d2);
        ds.push_back(hit);
      }
  const int n_vec = (int)ds.size();
  const int M0 = st->mmax[0], M1 = st->mmax[1], M2 = st->mmax[2];
  const long box = (long)(2 * M0 + 1) * (2 * M1 + 1) * (2 * M2 + 1);
  const size_t lut_bytes = (sizeof(int) * (size_t)nk * box + 255) / 256 * 256;
  const size_t vec_bytes = (sizeof(int) * 4 * (size_t)std::max(n_vec, 1) + 255) / 256 * 256;
  const size_t sf_bytes = sizeof(double2) * (size_t)std::max(n_vec, 1);
  const size_t part_bytes = sizeof(double) * ((size_t)nk * nb_max * ns + 64);
  void *wt, *wy, *wp;
  TDX_TRY(ws_get(ctx, WS_ADJ, lut_bytes + vec_bytes + sf_bytes, &wt));
  TDX_TRY(ws_get(ctx, WS_ADJ2, sizeof(double2) * 2 * (size_t)h.kb_max * npw_max * nb_max, &wy));
  TDX_TRY(ws_get(ctx, WS_ADJ3, part_bytes, &wp));
  int *d_lut = (int *)wt;
  int *d_vec = (int *)((char *)wt + lut_bytes);
  int *d_shell = d_vec + 3 * std::max(n_vec, 1);
  double2 *d_sf = (double2 *)((char *)wt + lut_bytes + vec_bytes);
  double2 *dW = (double2 *)wy;
  double2 *dY = dW + (size_t)h.kb_max * npw_max * nb_max;
  double *d_part = (double *)wp;
  double *d_vbar = d_part + (size_t)nk * nb_max * ns;
  if (n_vec) {
    TDX_HIP(hipMemcpyAsync(d_vec, dv.data(), sizeof(int) * dv.size(), hipMemcpyHostToDevice, s));
    TDX_HIP(hipMemcpyAsync(d_shell, ds.data(), sizeof(int) * ds.size(), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_shell_sf, dim3((n_vec + 127) / 128), dim3(128), 0, s, d_vec, n_vec, h.b0,
                       h.b1, h.b2, h.pos, md->n_atoms, d_sf);
    TDX_HIP(hipGetLastError());
    TDX_HIP(hipStreamSynchronize(s));
  }
  TDX_HIP(hipMemsetAsync(d_lut, 0xff, lut_bytes, s));
  TDX_HIP(hipMemsetAsync(d_part, 0, part_bytes, s));
  hipLaunchKernelGGL(k_lut, dim3((npw_max + 255) / 256, nk), dim3(256), 0, s, st->miller, st->npw,
                     npw_max, nk, M0, M1, M2, d_lut, box);
  TDX_HIP(hipGetLastError());
  const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
  for (int g0 = 0; g0 < nk;) {
    const int n = h.npw[h.order[g0]];
    int g1 = g0;
    while (g1 < nk && h.npw[h.order[g1]] == n && g1 - g0 < h.kb_max) ++g1;
    const int nkb = g1 - g0;
    TDX_TRY(eig_batch(ctx, st->miller, npw_max, h, g0, nkb, n, s));
    for (int kk = 0; kk < nkb; ++kk) {
      const int k = h.order[g0 + kk];
      const rocblas_double_complex *psi = (const rocblas_double_complex *)(h.dA + (size_t)kk * n * n);
      rocblas_double_complex *W = (rocblas_double_complex *)(dW + (size_t)kk * nb_max * n);
      rocblas_double_complex *Y = (rocblas_double_complex *)(dY + (size_t)kk * nb_max * n);
      const rocblas_double_complex *cb =
          (const rocblas_double_complex *)(coef_bar + 2 * (size_t)k * nb_max * npw_max);
      // W = Psi^H Cbar: overlaps of the cotangent rows with every eigenvector
      TDX_REQUIRE(rocblas_zgemm(ctx->blas, rocblas_operation_conjugate_transpose,
                                rocblas_operation_none, n, nb_max, n, &one, psi, n, cb, npw_max,
                                &zero, W, n) == rocblas_status_success,
                  TDX_ERR_HIP, "rocblas_zgemm failed");
      hipLaunchKernelGGL(k_eig_scale, dim3((n + 255) / 256, nb_max), dim3(256), 0, s,
                         (double2 *)W, h.dD + (size_t)kk * n, n, nb_max, st->nb, k);
      TDX_HIP(hipGetLastError());
      // Y = Psi (F o W): y_n = sum_{m != n} psi_m <m|cbar_n> / (eps_n - eps_m)
      TDX_REQUIRE(rocblas_zgemm(ctx->blas, rocblas_operation_none, rocblas_operation_none, n,
                                nb_max, n, &one, psi, n, W, n, &zero, Y, n) ==
                      rocblas_status_success,
                  TDX_ERR_HIP, "rocblas_zgemm failed");
    }
    hipLaunchKernelGGL(k_shell_contract, dim3(nb_max, nkb), dim3(256), 0, s,
                       (const double2 *)st->coef, eps_bar, st->npw, st->nb, st->miller, nb_max,
                       npw_max, h.klist + g0, (const double2 *)dY, n, d_lut, box, M0, M1, M2,
                       d_vec, d_shell, d_sf, n_vec, ns, d_part);
    TDX_HIP(hipGetLastError());
    TDX_HIP(hipStreamSynchronize(s));
    g0 = g1;
  }
  hipLaunchKernelGGL(k_shell_sum, dim3(ns), dim3(256), 0, s, d_part, st->nb, nk, nb_max, ns,
                     d_vbar);
  TDX_HIP(hipGetLastError());
  TDX_HIP(hipMemcpyAsync(v_bar, d_vbar, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
  TDX_HIP(hipStreamSynchronize(s));
  return TDX_OK;
}

}  // extern "C"
