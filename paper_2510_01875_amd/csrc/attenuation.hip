// Constraints-based attenuation of narrow-band fluctuations (Sec. 3,
// Eqs. 3-7, Figs. 3 and 4): a bank of Savitzky-Golay filters applied to S on
// the frequency grid, the scores of the window/degree grid search (AICc, a
// frequency-domain penalty at the fluctuations' frequencies found from the
// spectrum of dS/dw, a curvature penalty), the imaginary-time conditions on
// the residual F_n = F_TDDFT - F_p, and the selection.  All FP64; every
// reduction is a fixed-order tree, so results are bitwise reproducible.
#include <cmath>

#include "internal.h"

namespace tdx {
namespace {

constexpr int kSgMaxDeg = 8;
constexpr int kRedThreads = 256;
constexpr int kMaxTargets = 16;

// Fixed-order sum over the block (blockDim.x == kRedThreads); every thread
// gets the total.
__device__ double block_sum(double v, double *sh) {
  __syncthreads();
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// Output point i of the degree-P filter with w-point windows: the
// least-squares polynomial over the window centred on i (moved inside the
// grid at the edges) evaluated at i, and the weight of S_i in that value
// (diagonal of the smoother).  Coordinates t = (j - c) / a with c the window
// centre and a = max(c, 1) keep the Gram matrix well scaled; it is factored
// by Cholesky, value = u.v and weight = u.u with L u = phi(t_i), L v = rhs.
template <int P>
__device__ void sg_point(const double *S, int n, int w, int i, double *out, double *hii) {
  constexpr int M = P + 1;
  const int h = w / 2;
  const int s = min(max(i - h, 0), n - w);
  const double c = 0.5 * (w - 1), a = fmax(c, 1.0);
  double G[M][M], r[M];
#pragma unroll
  for (int x = 0; x < M; ++x) {
    r[x] = 0.0;
#pragma unroll
    for (int y = 0; y < M; ++y) G[x][y] = 0.0;
  }
  for (int j = 0; j < w; ++j) {
    const double t = (j - c) / a, yj = S[s + j];
    double ph[M];
    ph[0] = 1.0;
#pragma unroll
    for (int x = 1; x < M; ++x) ph[x] = ph[x - 1] * t;
#pragma unroll
    for (int x = 0; x < M; ++x) {
      r[x] += ph[x] * yj;
#pragma unroll
      for (int y = 0; y <= x; ++y) G[x][y] += ph[x] * ph[y];
    }
  }
  // Cholesky G = L L^T in the lower triangle
#pragma unroll
  for (int k = 0; k < M; ++k) {
    double d = G[k][k];
#pragma unroll
    for (int l = 0; l < k; ++l) d -= G[k][l] * G[k][l];
    const double lkk = sqrt(d);
    G[k][k] = lkk;
#pragma unroll
    for (int x = k + 1; x < M; ++x) {
      double e = G[x][k];
#pragma unroll
      for (int l = 0; l < k; ++l) e -= G[x][l] * G[k][l];
      G[x][k] = e / lkk;
    }
  }
  const double ti = (i - s - c) / a;
  double u[M], v[M];
  double p = 1.0;
#pragma unroll
  for (int x = 0; x < M; ++x) {
    double eu = p, ev = r[x];
#pragma unroll
    for (int l = 0; l < x; ++l) {
      eu -= G[x][l] * u[l];
      ev -= G[x][l] * v[l];
    }
    u[x] = eu / G[x][x];
    v[x] = ev / G[x][x];
    p *= ti;
  }
  double val = 0.0, hw = 0.0;
#pragma unroll
  for (int x = 0; x < M; ++x) {
    val += u[x] * v[x];
    hw += u[x] * u[x];
  }
  *out = val;
  *hii = hw;
}

// grid (ceil(n / 256), n_filt): filter f = blockIdx.y, point i.
__global__ void __launch_bounds__(256)
    k_sg_filter(const double *S, int n, const int *win, const int *deg, double *Sp,
                double *hdiag) {
  const int f = blockIdx.y, i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int w = win[f];
  double val = 0.0, hw = 0.0;
  switch (deg[f]) {  // uniform over the block
    case 0: sg_point<0>(S, n, w, i, &val, &hw); break;
    case 1: sg_point<1>(S, n, w, i, &val, &hw); break;
    case 2: sg_point<2>(S, n, w, i, &val, &hw); break;
    case 3: sg_point<3>(S, n, w, i, &val, &hw); break;
    case 4: sg_point<4>(S, n, w, i, &val, &hw); break;
    case 5: sg_point<5>(S, n, w, i, &val, &hw); break;
    case 6: sg_point<6>(S, n, w, i, &val, &hw); break;
    case 7: sg_point<7>(S, n, w, i, &val, &hw); break;
    default: sg_point<8>(S, n, w, i, &val, &hw); break;
  }
  Sp[(size_t)f * n + i] = val;
  if (hdiag) hdiag[(size_t)f * n + i] = hw;
}

// Power of the central-difference derivative D_i = (y_{i+1} - y_{i-1}) /
// (w_{i+1} - w_{i-1}), i = 1..n-2, at frequency nu (cycles per unit of w):
// |(1/(n-2)) sum_i D_i exp(-2 pi i nu w_i)|^2.  Block-wide.
__device__ double deriv_power(const double *y, const double *om, int n, double nu, double *sh) {
  double re = 0.0, im = 0.0;
  for (int i = 1 + threadIdx.x; i + 1 < n; i += kRedThreads) {
    const double d = (y[i + 1] - y[i - 1]) / (om[i + 1] - om[i - 1]);
    double sn, cs;
    sincospi(-2.0 * nu * om[i], &sn, &cs);
    re += d * cs;
    im += d * sn;
  }
  re = block_sum(re, sh);
  im = block_sum(im, sh);
  const double m = (double)(n - 2);
  return (re * re + im * im) / (m * m);
}

// one block per (set, nu): psd[set][k]
__global__ void __launch_bounds__(kRedThreads)
    k_deriv_psd(const double *S, const double *om, int n, const double *nu, int n_nu,
                double *psd) {
  __shared__ double sh[kRedThreads];
  const int k = blockIdx.x, set = blockIdx.y;
  const double p = deriv_power(S + (size_t)set * n, om, n, nu[k], sh);
  if (threadIdx.x == 0) psd[(size_t)set * n_nu + k] = p;
}

// one block per filter: scores[f] = (RSS, k_eff, AICc, P_freq, P_curv)
__global__ void __launch_bounds__(kRedThreads)
    k_sg_scores(const double *S, const double *Sp, const double *hdiag, const double *om, int n,
                const double *nu, int n_nu, double *scores) {
  __shared__ double sh[kRedThreads];
  const int f = blockIdx.x;
  const double *y = Sp + (size_t)f * n, *hd = hdiag + (size_t)f * n;
  double rss = 0.0, k = 0.0, c_p = 0.0, c_0 = 0.0;
  for (int i = threadIdx.x; i < n; i += kRedThreads) {
    const double e = y[i] - S[i];
    rss += e * e;
    k += hd[i];
    if (i > 0 && i + 1 < n) {
      const double a = y[i + 1] - 2.0 * y[i] + y[i - 1];
      const double b = S[i + 1] - 2.0 * S[i] + S[i - 1];
      c_p += a * a;
      c_0 += b * b;
    }
  }
  rss = block_sum(rss, sh);
  k = block_sum(k, sh);
  c_p = block_sum(c_p, sh);
  c_0 = block_sum(c_0, sh);
  double pf = 0.0;
  for (int t = 0; t < n_nu; ++t)
    pf += deriv_power(y, om, n, nu[t], sh) / deriv_power(S, om, n, nu[t], sh);
  if (threadIdx.x == 0) {
    const double dn = (double)n, den = dn - k - 1.0;
    const double aicc = den > 0.0 ? dn * log(rss / dn) + 2.0 * k + 2.0 * k * (k + 1.0) / den
                                  : INFINITY;
    double *o = scores + (size_t)f * 5;
    o[0] = rss;
    o[1] = k;
    o[2] = aicc;
    o[3] = n_nu > 0 ? pf / n_nu : 0.0;
    o[4] = c_0 > 0.0 ? c_p / c_0 : NAN;
  }
}

// one block per set: out[set] = (max |F_n / F_ref|, Fbar_n / F_ref(beta/2),
// sigma_n / F_ref(beta/2)), F_n = F_ref - F_p[set]; NaN for a grid that does
// not start at 0, end at beta/2 or beta, and hold beta/2.
__global__ void __launch_bounds__(kRedThreads)
    k_residual_itcf(const double *Fr, const double *Fp, const double *tau, int n_tau,
                    double beta, double *out) {
  __shared__ double sh[kRedThreads];
  const int set = blockIdx.x;
  const double *fp = Fp + (size_t)set * n_tau;
  const double tol = 1e-12 * beta;
  const double t_end = tau[n_tau - 1];
  const bool half = fabs(t_end - 0.5 * beta) <= tol, full = fabs(t_end - beta) <= tol;
  // integrals over the grid; a grid ending at beta/2 covers half of [0, beta]
  // and F_n(tau) = F_n(beta - tau) for every S, so each doubles
  const double span = half ? 0.5 * beta : beta;
  double a = 0.0, e = 0.0;
  for (int j = threadIdx.x; j < n_tau; j += kRedThreads) {
    const double d = Fr[j] - fp[j];
    e = fmax(e, fabs(d / Fr[j]));
    if (j + 1 < n_tau) a += 0.5 * (tau[j + 1] - tau[j]) * (d + (Fr[j + 1] - fp[j + 1]));
  }
  a = block_sum(a, sh);
  const double mean = a / span;
  double q = 0.0;
  for (int j = threadIdx.x; j + 1 < n_tau; j += kRedThreads) {
    const double d0 = Fr[j] - fp[j] - mean, d1 = Fr[j + 1] - fp[j + 1] - mean;
    q += 0.5 * (tau[j + 1] - tau[j]) * (d0 * d0 + d1 * d1);
  }
  q = block_sum(q, sh);
  // max over the block by the same tree (all values are >= 0)
  __syncthreads();
  sh[threadIdx.x] = e;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int mid = -1;
    for (int j = 0; j < n_tau; ++j)
      if (fabs(tau[j] - 0.5 * beta) <= tol) mid = j;
    const bool ok = n_tau > 1 && tau[0] == 0.0 && (half || full) && mid >= 0;
    const double fm = ok ? Fr[mid] : NAN;
    // root-mean-square deviation over [0, beta]: the integral over the grid
    // is q * beta / span, its mean over [0, beta] q / span
    const double sigma = sqrt(q / span);
    double *o = out + (size_t)set * 3;
    o[0] = ok ? sh[0] : NAN;
    o[1] = ok ? mean / fm : NAN;
    o[2] = ok ? sigma / fm : NAN;
  }
}

}  // namespace
}  // namespace tdx

using namespace tdx;

extern "C" {

int tdx_sg_filter(tdx_ctx *ctx, const double *S, int n_w, const int *windows,
                  const int *degrees, int n_filt, double *Sp, double *hdiag, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && S && (n_filt == 0 || (windows && degrees && Sp)), TDX_ERR_INVALID_ARG,
              "null argument");
  TDX_REQUIRE(n_w > 0 && n_filt >= 0, TDX_ERR_SHAPE, "bad sizes");
  for (int f = 0; f < n_filt; ++f) {
    const int w = windows[f], p = degrees[f];
    TDX_REQUIRE(p >= 0 && p <= kSgMaxDeg, TDX_ERR_INVALID_ARG,
                "filter %d: degree %d outside 0..%d", f, p, kSgMaxDeg);
    TDX_REQUIRE(w % 2 == 1 && w > p && w <= n_w, TDX_ERR_INVALID_ARG,
                "filter %d: window %d must be odd, above the degree %d and at most %d", f, w,
                p, n_w);
  }
  TDX_TRY(check_device(ctx));
  if (n_filt == 0) return TDX_OK;
  hipStream_t s = as_stream(stream);
  void *w1;
  TDX_TRY(ws_get(ctx, WS_SG, sizeof(int) * 2 * (size_t)n_filt, &w1));
  int *d_win = (int *)w1, *d_deg = d_win + n_filt;
  TDX_HIP(hipMemcpyAsync(d_win, windows, sizeof(int) * n_filt, hipMemcpyHostToDevice, s));
  TDX_HIP(hipMemcpyAsync(d_deg, degrees, sizeof(int) * n_filt, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_sg_filter, dim3((n_w + 255) / 256, n_filt), dim3(256), 0, s, S, n_w,
                     d_win, d_deg, Sp, hdiag);
  TDX_HIP(hipGetLastError());
  // the window and degree lists are pageable host memory copied on the stream
  TDX_HIP(hipStreamSynchronize(s));
  return TDX_OK;
}

int tdx_derivative_psd(tdx_ctx *ctx, const double *S, const double *omega, int n_w, int n_set,
                       const double *nu, int n_nu, double *psd, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && S && omega && ((n_set == 0 || n_nu == 0) || (nu && psd)),
              TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_w >= 3 && n_set >= 0 && n_nu >= 0, TDX_ERR_SHAPE, "bad sizes");
  TDX_TRY(check_device(ctx));
  if (n_set == 0 || n_nu == 0) return TDX_OK;
  hipLaunchKernelGGL(k_deriv_psd, dim3(n_nu, n_set), dim3(kRedThreads), 0, as_stream(stream), S,
                     omega, n_w, nu, n_nu, psd);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

int tdx_sg_scores(tdx_ctx *ctx, const double *S, const double *Sp, const double *hdiag,
                  const double *omega, int n_w, int n_filt, const double *nu, int n_nu,
                  double *scores, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && S && omega && (nu || n_nu == 0) && (n_filt == 0 || (Sp && hdiag && scores)),
              TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_w >= 3 && n_filt >= 0, TDX_ERR_SHAPE, "bad sizes");
  TDX_REQUIRE(n_nu >= 0 && n_nu <= kMaxTargets, TDX_ERR_SHAPE, "at most %d target frequencies",
              kMaxTargets);
  TDX_TRY(check_device(ctx));
  if (n_filt == 0) return TDX_OK;
  hipLaunchKernelGGL(k_sg_scores, dim3(n_filt), dim3(kRedThreads), 0, as_stream(stream), S, Sp,
                     hdiag, omega, n_w, nu, n_nu, scores);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

int tdx_residual_itcf(tdx_ctx *ctx, const double *F_ref, const double *F_p, int n_set,
                      const double *tau, int n_tau, double beta, double *out,
                      tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && F_ref && tau && (n_set == 0 || (F_p && out)), TDX_ERR_INVALID_ARG,
              "null argument");
  TDX_REQUIRE(n_tau > 1 && n_set >= 0, TDX_ERR_SHAPE, "bad sizes");
  TDX_REQUIRE(std::isfinite(beta) && beta > 0, TDX_ERR_INVALID_ARG, "bad beta");
  TDX_TRY(check_device(ctx));
  if (n_set == 0) return TDX_OK;
  hipLaunchKernelGGL(k_residual_itcf, dim3(n_set), dim3(kRedThreads), 0, as_stream(stream),
                     F_ref, F_p, tau, n_tau, beta, out);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

int tdx_sg_select(const double *scores, const double *resid, int n_filt, int n_w, double lam_f,
                  double lam_c, double mean_tol, double sigma_tol, int *best) {
  clear_error();
  TDX_REQUIRE(best && (scores || n_filt == 0), TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_filt >= 0 && n_w > 0, TDX_ERR_SHAPE, "bad sizes");
  TDX_REQUIRE(std::isfinite(lam_f) && lam_f >= 0 && std::isfinite(lam_c) && lam_c >= 0,
              TDX_ERR_INVALID_ARG, "penalty weights must be finite and non-negative");
  int b = -1;
  double jb = INFINITY;
  for (int f = 0; f < n_filt; ++f) {
    const double *o = scores + 5 * (size_t)f;
    const double J = o[2] / n_w + lam_f * o[3] + lam_c * o[4];
    if (!std::isfinite(J)) continue;
    if (resid) {
      const double *r = resid + 3 * (size_t)f;
      if (!(fabs(r[1]) <= mean_tol && r[2] <= sigma_tol)) continue;
    }
    if (J < jb) {
      jb = J;
      b = f;
    }
  }
  *best = b;
  return TDX_OK;
}

}  // extern "C"
