// S(q,w) by the fluctuation-dissipation theorem (Eq. 8) and F(q,tau) by the
// two-sided Laplace transform (Eq. 1) with detailed balance, both FP64.
#include <cmath>

#include "internal.h"

namespace tdx {
namespace {

// S = -Im chi / (pi n (1 - e^{-beta w})); w = 0 takes the limit from the
// next grid point, -Im chi(w1) / (pi n beta w1).
__global__ void k_dsf(const double2 *chi, const double *w, int n, double beta, double dens,
                      double *S) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double wi = w[i];
  double v;
  if (wi != 0.0) {
    v = -chi[i].y / (M_PI * dens * (-expm1(-beta * wi)));
  } else if (i + 1 < n && w[i + 1] > 0.0) {
    v = -chi[i + 1].y / (M_PI * dens * beta * w[i + 1]);
  } else {
    v = NAN;  // w = 0 without a positive neighbour
  }
  S[i] = v;
}

// F(tau) = sum_j c_j S_j (e^{-tau w_j} + e^{-(beta - tau) w_j}), one block
// per tau, fixed-order tree reduction.
__global__ void __launch_bounds__(256)
    k_itcf(const double *S, const double *w, int n, double beta, const double *tau, double *F) {
  __shared__ double sh[256];
  const int it = blockIdx.x;
  const double t = tau[it];
  double acc = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) {
    double c = 0.0;
    if (j > 0) c += 0.5 * (w[j] - w[j - 1]);
    if (j + 1 < n) c += 0.5 * (w[j + 1] - w[j]);
    acc += c * S[j] * (exp(-t * w[j]) + exp(-(beta - t) * w[j]));
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) F[it] = sh[0];
}

// Imaginary-time metrics of one ITCF per block (Sec. 2, Eq. 2):
//   m[0] = F(beta/2), m[1] = A = int_0^beta F dtau, m[2] = F~(beta/2),
//   m[3] = int_0^beta F~ dtau = A - beta F(0), m[4] = chi(q) = -n A,
// with F~(tau) = F(tau) - F(0) and the integral by the composite trapezoid
// on the tau grid.  A grid ending at beta/2 stands for [0, beta] by the
// symmetry F(tau) = F(beta - tau) (the integral doubles).  A grid that does
// not start at 0, end at beta/2 or beta, or hold beta/2 gives NaN.
__global__ void __launch_bounds__(64)
    k_itcf_metrics(const double *F, int n_tau, const double *tau, double beta, double dens,
                   double *m) {
  __shared__ double sh[64];
  const int set = blockIdx.x;
  const double *f = F + (size_t)set * n_tau;
  const double tol = 1e-12 * beta;
  const double t_end = tau[n_tau - 1];
  const bool half = fabs(t_end - 0.5 * beta) <= tol, full = fabs(t_end - beta) <= tol;
  double acc = 0.0;
  for (int j = threadIdx.x; j + 1 < n_tau; j += 64)
    acc += 0.5 * (tau[j + 1] - tau[j]) * (f[j] + f[j + 1]);
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 32; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int mid = -1;
    for (int j = 0; j < n_tau; ++j)
      if (fabs(tau[j] - 0.5 * beta) <= tol) mid = j;
    const bool ok = n_tau > 1 && tau[0] == 0.0 && (half || full) && mid >= 0;
    const double A = (half ? 2.0 : 1.0) * sh[0];
    const double f0 = f[0], fm = ok ? f[mid] : NAN;
    double *o = m + (size_t)set * 5;
    o[0] = ok ? fm : NAN;
    o[1] = ok ? A : NAN;
    o[2] = ok ? fm - f0 : NAN;
    o[3] = ok ? A - beta * f0 : NAN;
    o[4] = ok ? -dens * A : NAN;
  }
}

// Im chi at grid point j from S by the FDT (Eq. 8): -pi n (1 - e^{-beta w}) S.
__device__ inline double im_chi_of(const double *S, const double *w, int j, double beta,
                                   double dens) {
  return -M_PI * dens * (-expm1(-beta * w[j])) * S[j];
}

// Per frequency w_i (one block): chi(w_i) with Im chi from S and Re chi by
// the Kramers-Kronig relation
//   Re chi(w) = (1/pi) P int_0^wmax f(w') [1/(w' - w) + 1/(w' + w)] dw',
// f = Im chi linear between grid points, so that on [a, b] with slope s
//   int f(w') / (w' - c) dw' = f(c) (ln|b - c| - ln|a - c|) + s (b - a);
// the logarithms of zero at c = w_i cancel between the two intervals that
// meet there (f is continuous), which is the principal value, so they are
// left out.  Then eps^{-1} = 1 + (4 pi / q^2) chi (Eq. A-1) and
// sigma = -i w (eps - 1) / (4 pi) (Eq. A-2).  Fixed-order reduction.
__global__ void __launch_bounds__(256)
    k_dielectric(const double *S, const double *w, int n, double beta, double dens, double q2,
                 double2 *chi, double2 *eps_inv, double2 *sigma) {
  __shared__ double sh[256];
  const int i = blockIdx.x;
  const double wi = w[i];
  double acc = 0.0;
  for (int j = threadIdx.x; j + 1 < n; j += 256) {
    const double a = w[j], b = w[j + 1], fa = im_chi_of(S, w, j, beta, dens),
                 fb = im_chi_of(S, w, j + 1, beta, dens);
    const double sl = (fb - fa) / (b - a);
    double t = 2.0 * sl * (b - a);
    const double cs[2] = {wi, -wi};
    for (int k = 0; k < 2; ++k) {
      const double c = cs[k], fc = fa + sl * (c - a);
      const double lb = b != c ? log(fabs(b - c)) : 0.0, la = a != c ? log(fabs(a - c)) : 0.0;
      t += fc * (lb - la);
    }
    acc += t;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double re = sh[0] / M_PI, im = im_chi_of(S, w, i, beta, dens);
    const double v = 4.0 * M_PI / q2;
    const double er = 1.0 + v * re, ei = v * im;  // eps^{-1}
    const double d = er * er + ei * ei;
    const double pr = er / d - 1.0, pi = -ei / d;  // eps - 1
    if (chi) chi[i] = make_double2(re, im);
    if (eps_inv) eps_inv[i] = make_double2(er, ei);
    if (sigma) sigma[i] = make_double2(wi * pi / (4.0 * M_PI), -wi * pr / (4.0 * M_PI));
  }
}

}  // namespace
}  // namespace tdx

using namespace tdx;

extern "C" {

int tdx_dsf(tdx_ctx *ctx, const double *chi00, const double *omega, int n_w, double beta,
            double density, double *S, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && chi00 && omega && S, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_w > 0, TDX_ERR_SHAPE, "n_w must be positive");
  TDX_REQUIRE(std::isfinite(beta) && beta > 0 && std::isfinite(density) && density > 0,
              TDX_ERR_INVALID_ARG, "bad beta or density");
  TDX_TRY(check_device(ctx));
  hipStream_t s = as_stream(stream);
  hipLaunchKernelGGL(k_dsf, dim3((n_w + 255) / 256), dim3(256), 0, s, (const double2 *)chi00,
                     omega, n_w, beta, density, S);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

int tdx_itcf(tdx_ctx *ctx, const double *S, const double *omega, int n_w, double beta,
             const double *tau, int n_tau, double *F, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && S && omega && tau && F, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_w > 0 && n_tau > 0, TDX_ERR_SHAPE, "bad sizes");
  TDX_REQUIRE(std::isfinite(beta) && beta > 0, TDX_ERR_INVALID_ARG, "bad beta");
  hipLaunchKernelGGL(k_itcf, dim3(n_tau), dim3(256), 0, as_stream(stream), S, omega, n_w, beta,
                     tau, F);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

int tdx_itcf_metrics(tdx_ctx *ctx, const double *F, int n_set, const double *tau, int n_tau,
                     double beta, double density, double *metrics, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && F && tau && metrics, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_set > 0 && n_tau > 1, TDX_ERR_SHAPE, "bad sizes");
  TDX_REQUIRE(std::isfinite(beta) && beta > 0 && std::isfinite(density) && density > 0,
              TDX_ERR_INVALID_ARG, "bad beta or density");
  TDX_TRY(check_device(ctx));
  hipLaunchKernelGGL(k_itcf_metrics, dim3(n_set), dim3(64), 0, as_stream(stream), F, n_tau, tau,
                     beta, density, metrics);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

int tdx_dielectric(tdx_ctx *ctx, const double *S, const double *omega, int n_w, double beta,
                   double density, double q2, double *chi, double *eps_inv, double *sigma,
                   tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && S && omega, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_w > 1, TDX_ERR_SHAPE, "need at least two frequencies");
  TDX_REQUIRE(std::isfinite(beta) && beta > 0 && std::isfinite(density) && density > 0 &&
                  std::isfinite(q2) && q2 > 0,
              TDX_ERR_INVALID_ARG, "bad beta, density or q^2");
  TDX_TRY(check_device(ctx));
  hipLaunchKernelGGL(k_dielectric, dim3(n_w), dim3(256), 0, as_stream(stream), S, omega, n_w,
                     beta, density, q2, (double2 *)chi, (double2 *)eps_inv, (double2 *)sigma);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

int tdx_eta_reference(const double *metrics, const double *eta, int n_eta, double tol,
                      int *ref_index) {
  clear_error();
  TDX_REQUIRE(metrics && eta && ref_index, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_eta > 0, TDX_ERR_SHAPE, "n_eta must be positive");
  TDX_REQUIRE(std::isfinite(tol) && tol >= 0, TDX_ERR_INVALID_ARG, "bad tolerance");
  for (int i = 0; i < n_eta; ++i) {
    TDX_REQUIRE(std::isfinite(eta[i]) && eta[i] > 0 && (i == 0 || eta[i] > eta[i - 1]),
                TDX_ERR_INVALID_ARG, "eta must be positive and increasing");
    for (int c = 0; c < 5; ++c)
      TDX_REQUIRE(std::isfinite(metrics[5 * i + c]), TDX_ERR_NUMERIC,
                  "metric %d of eta %d is not finite", c, i);
  }
  const double a0 = metrics[2], b0 = metrics[3];
  int ref = 0;
  for (int i = 1; i < n_eta; ++i) {
    const double a = metrics[5 * i + 2], b = metrics[5 * i + 3];
    if (fabs(a - a0) > tol * fabs(a0) || fabs(b - b0) > tol * fabs(b0)) break;
    ref = i;
  }
  *ref_index = ref;
  return TDX_OK;
}

}  // extern "C"
