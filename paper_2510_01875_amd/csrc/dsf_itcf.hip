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

}  // extern "C"
