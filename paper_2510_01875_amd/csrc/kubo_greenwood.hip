// The Kubo-Greenwood route (Sec. A.3, with Eqs. 8, A-1, A-2): from a
// conductivity sigma(w) in the optical limit to the scaled structure factor
// S* = v(q) S, on which the eta test, the attenuation and the way back to
// eps^{-1} and sigma (the dielectric step with q^2 = 4 pi) run unchanged.
// FP64.
#include <cmath>

#include "internal.h"

namespace tdx {
namespace {

// Im chi* = Im 1/eps with eps = 1 + 4 pi i sigma / w (w != 0):
// eps = (1 - 4 pi Im sigma / w) + i (4 pi Re sigma / w), Im 1/eps = -Im eps / |eps|^2.
__device__ inline double im_chi_star(double2 s, double w) {
  const double er = 1.0 - 4.0 * M_PI * s.y / w, ei = 4.0 * M_PI * s.x / w;
  return -ei / (er * er + ei * ei);
}

// S* = -Im chi* / (pi n (1 - e^{-beta w})), the normalisation of S; w = 0
// takes the limit from the next grid point, -Im chi*(w1) / (pi n beta w1).
__global__ void k_kg_dsf(const double2 *sig, const double *w, int n, double beta, double dens,
                         double *S) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double wi = w[i];
  double v;
  if (wi != 0.0) {
    v = -im_chi_star(sig[i], wi) / (M_PI * dens * (-expm1(-beta * wi)));
  } else if (i + 1 < n && w[i + 1] > 0.0) {
    v = -im_chi_star(sig[i + 1], w[i + 1]) / (M_PI * dens * beta * w[i + 1]);
  } else {
    v = NAN;  // w = 0 without a positive neighbour
  }
  S[i] = v;
}

}  // namespace
}  // namespace tdx

using namespace tdx;

extern "C" {

int tdx_kg_dsf(tdx_ctx *ctx, const double *sigma, const double *omega, int n_w, double beta,
               double density, double *S_star, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && sigma && omega && S_star, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_w > 0, TDX_ERR_SHAPE, "n_w must be positive");
  TDX_REQUIRE(std::isfinite(beta) && beta > 0 && std::isfinite(density) && density > 0,
              TDX_ERR_INVALID_ARG, "bad beta or density");
  TDX_TRY(check_device(ctx));
  hipLaunchKernelGGL(k_kg_dsf, dim3((n_w + 255) / 256), dim3(256), 0, as_stream(stream),
                     (const double2 *)sigma, omega, n_w, beta, density, S_star);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

}  // extern "C"
