// The Kubo-Greenwood route (Sec. A.3, with Eqs. 8, A-1, A-2): from a
// conductivity sigma(w) in the optical limit to the scaled structure factor
// S* = v(q) S, on which the eta test, the attenuation and the way back to
// eps^{-1} and sigma (the dielectric step with q^2 = 4 pi) run unchanged;
// and the Kubo-Greenwood conductivity of the states that the route starts
// from.  FP64.
//
// The conductivity in two steps: per transition t = (k, n -> m) of the
// q = 0 list, W_t = (df / delta) (1/3) sum_a |<m|p_a|n>|^2 (one wavefront per
// transition, its lanes striding the plane waves of k: both orbitals are
// rows of the same k, so the reads are contiguous and the rows of a k stay
// in L2 across its transitions); then sigma(w) = 2 i / (Omega N_k)
// sum_t W_t / (w - delta_t + i eta) as fixed-size chunks of transitions per
// workgroup (staged in LDS, one frequency per thread) and a fixed-order sum
// of the chunk partials, so the result does not depend on scheduling.
#include <algorithm>
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

constexpr int kKgChunk = 2048;  // transitions per partial (32 KB of LDS)

// W_t for transitions [0, n): one wavefront per transition.
__global__ void __launch_bounds__(256)
    k_kg_weights(const int *tk, const int *tn, const int *tm, const double *delta,
                 const double *df, long long n, const double2 *coef, const int *miller,
                 const int *npw, int npw_max, int nb_max, int N0, int N1, int N2, double3 b0,
                 double3 b1, double3 b2, double *W) {
  const long long t = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= n) return;  // uniform across the wavefront
  const int k = tk[t];
  const int r0 = k / (N1 * N2), r1 = (k / N2) % N1, r2 = k % N2;
  const double kr0 = (2.0 * r0 + 1.0 - N0) / (2.0 * N0), kr1 = (2.0 * r1 + 1.0 - N1) / (2.0 * N1),
               kr2 = (2.0 * r2 + 1.0 - N2) / (2.0 * N2);
  const double2 *cn = coef + ((size_t)k * nb_max + tn[t]) * npw_max;
  const double2 *cm = coef + ((size_t)k * nb_max + tm[t]) * npw_max;
  const int *mk = miller + (size_t)k * npw_max * 3;
  double p[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  for (int g = lane; g < npw[k]; g += 64) {
    const double m0 = kr0 + mk[3 * g], m1 = kr1 + mk[3 * g + 1], m2 = kr2 + mk[3 * g + 2];
    const double gx = m0 * b0.x + m1 * b1.x + m2 * b2.x;
    const double gy = m0 * b0.y + m1 * b1.y + m2 * b2.y;
    const double gz = m0 * b0.z + m1 * b1.z + m2 * b2.z;
    const double2 a = cm[g], b = cn[g];
    // conj(a) b
    const double zr = a.x * b.x + a.y * b.y, zi = a.x * b.y - a.y * b.x;
    p[0][0] += gx * zr; p[0][1] += gx * zi;
    p[1][0] += gy * zr; p[1][1] += gy * zi;
    p[2][0] += gz * zr; p[2][1] += gz * zi;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      p[a][0] += __shfl_xor(p[a][0], off);
      p[a][1] += __shfl_xor(p[a][1], off);
    }
  if (lane == 0) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) s += p[a][0] * p[a][0] + p[a][1] * p[a][1];
    W[t] = df[t] / delta[t] * (s / 3.0);
  }
}

// part[c][w] = sum over chunk c of W_t / (w - delta_t + i eta); grid
// (frequency blocks, chunks), one frequency per thread.
__global__ void __launch_bounds__(256)
    k_kg_partial(const double *W, const double *delta, long long n, const double *omega, int n_w,
                 double eta, double2 *part) {
  __shared__ double sw[kKgChunk], sd[kKgChunk];
  const long long t0 = (long long)blockIdx.y * kKgChunk;
  const int len = (int)std::min<long long>(kKgChunk, n - t0);
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    sw[i] = W[t0 + i];
    sd[i] = delta[t0 + i];
  }
  __syncthreads();
  const int wi = blockIdx.x * blockDim.x + threadIdx.x;
  if (wi >= n_w) return;
  const double w = omega[wi], e2 = eta * eta;
  double sr = 0.0, si = 0.0;
  for (int i = 0; i < len; ++i) {
    // W / (x + i eta) = W (x - i eta) / (x^2 + eta^2)
    const double x = w - sd[i];
    const double c = sw[i] / (x * x + e2);
    sr += c * x;
    si -= c * eta;
  }
  part[(size_t)blockIdx.y * n_w + wi] = make_double2(sr, si);
}

// sigma[w] = i pref sum_c part[c][w], chunks in order.
__global__ void k_kg_reduce(const double2 *part, int n_chunks, int n_w, double pref,
                            double2 *sigma) {
  const int wi = blockIdx.x * blockDim.x + threadIdx.x;
  if (wi >= n_w) return;
  double sr = 0.0, si = 0.0;
  for (int c = 0; c < n_chunks; ++c) {
    const double2 v = part[(size_t)c * n_w + wi];
    sr += v.x;
    si += v.y;
  }
  sigma[wi] = make_double2(-pref * si, pref * sr);
}

size_t kg_chunks(long long n_trans) { return (size_t)((n_trans + kKgChunk - 1) / kKgChunk); }

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

size_t tdx_kg_work_bytes(int64_t n_trans, int n_w) {
  if (n_trans < 0 || n_w < 0) return 0;
  const size_t w = ((size_t)n_trans * sizeof(double) + 255) / 256 * 256;
  return w + kg_chunks(n_trans) * (size_t)n_w * sizeof(double2);
}

int tdx_kg_conductivity(tdx_ctx *ctx, const tdx_states *st, const tdx_translist *tl,
                        int64_t n_trans, const double *omega, int n_w, double eta, double *sigma,
                        void *work, size_t work_bytes, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && st && tl && omega && sigma, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_w > 0 && n_trans >= 0, TDX_ERR_SHAPE, "n_w must be positive, n_trans >= 0");
  TDX_REQUIRE(!tl->paired, TDX_ERR_INVALID_ARG,
              "the conductivity takes the full q = 0 list, not a paired one");
  TDX_REQUIRE(std::isfinite(eta) && eta > 0, TDX_ERR_INVALID_ARG, "eta must be positive");
  TDX_REQUIRE(st->omega_cell > 0 && st->n_k > 0, TDX_ERR_INVALID_ARG,
              "states without a cell volume (build them first)");
  TDX_REQUIRE(n_trans <= tl->capacity, TDX_ERR_SHAPE, "n_trans %lld exceeds the list capacity",
              (long long)n_trans);
  TDX_TRY(check_device(ctx));
  hipStream_t s = as_stream(stream);
  const double pref = 2.0 / (st->omega_cell * st->n_k);
  if (n_trans == 0) {
    // sigma = 0 without a memset: one reduction over no chunks
    hipLaunchKernelGGL(k_kg_reduce, dim3((n_w + 255) / 256), dim3(256), 0, s, nullptr, 0, n_w,
                       pref, (double2 *)sigma);
    TDX_HIP(hipGetLastError());
    return TDX_OK;
  }
  TDX_REQUIRE(work && work_bytes >= tdx_kg_work_bytes(n_trans, n_w), TDX_ERR_SHAPE,
              "work needs %zu bytes", tdx_kg_work_bytes(n_trans, n_w));
  TDX_REQUIRE(tl->k && tl->n && tl->m && tl->delta && tl->df, TDX_ERR_INVALID_ARG,
              "transition arrays missing");
  const size_t n_chunks = kg_chunks(n_trans);
  TDX_REQUIRE(n_chunks <= 65535, TDX_ERR_SHAPE, "%lld transitions exceed %d chunks",
              (long long)n_trans, 65535);
  double *W = (double *)work;
  double2 *part = (double2 *)((char *)work + ((size_t)n_trans * sizeof(double) + 255) / 256 * 256);
  const double3 b0 = make_double3(st->bvec[0], st->bvec[1], st->bvec[2]);
  const double3 b1 = make_double3(st->bvec[3], st->bvec[4], st->bvec[5]);
  const double3 b2 = make_double3(st->bvec[6], st->bvec[7], st->bvec[8]);
  const long long nb4 = (n_trans + 3) / 4;
  TDX_REQUIRE(nb4 < (1LL << 31), TDX_ERR_SHAPE, "too many transitions");
  hipLaunchKernelGGL(k_kg_weights, dim3((unsigned)nb4), dim3(256), 0, s, tl->k, tl->n, tl->m,
                     tl->delta, tl->df, (long long)n_trans, (const double2 *)st->coef, st->miller,
                     st->npw, st->npw_max, st->nb_max, st->kgrid[0], st->kgrid[1], st->kgrid[2],
                     b0, b1, b2, W);
  TDX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_kg_partial, dim3((n_w + 255) / 256, (unsigned)n_chunks), dim3(256), 0, s,
                     W, tl->delta, (long long)n_trans, omega, n_w, eta, part);
  TDX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_kg_reduce, dim3((n_w + 255) / 256), dim3(256), 0, s, part,
                     (int)n_chunks, n_w, pref, (double2 *)sigma);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

}  // extern "C"
