// chi0_GG'(q,w) = pref * sum_t df_t / (w - delta_t + i eta) rho_t(G) conj(rho_t(G'))
// (for a time-reversal-paired list each kept t carries its partner too, with
// the weight df_t [1/(w - delta_t + i eta) - 1/(w + delta_t + i eta)])
//
// A complex contraction over transitions t, run as a real GEMM on MFMA:
// for every (w, G, G') with the left operand A = w_t(w) rho_t(G) formed in
// registers,
//   Re chi0 = sum_t [Re A, Im A] . [Re rho', Im rho']
//   Im chi0 = sum_t [Re A, Im A] . [-Im rho', Re rho']
// so that a K-step of 4 in the 16x16x4 MFMA covers two transitions.
//
// This file holds the FP64 form (16x16x4 FP64 MFMA) and the entry point;
// the FP32 form is in chi0_f32.hip and the split-BF16 form in
// chi0_bf16x3.hip.
//
// Work split: a workgroup owns a 16 (G) x 16 (G') block for 32 frequencies
// (4 waves x 8) and one fixed slice of the transition list; per chunk of 32
// transitions the rho rows of both blocks and the FP64 weights of the 32
// frequencies are staged in LDS.  Slices are summed by a second kernel in a
// fixed order (no atomics: bitwise reproducible).
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace tdx {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kWPerWave = 8;                 // frequencies per wave
constexpr int kWBlock = kWaves * kWPerWave;  // frequencies per workgroup
constexpr int kTChunk = 32;                  // transitions per LDS chunk

// Partial sums part[slice][w][G][G'] (complex FP64), unscaled.
__global__ void __launch_bounds__(256)
    k_chi0_f64(const double2 *P, int ld, const double *delta, const double *df, int paired,
                long long n_trans, long long slice_len, const double *omega, int n_w, double eta,
                int n_g, double2 *part) {
  __shared__ double2 rg[kTChunk][16];       // rho_t(G) of the row block
  __shared__ double2 rgp[kTChunk][16];      // rho_t(G') of the column block
  __shared__ double2 wt[kTChunk][kWBlock];  // weights

  const int nblk = ld / 16;
  const int gb = blockIdx.y / nblk, gbp = blockIdx.y % nblk;
  const int w0 = blockIdx.x * kWBlock;
  const long long t_lo = (long long)blockIdx.z * slice_len;
  const long long t_hi = std::min(n_trans, t_lo + slice_len);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, kk = lane >> 4, part_sel = kk & 1, tsub = kk >> 1;

  f64x4 accr[kWPerWave], acci[kWPerWave];
#pragma unroll
  for (int i = 0; i < kWPerWave; ++i) {
    accr[i] = f64x4{0, 0, 0, 0};
    acci[i] = f64x4{0, 0, 0, 0};
  }

  for (long long tc = t_lo; tc < t_hi; tc += kTChunk) {
    __syncthreads();
    // stage rho rows (zero beyond the slice) and weights
    for (int e = tid; e < kTChunk * 16; e += 256) {
      const int tl = e / 16, c = e % 16;
      const long long t = tc + tl;
      double2 a = make_double2(0, 0), b = make_double2(0, 0);
      if (t < t_hi) {
        a = P[(size_t)t * ld + gb * 16 + c];
        b = P[(size_t)t * ld + gbp * 16 + c];
      }
      rg[tl][c] = a;
      rgp[tl][c] = b;
    }
    for (int e = tid; e < kTChunk * kWBlock; e += 256) {
      const int tl = e / kWBlock, wi = e % kWBlock;
      const long long t = tc + tl;
      double2 w = make_double2(0, 0);
      if (t < t_hi && w0 + wi < n_w) {
        const double om = omega[w0 + wi], d = delta[t];
        if (paired) {
          // 2 df delta / D, D = (w + i eta)^2 - delta^2 = (w - delta)(w + delta) - eta^2 + 2 i w eta
          const double dr = (om - d) * (om + d) - eta * eta, di = 2.0 * om * eta;
          const double s = 2.0 * df[t] * d / fma(dr, dr, di * di);
          w = make_double2(s * dr, -s * di);
        } else {
          // df / (x + i eta) = df (x - i eta) / (x^2 + eta^2), x = w - delta
          const double x = om - d;
          const double s = df[t] / fma(x, x, eta * eta);
          w = make_double2(s * x, -s * eta);
        }
      }
      wt[tl][wi] = w;
    }
    __syncthreads();

#pragma unroll 2
    for (int pr = 0; pr < kTChunk / 2; ++pr) {
      const int tl = 2 * pr + tsub;
      const double2 rb = rgp[tl][r];
      const double2 ra = rg[tl][r];
      const double br = part_sel ? rb.y : rb.x;
      const double bi = part_sel ? rb.x : -rb.y;
#pragma unroll
      for (int i = 0; i < kWPerWave; ++i) {
        const double2 w = wt[tl][wave * kWPerWave + i];
        const double a = part_sel ? fma(w.x, ra.y, w.y * ra.x) : fma(w.x, ra.x, -w.y * ra.y);
        accr[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, br, accr[i], 0, 0, 0);
        acci[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bi, acci[i], 0, 0, 0);
      }
    }
  }
  // D[row][col], column lane%16; element j is row lane/16 + 4j for the f64
  // 16x16x4 MFMA
  const int col = gbp * 16 + (lane & 15);
#pragma unroll
  for (int i = 0; i < kWPerWave; ++i) {
    const int w = w0 + wave * kWPerWave + i;
    if (w >= n_w) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = gb * 16 + (lane >> 4) + 4 * j;
      if (row < n_g && col < n_g)
        part[(((size_t)blockIdx.z * n_w + w) * n_g + row) * n_g + col] =
            make_double2(accr[i][j], acci[i][j]);
    }
  }
}

__global__ void k_reduce_slices(const double2 *part, int n_slices, size_t per_slice, double pref,
                                double2 *out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < per_slice;
       i += (size_t)gridDim.x * blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int s = 0; s < n_slices; ++s) {
      const double2 v = part[(size_t)s * per_slice + i];
      re += v.x;
      im += v.y;
    }
    out[i] = make_double2(pref * re, pref * im);
  }
}

}  // namespace

// FP32 path (chi0_f32.hip).
void chi0_f32_shape(int *wblock, int *cols, int *chunk);
int chi0_f32_launch(const void *P, int ld, const double *delta, const double *df, int paired,
                    long long n_trans, long long slice_len, int slices, const double *omega,
                    int n_w, double eta, int n_g, double2 *part, hipStream_t s);

// Split-BF16 path (chi0_bf16x3.hip).
int chi0_bf16x3(tdx_ctx *ctx, const void *P, int ld, const double *delta, const double *df,
                int paired, long long n_trans, const double *omega, int n_w, double eta, int n_g,
                double pref, double2 *chi0, hipStream_t s);

}  // namespace tdx

using namespace tdx;

extern "C" int tdx_chi0(tdx_ctx *ctx, const tdx_translist *tl, int64_t n_trans, const void *P,
                        int n_g, int prec, const double *omega, int n_w, double eta, double pref,
                        double *chi0, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && tl && P && omega && chi0, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(prec >= TDX_PREC_FP64 && prec <= TDX_PREC_BF16X3, TDX_ERR_INVALID_ARG, "bad prec");
  TDX_REQUIRE(n_g > 0 && n_w > 0 && n_trans >= 0 && n_trans <= tl->capacity, TDX_ERR_SHAPE,
              "bad sizes");
  TDX_REQUIRE(std::isfinite(eta) && eta > 0 && std::isfinite(pref), TDX_ERR_INVALID_ARG,
              "bad eta or prefactor");
  TDX_TRY(check_device(ctx));
  hipStream_t s = as_stream(stream);
  const int ld = (n_g + 15) / 16 * 16;
  const size_t out_elems = (size_t)n_w * n_g * n_g;
  if (n_trans == 0) {
    // a reduction over no slices writes zeros (a kernel, not a memset node,
    // so a caller may capture this call)
    const unsigned rb = (unsigned)std::min<size_t>((out_elems + 255) / 256, 8192);
    hipLaunchKernelGGL(k_reduce_slices, dim3(rb), dim3(256), 0, s, (const double2 *)nullptr, 0,
                       out_elems, pref, (double2 *)chi0);
    TDX_HIP(hipGetLastError());
    return TDX_OK;
  }
  if (prec == TDX_PREC_BF16X3)
    return chi0_bf16x3(ctx, P, ld, tl->delta, tl->df, tl->paired, n_trans, omega, n_w, eta, n_g,
                       pref,
                       (double2 *)chi0, s);
  const int nblk = ld / 16;
  int wblock = kWBlock, cols = 16, chunk = kTChunk;
  if (prec == TDX_PREC_FP32) chi0_f32_shape(&wblock, &cols, &chunk);
  const long long base =
      (long long)((n_w + wblock - 1) / wblock) * nblk * ((ld + cols - 1) / cols);
  // enough slices to fill the chip; each slice a multiple of the chunk
  long long slices = std::max<long long>(1, (4096 + base - 1) / base);
  slices = std::min<long long>(slices, (n_trans + chunk - 1) / chunk);
  slices = std::min<long long>(slices, 512);
  long long slice_len = (n_trans + slices - 1) / slices;
  slice_len = (slice_len + chunk - 1) / chunk * chunk;
  slices = (n_trans + slice_len - 1) / slice_len;
  void *w;
  TDX_TRY(ws_get(ctx, WS_PARTIAL, sizeof(double2) * out_elems * slices, &w));
  double2 *part = (double2 *)w;
  if (prec == TDX_PREC_FP64) {
    dim3 grid((n_w + kWBlock - 1) / kWBlock, nblk * nblk, (unsigned)slices);
    hipLaunchKernelGGL(k_chi0_f64, grid, dim3(256), 0, s, (const double2 *)P, ld, tl->delta,
                       tl->df, (int)tl->paired, (long long)n_trans, slice_len, omega, n_w, eta,
                       n_g, part);
  } else {
    TDX_TRY(chi0_f32_launch(P, ld, tl->delta, tl->df, (int)tl->paired, (long long)n_trans,
                            slice_len, (int)slices, omega, n_w, eta, n_g, part, s));
  }
  TDX_HIP(hipGetLastError());
  const unsigned rb = (unsigned)std::min<size_t>((out_elems + 255) / 256, 8192);
  hipLaunchKernelGGL(k_reduce_slices, dim3(rb), dim3(256), 0, s, part, (int)slices, out_elems,
                     pref, (double2 *)chi0);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}
