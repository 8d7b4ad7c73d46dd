// chi0_GG'(q,w) = pref * sum_t df_t / (w - delta_t + i eta) rho_t(G) conj(rho_t(G'))
// (for a time-reversal-paired list each kept t carries its partner too, with
// the weight df_t [1/(w - delta_t + i eta) - 1/(w + delta_t + i eta)]).
//
// The entry point and the slice reduction.  The contraction kernels: FP32 and
// FP64 in chi0_fp.hip, split-BF16 in chi0_bf16x3.hip (with its batches in
// chi0_batch.hip).  The transition axis is cut into slices whose FP64
// partials are summed here in a fixed order (no atomics: bitwise
// reproducible).
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace tdx {
namespace {

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

// FP32 and FP64 paths (chi0_fp.hip).
int chi0_fp_variant_count(bool f64);
void chi0_fp_shape(bool f64, int v, int *wblock, int *cols, int *chunk);
int chi0_fp_launch(bool f64, int v, const void *P, int ld, const double *delta, const double *df,
                   int paired, long long n_trans, long long slice_len, int slices,
                   const double *omega, int n_w, double eta, int n_g, double2 *part,
                   hipStream_t s);

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
  const bool f64 = prec == TDX_PREC_FP64;
  const int tv = ctx->tune[prec][std::min(nblk, 63)].variant;
  const int v = tv >= 0 && tv < chi0_fp_variant_count(f64) ? tv : 0;
  int wblock, cols, chunk;
  chi0_fp_shape(f64, v, &wblock, &cols, &chunk);
  const long long base =
      (long long)((n_w + wblock - 1) / wblock) * nblk * ((ld + cols - 1) / cols);
  // enough slices to fill the chip (or the context's fixed length); each
  // slice a multiple of the chunk
  long long slices = std::max<long long>(1, (4096 + base - 1) / base);
  slices = std::min<long long>(slices, (n_trans + chunk - 1) / chunk);
  slices = std::min<long long>(slices, 512);
  long long slice_len = (n_trans + slices - 1) / slices;
  if (ctx->slice_len > 0) slice_len = ctx->slice_len;
  slice_len = (slice_len + chunk - 1) / chunk * chunk;
  slices = (n_trans + slice_len - 1) / slice_len;
  TDX_REQUIRE(slices <= 65535, TDX_ERR_SHAPE, "%lld slices exceed the grid (slice length %lld)",
              slices, slice_len);
  void *w;
  TDX_TRY(ws_get(ctx, WS_PARTIAL, sizeof(double2) * out_elems * slices, &w));
  double2 *part = (double2 *)w;
  TDX_TRY(chi0_fp_launch(f64, v, P, ld, tl->delta, tl->df, (int)tl->paired, (long long)n_trans,
                         slice_len, (int)slices, omega, n_w, eta, n_g, part, s));
  TDX_HIP(hipGetLastError());
  const unsigned rb = (unsigned)std::min<size_t>((out_elems + 255) / 256, 8192);
  hipLaunchKernelGGL(k_reduce_slices, dim3(rb), dim3(256), 0, s, part, (int)slices, out_elems,
                     pref, (double2 *)chi0);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}
