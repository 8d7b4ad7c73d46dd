// Split-BF16 chi0 contraction on the 16x16x32 bf16 MFMA of gfx950.
//
// Every real operand x is carried as x = hi + lo (bf16, round to nearest
// even) and a product as hi*hi' + hi*lo' + lo*hi' accumulated in FP32; the
// dropped lo*lo' term and the two roundings leave a relative error near
// 2^-16 per product.  The left operand A = w_t(w) rho_t(G) is formed in FP32
// from the FP64 weight and the stored pair density, then split.
//
// Layout of one MFMA (K = 32 real = 16 transitions, re/im interleaved):
//   A[G][2t + p] = (Re, Im)(w_t rho_t(G)),
//   B_re[2t + p][G'] = (Re, Im) rho_t(G'),  B_im[2t + p][G'] = (-Im, Re) rho_t(G'),
// so that D_re = Re chi0 and D_im = Im chi0.
//
// A workgroup owns 16 G x 64 G' for 16 frequencies (4 waves x 4) over one
// slice of transitions; 64 transitions per LDS chunk.  FP32 sums run in two
// levels (flushed every kFlush transitions) and slices are reduced in FP64.
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace tdx {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWPerWave = 4;
constexpr int kWBlock = 16;   // 4 waves x 4 frequencies
constexpr int kCols = 64;     // G' per workgroup (4 sub-blocks of 16)
constexpr int kSub = 4;
constexpr int kChunk = 64;    // transitions per LDS chunk
constexpr int kFlush = 1024;  // transitions per inner FP32 partial

__device__ inline bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// (re | im << 16) -> (-im | re << 16)
__device__ inline unsigned int rot_neg(unsigned int w) {
  return ((w >> 16) ^ 0x8000u) | (w << 16);
}

__device__ inline unsigned int pack_bf16(float lo_elem, float hi_elem) {
  const __bf16 a = (__bf16)lo_elem, b = (__bf16)hi_elem;  // RNE on gfx950
  return (unsigned int)__builtin_bit_cast(unsigned short, a) |
         ((unsigned int)__builtin_bit_cast(unsigned short, b) << 16);
}

__device__ inline float lo_f(unsigned int w) { return __uint_as_float(w << 16); }
__device__ inline float hi_f(unsigned int w) { return __uint_as_float(w & 0xffff0000u); }

__global__ void __launch_bounds__(256)
    k_chi0_bf16x3(const uint2 *P, int ld, const double *delta, const double *df,
                  long long n_trans, long long slice_len, const double *omega, int n_w,
                  double eta, int n_g, int nblk4, double2 *part) {
  __shared__ uint2 cq[kChunk][kCols];           // (re_hi|im_hi, re_lo|im_lo) of G' block
  __shared__ float2 rq[kChunk][16];             // rho_t(G) = hi + lo (FP32) of G block
  __shared__ float2 wt[kChunk][kWBlock];        // weights (FP32 from FP64)

  const int gb = blockIdx.y / nblk4, gc = blockIdx.y % nblk4;
  const int col0 = gc * kCols;
  const int w0 = blockIdx.x * kWBlock;
  const long long t_lo = (long long)blockIdx.z * slice_len;
  const long long t_hi = std::min(n_trans, t_lo + slice_len);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, kq = lane >> 4;

  f32x4 sr[kWPerWave][kSub], si[kWPerWave][kSub];  // inner partials
  f32x4 br[kWPerWave][kSub], bi[kWPerWave][kSub];  // outer sums
#pragma unroll
  for (int i = 0; i < kWPerWave; ++i)
#pragma unroll
    for (int b = 0; b < kSub; ++b) {
      sr[i][b] = f32x4{0, 0, 0, 0};
      si[i][b] = f32x4{0, 0, 0, 0};
      br[i][b] = f32x4{0, 0, 0, 0};
      bi[i][b] = f32x4{0, 0, 0, 0};
    }
  int since = 0;

  for (long long tc = t_lo; tc < t_hi; tc += kChunk) {
    __syncthreads();
    for (int e = tid; e < kChunk * kCols; e += 256) {
      const int tl = e / kCols, c = e % kCols;
      const long long t = tc + tl;
      uint2 v = make_uint2(0u, 0u);
      if (t < t_hi && col0 + c < ld) v = P[(size_t)t * ld + col0 + c];
      cq[tl][c] = v;
    }
    for (int e = tid; e < kChunk * 16; e += 256) {
      const int tl = e / 16, c = e % 16;
      const long long t = tc + tl;
      float2 v = make_float2(0.f, 0.f);
      if (t < t_hi) {
        const uint2 q = P[(size_t)t * ld + gb * 16 + c];
        v = make_float2(lo_f(q.x) + lo_f(q.y), hi_f(q.x) + hi_f(q.y));
      }
      rq[tl][c] = v;
    }
    for (int e = tid; e < kChunk * kWBlock; e += 256) {
      const int tl = e / kWBlock, wi = e % kWBlock;
      const long long t = tc + tl;
      float2 w = make_float2(0.f, 0.f);
      if (t < t_hi && w0 + wi < n_w) {
        const double x = omega[w0 + wi] - delta[t];
        const double s = df[t] / fma(x, x, eta * eta);
        w = make_float2((float)(s * x), (float)(-s * eta));
      }
      wt[tl][wi] = w;
    }
    __syncthreads();

    for (int step = 0; step < kChunk / 16; ++step) {
      const int tb = step * 16 + 4 * kq;  // this lane's four transitions
      u32x4 bhr[kSub], blr[kSub], bhi[kSub], bli[kSub];
#pragma unroll
      for (int b = 0; b < kSub; ++b) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint2 q = cq[tb + j][b * 16 + r];
          bhr[b][j] = q.x;
          blr[b][j] = q.y;
          bhi[b][j] = rot_neg(q.x);
          bli[b][j] = rot_neg(q.y);
        }
      }
      float2 rho[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) rho[j] = rq[tb + j][r];
#pragma unroll
      for (int i = 0; i < kWPerWave; ++i) {
        u32x4 ah, al;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float2 w = wt[tb + j][wave * kWPerWave + i];
          const float are = fmaf(w.x, rho[j].x, -w.y * rho[j].y);
          const float aim = fmaf(w.x, rho[j].y, w.y * rho[j].x);
          const unsigned int h = pack_bf16(are, aim);
          ah[j] = h;
          al[j] = pack_bf16(are - lo_f(h), aim - hi_f(h));
        }
        const bf16x8 Ah = as_bf16x8(ah), Al = as_bf16x8(al);
#pragma unroll
        for (int b = 0; b < kSub; ++b) {
          f32x4 cr = sr[i][b], ci = si[i][b];
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, as_bf16x8(bhr[b]), cr, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, as_bf16x8(blr[b]), cr, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, as_bf16x8(bhr[b]), cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, as_bf16x8(bhi[b]), ci, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, as_bf16x8(bli[b]), ci, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, as_bf16x8(bhi[b]), ci, 0, 0, 0);
          sr[i][b] = cr;
          si[i][b] = ci;
        }
      }
    }
    since += kChunk;
    if (since >= kFlush) {
      since = 0;
#pragma unroll
      for (int i = 0; i < kWPerWave; ++i)
#pragma unroll
        for (int b = 0; b < kSub; ++b) {
          br[i][b] += sr[i][b];
          bi[i][b] += si[i][b];
          sr[i][b] = f32x4{0, 0, 0, 0};
          si[i][b] = f32x4{0, 0, 0, 0};
        }
    }
  }
#pragma unroll
  for (int i = 0; i < kWPerWave; ++i) {
    const int w = w0 + wave * kWPerWave + i;
    if (w >= n_w) continue;
#pragma unroll
    for (int b = 0; b < kSub; ++b) {
      const int col = col0 + b * 16 + (lane & 15);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = gb * 16 + 4 * (lane >> 4) + j;
        if (row < n_g && col < n_g)
          part[(((size_t)blockIdx.z * n_w + w) * n_g + row) * n_g + col] =
              make_double2((double)br[i][b][j] + (double)sr[i][b][j],
                           (double)bi[i][b][j] + (double)si[i][b][j]);
      }
    }
  }
}

__global__ void k_reduce_slices_b(const double2 *part, int n_slices, size_t per_slice,
                                  double pref, double2 *out) {
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

int chi0_bf16x3(tdx_ctx *ctx, const void *P, int ld, const double *delta, const double *df,
                long long n_trans, const double *omega, int n_w, double eta, int n_g,
                double pref, double2 *chi0, hipStream_t s) {
  const int nblk = ld / 16;
  const int nblk4 = (ld + kCols - 1) / kCols;
  const size_t out_elems = (size_t)n_w * n_g * n_g;
  const long long base = (long long)((n_w + kWBlock - 1) / kWBlock) * nblk * nblk4;
  long long slices = std::max<long long>(1, (4096 + base - 1) / base);
  slices = std::min<long long>(slices, (n_trans + kChunk - 1) / kChunk);
  slices = std::min<long long>(slices, 512);
  long long slice_len = (n_trans + slices - 1) / slices;
  slice_len = (slice_len + kChunk - 1) / kChunk * kChunk;
  slices = (n_trans + slice_len - 1) / slice_len;
  void *w;
  TDX_TRY(ws_get(ctx, WS_PARTIAL, sizeof(double2) * out_elems * slices, &w));
  double2 *part = (double2 *)w;
  dim3 grid((n_w + kWBlock - 1) / kWBlock, nblk * nblk4, (unsigned)slices);
  hipLaunchKernelGGL(k_chi0_bf16x3, grid, dim3(256), 0, s, (const uint2 *)P, ld, delta, df,
                     n_trans, slice_len, omega, n_w, eta, n_g, nblk4, part);
  TDX_HIP(hipGetLastError());
  const unsigned rb = (unsigned)std::min<size_t>((out_elems + 255) / 256, 8192);
  hipLaunchKernelGGL(k_reduce_slices_b, dim3(rb), dim3(256), 0, s, part, (int)slices, out_elems,
                     pref, chi0);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

}  // namespace tdx
