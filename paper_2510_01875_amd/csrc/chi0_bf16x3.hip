// Split-BF16 chi0 contraction on the 16x16x32 bf16 MFMA of gfx950.
//
// Every real operand x is carried as x = hi + lo (bf16, round to nearest
// even) and a product as hi*hi' + hi*lo' + lo*hi' accumulated in FP32; the
// dropped lo*lo' term and the roundings leave a relative error near 2^-16
// per product.  The left operand A = w_t(w) rho_t(G) is formed in FP32 from
// the FP64 weight and the stored pair density, then split.
//
// One MFMA covers K = 32 reals = 16 transitions with (re, im) interleaved:
//   A[G][2t + p]     = (Re, Im)(w_t rho_t(G)),
//   B_re[2t + p][G'] = (Re, Im) rho_t(G'),   B_im[2t + p][G'] = (-Im, Re) rho_t(G'),
// so that D_re accumulates Re chi0 and D_im accumulates Im chi0.
//
// A workgroup owns 16 G x 64 G' for 16 frequencies (4 waves x 4) over one
// slice of transitions.  Per chunk of 32 transitions the B fragments (already
// in lane order and already rotated for the imaginary part), the FP32 rho rows
// and the weights are staged in LDS; the next chunk's global loads are in
// flight while the current chunk runs (two LDS buffers).  Each slice sums in
// FP32; slices are short (about 2^18 transitions) and reduced in FP64 in a
// fixed order.
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace tdx {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWPerWave = 4;
constexpr int kWBlock = 16;     // 4 waves x 4 frequencies
constexpr int kCols = 64;       // G' per workgroup
constexpr int kSub = 4;         // 16-column sub-blocks
constexpr int kChunk = 32;      // transitions per LDS buffer (2 MFMA K-steps)
constexpr int kSteps = kChunk / 16;
constexpr long long kSliceTarget = 1 << 18;

// LDS layout of one buffer (in 32-bit words)
constexpr int kBWords = kSteps * kSub * 4 * 64 * 4;  // [step][sub][comp][lane][4]
constexpr int kRhoWords = kChunk * 16 * 2;           // [t][row] float2
constexpr int kWtWords = kChunk * kWBlock * 2;       // [t][w] float2
constexpr int kBufWords = kBWords + kRhoWords + kWtWords;
constexpr size_t kLdsBytes = 2 * kBufWords * 4;

__device__ inline bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// (re | im << 16) -> (-im | re << 16)
__device__ inline unsigned int rot_neg(unsigned int w) {
  return ((w >> 16) ^ 0x8000u) | (w << 16);
}

__device__ inline unsigned int cvt_pk(float a, float b) {
  return __builtin_bit_cast(unsigned int, __builtin_convertvector((f32x2){a, b}, bf16x2));
}

__device__ inline float lo_f(unsigned int w) { return __uint_as_float(w << 16); }
__device__ inline float hi_f(unsigned int w) { return __uint_as_float(w & 0xffff0000u); }

struct Prefetch {
  uint2 b[8];      // B entries (t, col)
  uint2 a[2];      // rho rows (t, row)
  double d[2], f[2];
};

// Global loads of one chunk into registers.  Full chunks (every row inside
// the slice, the common case) load through strided pointers with no
// predicate; the ragged last chunk of the list clamps its rows into the array
// and store_chunk zeroes them.  Loads are unconditional so they stay in flight
// until the values are stored.
template <bool FULL>
__device__ inline void load_chunk(Prefetch &pf, const uint2 *P, size_t ld, int colc, int row0,
                                  const double *delta, const double *df, long long tc,
                                  long long n_trans, int tid) {
  const int tb = tid >> 6, ta = tid >> 4, ca = tid & 15;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const long long t = FULL ? tc + tb + 4 * i : std::min(tc + tb + 4 * i, n_trans - 1);
    pf.b[i] = P[(size_t)t * ld + colc];
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const long long t = FULL ? tc + ta + 16 * i : std::min(tc + ta + 16 * i, n_trans - 1);
    pf.a[i] = P[(size_t)t * ld + row0 + ca];
    pf.d[i] = delta[t];
    pf.f[i] = df[t];
  }
}

template <bool FULL>
__device__ inline void store_chunk(const Prefetch &pf, unsigned int *buf, double om0, double om1,
                                   bool w_ok, double eta, int tid, long long tc, long long t_hi,
                                   bool col_ok) {
  unsigned int *bw = buf;
  float2 *rq = (float2 *)(buf + kBWords);
  float2 *wt = (float2 *)(buf + kBWords + kRhoWords);
  const int c = tid & 63, b = c >> 4, tb = tid >> 6;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int tl = tb + 4 * i;
    const int s = tl >> 4, kq = (tl & 15) >> 2, jj = tl & 3, l = kq * 16 + (c & 15);
    const bool ok = col_ok && (FULL || tc + tl < t_hi);
    const unsigned int x = ok ? pf.b[i].x : 0u, y = ok ? pf.b[i].y : 0u;
    const int base = ((s * kSub + b) * 4) * 256 + l * 4 + jj;
    bw[base] = x;
    bw[base + 256] = y;
    bw[base + 512] = rot_neg(x);
    bw[base + 768] = rot_neg(y);
  }
  const int ta = tid >> 4, ca = tid & 15;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int tl = ta + 16 * i;
    const bool ok = FULL || tc + tl < t_hi;
    const uint2 q = pf.a[i];
    rq[tl * 16 + ca] = ok ? make_float2(lo_f(q.x) + lo_f(q.y), hi_f(q.x) + hi_f(q.y))
                          : make_float2(0.f, 0.f);
    // weight df / (w - delta + i eta) in FP64, stored in FP32, for the same
    // transition and frequency w0 + ca
    const double x = (i == 0 ? om0 : om1) - pf.d[i];
    const double sc = pf.f[i] / fma(x, x, eta * eta);
    wt[tl * kWBlock + ca] = ok && w_ok ? make_float2((float)(sc * x), (float)(-sc * eta))
                                       : make_float2(0.f, 0.f);
  }
}

__global__ void __launch_bounds__(256, 2)
    k_chi0_bf16x3(const uint2 *P, int ld, const double *delta, const double *df,
                  long long n_trans, long long slice_len, const double *omega, int n_w,
                  double eta, int n_g, int nblk4, double2 *part) {
  extern __shared__ unsigned int lds[];
  const int gb = blockIdx.y / nblk4, gc = blockIdx.y % nblk4;
  const int col0 = gc * kCols, row0 = gb * 16;
  const int w0 = blockIdx.x * kWBlock;
  const long long t_lo = (long long)blockIdx.z * slice_len;
  const long long t_hi = std::min(n_trans, t_lo + slice_len);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, kq = lane >> 4;

  f32x4 ar[kWPerWave][kSub], ai[kWPerWave][kSub];
#pragma unroll
  for (int i = 0; i < kWPerWave; ++i)
#pragma unroll
    for (int b = 0; b < kSub; ++b) {
      ar[i][b] = f32x4{0, 0, 0, 0};
      ai[i][b] = f32x4{0, 0, 0, 0};
    }

  Prefetch pf;
  const int colc = std::min(col0 + (tid & 63), ld - 1);
  const bool col_ok = col0 + (tid & 63) < ld;
  const int wi = w0 + (tid & 15);
  const bool w_ok = wi < n_w;
  const double om = omega[std::min(wi, n_w - 1)];
  const size_t lds_ = (size_t)ld;
  if (t_lo + kChunk <= t_hi) {
    load_chunk<true>(pf, P, lds_, colc, row0, delta, df, t_lo, n_trans, tid);
    store_chunk<true>(pf, lds, om, om, w_ok, eta, tid, t_lo, t_hi, col_ok);
  } else {
    load_chunk<false>(pf, P, lds_, colc, row0, delta, df, t_lo, n_trans, tid);
    store_chunk<false>(pf, lds, om, om, w_ok, eta, tid, t_lo, t_hi, col_ok);
  }
  __syncthreads();
  int cur = 0;
  for (long long tc = t_lo; tc < t_hi; tc += kChunk) {
    const long long nx = tc + kChunk;
    const bool more = nx < t_hi, full = nx + kChunk <= t_hi;
    if (more) {
      if (full)
        load_chunk<true>(pf, P, lds_, colc, row0, delta, df, nx, n_trans, tid);
      else
        load_chunk<false>(pf, P, lds_, colc, row0, delta, df, nx, n_trans, tid);
    }
    const unsigned int *buf = lds + cur * kBufWords;
    const u32x4 *bfr = (const u32x4 *)buf;
    const float2 *rq = (const float2 *)(buf + kBWords);
    const float2 *wt = (const float2 *)(buf + kBWords + kRhoWords);
#pragma unroll
    for (int s = 0; s < kSteps; ++s) {
      const int tb = s * 16 + 4 * kq;
      float2 rho[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) rho[j] = rq[(tb + j) * 16 + r];
      u32x4 ah[kWPerWave], al[kWPerWave];
#pragma unroll
      for (int i = 0; i < kWPerWave; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float2 w = wt[(tb + j) * kWBlock + wave * kWPerWave + i];
          const float are = fmaf(w.x, rho[j].x, -w.y * rho[j].y);
          const float aim = fmaf(w.x, rho[j].y, w.y * rho[j].x);
          const unsigned int h = cvt_pk(are, aim);
          ah[i][j] = h;
          al[i][j] = cvt_pk(are - lo_f(h), aim - hi_f(h));
        }
      }
#pragma unroll
      for (int b = 0; b < kSub; ++b) {
        const u32x4 *bp = bfr + ((s * kSub + b) * 4) * 64 + lane;
        const bf16x8 bhr = as_bf16x8(bp[0]), blr = as_bf16x8(bp[64]);
        const bf16x8 bhi = as_bf16x8(bp[128]), bli = as_bf16x8(bp[192]);
#pragma unroll
        for (int i = 0; i < kWPerWave; ++i) {
          const bf16x8 Ah = as_bf16x8(ah[i]), Al = as_bf16x8(al[i]);
          f32x4 cr = ar[i][b], ci = ai[i][b];
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, bhr, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, bhi, ci, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, blr, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, bli, ci, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, bhr, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, bhi, ci, 0, 0, 0);
          ar[i][b] = cr;
          ai[i][b] = ci;
        }
      }
    }
    if (more) {
      unsigned int *nb = lds + (cur ^ 1) * kBufWords;
      if (full)
        store_chunk<true>(pf, nb, om, om, w_ok, eta, tid, nx, t_hi, col_ok);
      else
        store_chunk<false>(pf, nb, om, om, w_ok, eta, tid, nx, t_hi, col_ok);
    }
    __syncthreads();
    cur ^= 1;
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
        const int row = row0 + 4 * (lane >> 4) + j;
        if (row < n_g && col < n_g)
          part[(((size_t)blockIdx.z * n_w + w) * n_g + row) * n_g + col] =
              make_double2((double)ar[i][b][j], (double)ai[i][b][j]);
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
  long long slices = std::max<long long>((n_trans + kSliceTarget - 1) / kSliceTarget,
                                         (4096 + base - 1) / base);
  slices = std::max<long long>(1, std::min<long long>(slices, (n_trans + kChunk - 1) / kChunk));
  slices = std::min<long long>(slices, 4096);
  long long slice_len = (n_trans + slices - 1) / slices;
  slice_len = (slice_len + kChunk - 1) / kChunk * kChunk;
  slices = (n_trans + slice_len - 1) / slice_len;
  void *w;
  TDX_TRY(ws_get(ctx, WS_PARTIAL, sizeof(double2) * out_elems * slices, &w));
  double2 *part = (double2 *)w;
  dim3 grid((n_w + kWBlock - 1) / kWBlock, nblk * nblk4, (unsigned)slices);
  TDX_HIP(hipFuncSetAttribute((const void *)k_chi0_bf16x3,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes));
  hipLaunchKernelGGL(k_chi0_bf16x3, grid, dim3(256), kLdsBytes, s, (const uint2 *)P, ld, delta,
                     df, n_trans, slice_len, omega, n_w, eta, n_g, nblk4, part);
  TDX_HIP(hipGetLastError());
  const unsigned rb = (unsigned)std::min<size_t>((out_elems + 255) / 256, 8192);
  hipLaunchKernelGGL(k_reduce_slices_b, dim3(rb), dim3(256), 0, s, part, (int)slices, out_elems,
                     pref, chi0);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

}  // namespace tdx
