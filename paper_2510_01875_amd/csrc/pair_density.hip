// Pair densities rho_t(G) = <n k| e^{-i(q+G).r} |m k+q> for every transition.
//
// With G2 = G1 + G + G_s in the basis of k' (k + q = k' + G_s):
//   rho_t(G) = sum_{G2 in basis(k')} conj(c_nk(G2 - G - G_s)) c_mk'(G2).
// One workgroup per (k, n) row of the transition list: the row's conj(c_nk)
// sits in LDS, the shifted copy U[G][G2] is gathered from it through a
// Miller-index lookup box, and the m-rows c_mk' stream through LDS tiles, so
// that rho[m][G] = sum_G2 U[G][G2] c_mk'(G2) is a small dense product.
// Accumulation is FP64; the store converts to the requested layout.
#include <hip/hip_bf16.h>

#include <cmath>

#include "internal.h"
#include "tables.h"

namespace tdx {
namespace {

constexpr int kTile = 16;   // G and m tile
constexpr int kChunk = 32;  // G2 chunk

// Rows of the split-BF16 layout: the transition count rounded up to 32 plus
// one more chunk of 32 zero rows, so that the chi0 kernel can read whole
// chunks past the end without clamping.
__host__ __device__ inline long long pad_rows(long long n_trans) {
  return ((n_trans + 31) / 32 + 1) * 32;
}

__device__ inline unsigned int pack_bf16(__hip_bfloat16 lo, __hip_bfloat16 hi) {
  return (unsigned int)__bfloat16_as_ushort(lo) | ((unsigned int)__bfloat16_as_ushort(hi) << 16);
}

// (re | im << 16) -> (-im | re << 16)
__device__ inline unsigned int rot_neg(unsigned int w) { return ((w >> 16) ^ 0x8000u) | (w << 16); }

template <int FMT>
__device__ inline void store(void *P, long long t, int g, int ld, long long n_trans, double re,
                             double im) {
  const size_t i = (size_t)t * ld + g;
  if (FMT == TDX_PREC_FP64) {
    ((double2 *)P)[i] = make_double2(re, im);
  } else if (FMT == TDX_PREC_FP32) {
    ((float2 *)P)[i] = make_float2((float)re, (float)im);
  } else {
    // fragment words [t/4][comp][ld][t%4] with comp = hi, lo, rot(hi), rot(lo)
    // and each word = (re, im) as two bf16, followed by rho in FP32 [T][ld]
    const float r32 = (float)re, i32 = (float)im;
    const __hip_bfloat16 rh = __float2bfloat16(r32), ih = __float2bfloat16(i32);
    const __hip_bfloat16 rl = __float2bfloat16(r32 - __bfloat162float(rh));
    const __hip_bfloat16 il = __float2bfloat16(i32 - __bfloat162float(ih));
    const unsigned int whi = pack_bf16(rh, ih), wlo = pack_bf16(rl, il);
    unsigned int *w = (unsigned int *)P + (((size_t)(t >> 2) * 4) * ld + g) * 4 + (t & 3);
    const size_t comp = (size_t)ld * 4;
    w[0] = whi;
    w[comp] = wlo;
    w[2 * comp] = rot_neg(whi);
    w[3 * comp] = rot_neg(wlo);
    float2 *R = (float2 *)((char *)P + (size_t)pad_rows(n_trans) * ld * 16);
    R[i] = make_float2(r32, i32);
  }
}

// Rows n_trans .. pad_rows(n_trans)-1 of both blocks (fragment words and
// FP32 rho) are zero.
__global__ void k_zero_pad(unsigned int *P, long long n_trans, int ld) {
  const long long rows = pad_rows(n_trans);
  const long long q0 = n_trans >> 2;
  const int r0 = (int)(n_trans & 3);
  const long long nq = rows / 4 - q0;
  const long long nfrag = nq * 16 * ld;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nfrag;
       e += (long long)gridDim.x * blockDim.x) {
    const int jj = (int)(e & 3);
    if (e < 16LL * ld && jj < r0) continue;  // live rows of the partial quad
    P[(size_t)q0 * 16 * ld + e] = 0u;
  }
  float2 *R = (float2 *)((char *)P + (size_t)rows * ld * 16);
  const long long nrho = (rows - n_trans) * ld;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nrho;
       e += (long long)gridDim.x * blockDim.x)
    R[(size_t)n_trans * ld + e] = make_float2(0.f, 0.f);
}

template <int FMT>
__global__ void __launch_bounds__(256)
    k_pair_density(const double2 *coef, const int *miller, const int *npw, int nb_max,
                   int npw_max, const int *tm, const long long *rowbeg, const long long *rowend,
                   const int *kpmap, const int *gsmap, const int *gbasis, int n_g, int ld,
                   const int *lut, long box, int M0, int M1, int M2, void *P,
                   long long n_trans) {
  extern __shared__ double2 ckn[];  // [npw_max] conj(c_nk)
  __shared__ double2 U[kTile][kChunk + 1];
  __shared__ double2 C[kTile][kChunk + 1];
  __shared__ int mrow[kTile];

  const int n = blockIdx.x, k = blockIdx.y;
  const long long t0 = rowbeg[(size_t)k * nb_max + n], t1 = rowend[(size_t)k * nb_max + n];
  if (t1 <= t0) return;
  const int kp = kpmap[k];
  const int gs0 = gsmap[3 * k], gs1 = gsmap[3 * k + 1], gs2 = gsmap[3 * k + 2];
  const int npk = npw[k], npj = npw[kp];
  const int tid = threadIdx.x;
  const int tx = tid % kTile, ty = tid / kTile;  // tx: G (or G2), ty: m

  for (int i = tid; i < npk; i += 256) {
    const double2 c = coef[((size_t)k * nb_max + n) * npw_max + i];
    ckn[i] = make_double2(c.x, -c.y);
  }
  __syncthreads();
  const int *lutk = lut + (size_t)k * box;
  const int *mj = miller + (size_t)kp * npw_max * 3;
  const int W1 = 2 * M1 + 1, W2 = 2 * M2 + 1;

  for (long long tb = t0; tb < t1; tb += kTile) {
    if (tid < kTile) mrow[tid] = (tb + tid < t1) ? tm[tb + tid] : -1;
    for (int gb = 0; gb < ld; gb += kTile) {
      double ar = 0.0, ai = 0.0;
      for (int jb = 0; jb < npj; jb += kChunk) {
        __syncthreads();
        // U[g][j] = conj(c_nk)(G2_j - G_g - G_s), 512 entries
        for (int e = tid; e < kTile * kChunk; e += 256) {
          const int g = e / kChunk, j = e % kChunk;
          const int gi = gb + g, ji = jb + j;
          double2 u = make_double2(0.0, 0.0);
          if (gi < n_g && ji < npj) {
            const int x0 = mj[3 * ji] - gbasis[3 * gi] - gs0 + M0;
            const int x1 = mj[3 * ji + 1] - gbasis[3 * gi + 1] - gs1 + M1;
            const int x2 = mj[3 * ji + 2] - gbasis[3 * gi + 2] - gs2 + M2;
            if (x0 >= 0 && x0 <= 2 * M0 && x1 >= 0 && x1 < W1 && x2 >= 0 && x2 < W2) {
              const int idx = lutk[((long)x0 * W1 + x1) * W2 + x2];
              if (idx >= 0) u = ckn[idx];
            }
          }
          U[g][j] = u;
        }
        // C[m][j] = c_mk'(G2_j)
        for (int e = tid; e < kTile * kChunk; e += 256) {
          const int mi = e / kChunk, j = e % kChunk;
          const int m = mrow[mi], ji = jb + j;
          C[mi][j] = (m >= 0 && ji < npj) ? coef[((size_t)kp * nb_max + m) * npw_max + ji]
                                          : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll 8
        for (int j = 0; j < kChunk; ++j) {
          const double2 u = U[tx][j], c = C[ty][j];
          ar = fma(u.x, c.x, ar);
          ar = fma(-u.y, c.y, ar);
          ai = fma(u.x, c.y, ai);
          ai = fma(u.y, c.x, ai);
        }
      }
      const long long t = tb + ty;
      if (t < t1) store<FMT>(P, t, gb + tx, ld, n_trans, ar, ai);
    }
    __syncthreads();
  }
}

int ld_of(int n_g) { return (n_g + 15) / 16 * 16; }

}  // namespace
}  // namespace tdx

using namespace tdx;

extern "C" {

size_t tdx_pair_density_bytes(int64_t n_trans, int n_g, int prec) {
  if (prec == TDX_PREC_BF16X3) return (size_t)pad_rows(n_trans) * ld_of(n_g) * 24;
  const size_t per = prec == TDX_PREC_FP64 ? 16 : 8;
  return (size_t)n_trans * ld_of(n_g) * per;
}

int tdx_pair_density(tdx_ctx *ctx, const tdx_states *st, const int qj[3], const tdx_translist *tl,
                     int64_t n_trans, const int *gbasis, int n_g, int prec, void *P,
                     tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && st && qj && tl && gbasis && P, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(prec >= TDX_PREC_FP64 && prec <= TDX_PREC_BF16X3, TDX_ERR_INVALID_ARG, "bad prec");
  TDX_REQUIRE(n_g > 0 && n_trans >= 0 && n_trans <= tl->capacity, TDX_ERR_SHAPE, "bad sizes");
  TDX_REQUIRE(st->npw_max * sizeof(double2) <= 120 * 1024, TDX_ERR_SHAPE,
              "plane-wave basis of %d exceeds the LDS row buffer", st->npw_max);
  TDX_TRY(check_device(ctx));
  if (n_trans == 0) return TDX_OK;
  hipStream_t s = as_stream(stream);
  const int nk = st->n_k, nb_max = st->nb_max;
  const int M0 = st->mmax[0], M1 = st->mmax[1], M2 = st->mmax[2];
  const long box = (long)(2 * M0 + 1) * (2 * M1 + 1) * (2 * M2 + 1);
  std::vector<int> kp, gs;
  kq_map(st->kgrid, qj, &kp, &gs);
  void *w1, *w2;
  const size_t lut_bytes = (sizeof(int) * (size_t)nk * box + 255) / 256 * 256;
  const size_t row_bytes = sizeof(long long) * 2 * (size_t)nk * nb_max;
  TDX_TRY(ws_get(ctx, WS_DENS, lut_bytes + row_bytes, &w1));
  TDX_TRY(ws_get(ctx, WS_MISC, sizeof(int) * 4 * (size_t)nk, &w2));
  int *d_lut = (int *)w1;
  long long *d_rb = (long long *)((char *)w1 + lut_bytes);
  long long *d_re = d_rb + (size_t)nk * nb_max;
  int *d_kp = (int *)w2, *d_gs = d_kp + nk;
  TDX_HIP(hipMemcpyAsync(d_kp, kp.data(), sizeof(int) * nk, hipMemcpyHostToDevice, s));
  TDX_HIP(hipMemcpyAsync(d_gs, gs.data(), sizeof(int) * 3 * nk, hipMemcpyHostToDevice, s));
  TDX_HIP(hipMemsetAsync(d_lut, 0xff, lut_bytes, s));
  TDX_HIP(hipMemsetAsync(d_rb, 0, row_bytes, s));
  hipLaunchKernelGGL(k_lut, dim3((st->npw_max + 255) / 256, nk), dim3(256), 0, s, st->miller,
                     st->npw, st->npw_max, nk, M0, M1, M2, d_lut, box);
  TDX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_rows, dim3(nk), dim3(256), 0, s, (const long long *)tl->k_offsets, tl->n,
                     nb_max, d_rb, d_re);
  TDX_HIP(hipGetLastError());
  const int ld = ld_of(n_g);
  const size_t lds = sizeof(double2) * st->npw_max;
  dim3 grid(nb_max, nk);
#define TDX_PD(F)                                                                              \
  TDX_HIP(hipFuncSetAttribute((const void *)k_pair_density<F>,                                 \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));          \
  hipLaunchKernelGGL(k_pair_density<F>, grid, dim3(256), lds, s, (const double2 *)st->coef,    \
                     st->miller, st->npw, nb_max, st->npw_max, tl->m, d_rb, d_re, d_kp, d_gs,  \
                     gbasis, n_g, ld, d_lut, box, M0, M1, M2, P, (long long)n_trans)
  if (prec == TDX_PREC_FP64) {
    TDX_PD(TDX_PREC_FP64);
  } else if (prec == TDX_PREC_FP32) {
    TDX_PD(TDX_PREC_FP32);
  } else {
    hipLaunchKernelGGL(k_zero_pad, dim3(64), dim3(256), 0, s, (unsigned int *)P,
                       (long long)n_trans, ld);
    TDX_HIP(hipGetLastError());
    TDX_PD(TDX_PREC_BF16X3);
  }
#undef TDX_PD
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

}  // extern "C"
