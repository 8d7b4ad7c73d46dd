// Pair densities rho_t(G) = <n k| e^{-i(q+G).r} |m k+q> for every transition.
//
// With G2 = G1 + G + G_s in the basis of k' (k + q = k' + G_s):
//   rho_t(G) = sum_{G2 in basis(k')} conj(c_nk(G2 - G - G_s)) c_mk'(G2).
// One wavefront per (k, n) row of the transition list computes the row as a
// complex matrix product on the FP64 MFMA (details at the kernel).
// Accumulation is FP64; the store converts to the requested layout.

#include <cmath>
#include <type_traits>

#include "internal.h"
#include "tables.h"

namespace tdx {
namespace {


// Rows of the split-BF16 layout: the transition count rounded up to 32 plus
// one more chunk of 32 zero rows, so that the chi0 kernel can read whole
// chunks past the end without clamping.
__host__ __device__ inline long long pad_rows(long long n_trans) {
  return ((n_trans + 31) / 32 + 1) * 32;
}

// Round-to-nearest-even of an FP32 value to bf16, from its bit pattern
// (finite inputs).  Integer arithmetic keeps the two roundings FP64 -> FP32
// -> bf16 separate: a fused FP64 -> bf16 conversion would round ties of the
// FP32 value differently.
__device__ inline unsigned int rne_bf16(float x) {
  const unsigned int u = __float_as_uint(x);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

template <int FMT>
__device__ inline void store(void *P, long long t, int g, int ld, long long n_trans, double re,
                             double im) {
  const size_t i = (size_t)t * ld + g;
  if (FMT == TDX_PREC_FP64) {
    ((double2 *)P)[i] = make_double2(re, im);
  } else if (FMT == TDX_PREC_FP32) {
    ((float2 *)P)[i] = make_float2((float)re, (float)im);
  } else {
    // fragment words [t/4][comp][ld][t%4] with comp = hi, lo and each word
    // = (re, im) as two bf16, followed by rho in FP32 [T][ld]
    const float r32 = (float)re, i32 = (float)im;
    const unsigned int rh = rne_bf16(r32), ih = rne_bf16(i32);
    const unsigned int rl = rne_bf16(r32 - __uint_as_float(rh << 16));
    const unsigned int il = rne_bf16(i32 - __uint_as_float(ih << 16));
    unsigned int *w = (unsigned int *)P + (((size_t)(t >> 2) * 2) * ld + g) * 4 + (t & 3);
    w[0] = rh | (ih << 16);
    w[(size_t)ld * 4] = rl | (il << 16);
    float2 *R = (float2 *)((char *)P + (size_t)pad_rows(n_trans) * ld * 8);
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
  const long long nfrag = nq * 8 * ld;  // words per quad: 2 components x ld x 4
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nfrag;
       e += (long long)gridDim.x * blockDim.x) {
    const int jj = (int)(e & 3);
    if (e < 8LL * ld && jj < r0) continue;  // live rows of the partial quad
    P[(size_t)q0 * 8 * ld + e] = 0u;
  }
  float2 *R = (float2 *)((char *)P + (size_t)rows * ld * 8);
  const long long nrho = (rows - n_trans) * ld;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nrho;
       e += (long long)gridDim.x * blockDim.x)
    R[(size_t)n_trans * ld + e] = make_float2(0.f, 0.f);
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kPdGT = 9;  // 16-wide G tiles held in accumulators at once

// One wavefront per (k, n) row of the transition list.  For the row's
// transitions m (tiles of 16) and the response vectors G (tiles of 16,
// kPdGT at a time) the pair densities are the complex matrix product
//   rho[m][G] = sum_{G2 in basis(k')} c_mk'(G2) U[G2][G],
//   U[G2][G] = conj(c_nk)(G2 - G - G_s)  (0 if outside the basis of k),
// on the FP64 16x16x4 MFMA, four real products per K-step of four G2.  Lane
// l feeds A = c_{m(l%16)}(G2 = 4 s + l/16) and B = U[4 s + l/16][16 gt + l%16];
// the B operand is gathered per lane through the Miller-index lookup box of
// k, which sits in LDS next to conj(c_nk).  The output element j of lane l is
// m row l/16 + 4 j, G column l%16.
template <int FMT>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2)))
    k_pair_density(const double2 *coef, const int *miller, const int *npw, int nb_max,
                   int npw_max, const int *tm, const long long *rowbeg, const long long *rowend,
                   const int *kpmap, const int *gsmap, const int *gbasis, int n_g, int ld,
                   const int *lut, long box, int M0, int M1, int M2, void *P,
                   long long n_trans) {
  extern __shared__ double2 ckn[];                 // [npw_max] conj(c_nk)
  int *lutk = (int *)(ckn + npw_max);              // [box] lookup of k
  const int n = blockIdx.x, k = blockIdx.y;
  const long long t0 = rowbeg[(size_t)k * nb_max + n], t1 = rowend[(size_t)k * nb_max + n];
  if (t1 <= t0) return;
  const int lane = threadIdx.x;
  const int kp = kpmap[k];
  const int gs0 = gsmap[3 * k], gs1 = gsmap[3 * k + 1], gs2 = gsmap[3 * k + 2];
  const int npk = npw[k], npj = npw[kp];
  for (int i = lane; i < npk; i += 64) {
    const double2 c = coef[((size_t)k * nb_max + n) * npw_max + i];
    ckn[i] = make_double2(c.x, -c.y);
  }
  for (long i = lane; i < box; i += 64) lutk[i] = lut[(size_t)k * box + i];
  __syncthreads();
  const int W1 = 2 * M1 + 1, W2 = 2 * M2 + 1;
  const int *mj = miller + (size_t)kp * npw_max * 3;
  const double2 *cj = coef + (size_t)kp * nb_max * npw_max;
  const int r = lane & 15, kq = lane >> 4;
  const int n_gt = ld / 16;
  for (long long tm0 = t0; tm0 < t1; tm0 += 16) {
    // this lane's A row: transition tm0 + r (zero past the row)
    const bool row_ok = tm0 + r < t1;
    const double2 *crow = cj + (size_t)(row_ok ? tm[tm0 + r] : 0) * npw_max;
    // NQ tiles of 16 G starting at tile gt0 (NQ a compile-time count, so the
    // K-step below is straight-line code)
    auto tiles = [&](int gt0, auto nq_c) {
      constexpr int NQ = decltype(nq_c)::value;
      f64x4 acr[NQ], aci[NQ];
      // G + G_s of this lane's column in each tile, packed as three 10-bit
      // fields offset by 512
      unsigned gp[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        acr[q] = aci[q] = f64x4{0.0, 0.0, 0.0, 0.0};
        const int g = std::min((gt0 + q) * 16 + r, n_g - 1);
        gp[q] = (unsigned)(gbasis[3 * g] + gs0 + 512) |
                ((unsigned)(gbasis[3 * g + 1] + gs1 + 512) << 10) |
                ((unsigned)(gbasis[3 * g + 2] + gs2 + 512) << 20);
      }
      // A operand one K-step ahead (a global load whose latency the current
      // step's MFMAs cover)
      auto load_a = [&](int j0) {
        const int j = j0 + kq;
        return j < npj && row_ok ? crow[j] : make_double2(0.0, 0.0);
      };
      double2 a_next = load_a(0);
      for (int j0 = 0; j0 < npj; j0 += 4) {
        const int j = j0 + kq;
        const double2 a = a_next;
        a_next = load_a(j0 + 4);
        const int jc = std::min(j, npj - 1);
        const int m0 = mj[3 * jc] + M0, m1 = mj[3 * jc + 1] + M1, m2 = mj[3 * jc + 2] + M2;
        // B operands of every tile: all lookups first, then all values, with
        // no branches (out-of-range entries read slot 0 and are zeroed)
        int li[NQ];
        bool ok[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int g = (gt0 + q) * 16 + r;
          const int x0 = m0 + 512 - (int)(gp[q] & 1023u);
          const int x1 = m1 + 512 - (int)((gp[q] >> 10) & 1023u);
          const int x2 = m2 + 512 - (int)(gp[q] >> 20);
          ok[q] = j < npj && g < n_g && x0 >= 0 && x0 <= 2 * M0 && x1 >= 0 && x1 < W1 &&
                  x2 >= 0 && x2 < W2;
          li[q] = ok[q] ? ((x0 * W1 + x1) * W2 + x2) : 0;
        }
        int idx[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) idx[q] = lutk[li[q]];
        double2 u[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const bool hit = ok[q] && idx[q] >= 0;
          const double2 v = ckn[hit ? idx[q] : 0];
          u[q] = hit ? v : make_double2(0.0, 0.0);
        }
        // per accumulator the same order of products as one tile at a time
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          acr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, u[q].x, acr[q], 0, 0, 0);
          aci[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, u[q].y, aci[q], 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          acr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, u[q].y, acr[q], 0, 0, 0);
          aci[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, u[q].x, aci[q], 0, 0, 0);
        }
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const long long t = tm0 + kq + 4 * e;
          if (t < t1) store<FMT>(P, t, (gt0 + q) * 16 + r, ld, n_trans, acr[q][e], aci[q][e]);
        }
      }
    };
    for (int gt0 = 0; gt0 < n_gt; gt0 += kPdGT) {
      switch (std::min(kPdGT, n_gt - gt0)) {  // uniform across the wave
        case 1: tiles(gt0, std::integral_constant<int, 1>{}); break;
        case 2: tiles(gt0, std::integral_constant<int, 2>{}); break;
        case 3: tiles(gt0, std::integral_constant<int, 3>{}); break;
        case 4: tiles(gt0, std::integral_constant<int, 4>{}); break;
        case 5: tiles(gt0, std::integral_constant<int, 5>{}); break;
        case 6: tiles(gt0, std::integral_constant<int, 6>{}); break;
        case 7: tiles(gt0, std::integral_constant<int, 7>{}); break;
        case 8: tiles(gt0, std::integral_constant<int, 8>{}); break;
        default: tiles(gt0, std::integral_constant<int, kPdGT>{}); break;
      }
    }
  }
}

int ld_of(int n_g) { return (n_g + 15) / 16 * 16; }

}  // namespace
}  // namespace tdx

using namespace tdx;

extern "C" {

size_t tdx_pair_density_bytes(int64_t n_trans, int n_g, int prec) {
  if (prec == TDX_PREC_BF16X3) return (size_t)pad_rows(n_trans) * ld_of(n_g) * 16;
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
  for (int i = 0; i < 3; ++i)
    TDX_REQUIRE(st->mmax[i] < 200, TDX_ERR_SHAPE, "Miller range %d too large", st->mmax[i]);
  TDX_REQUIRE(st->npw_max * sizeof(double2) +
                      sizeof(int) * (size_t)(2 * st->mmax[0] + 1) * (2 * st->mmax[1] + 1) *
                          (2 * st->mmax[2] + 1) <=
                  150 * 1024,
              TDX_ERR_SHAPE, "plane-wave basis of %d and its lookup box exceed LDS",
              st->npw_max);
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
                     nb_max, (long long)n_trans, d_rb, d_re);
  TDX_HIP(hipGetLastError());
  const int ld = ld_of(n_g);
  const size_t lds = sizeof(double2) * st->npw_max + sizeof(int) * (size_t)box;
  dim3 grid(nb_max, nk);
#define TDX_PD(F)                                                                              \
  TDX_HIP(hipFuncSetAttribute((const void *)k_pair_density<F>,                                 \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));          \
  hipLaunchKernelGGL(k_pair_density<F>, grid, dim3(64), lds, s, (const double2 *)st->coef,     \
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
