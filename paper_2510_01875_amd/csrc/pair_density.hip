// Pair densities rho_t(G) = <n k| e^{-i(q+G).r} |m k+q> for every transition.
//
// With G2 = G1 + G + G_s in the basis of k' (k + q = k' + G_s):
//   rho_t(G) = sum_{G2 in basis(k')} conj(c_nk(G2 - G - G_s)) c_mk'(G2).
// One wavefront per group of transitions sharing one side computes the group
// as a complex matrix product on the FP64 MFMA: (k, n) rows of the list, and
// for rows too short to fill the MFMA, (k, m) columns (details at the
// kernels).
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

// Rows (k, n) with fewer transitions than this run in column groups (k, m)
// instead: a (k, n) row of an empty band n pairs it with the few occupied
// bands m (five to seven on the crystal workload), which would fill under
// half of the 16 MFMA rows, while the column (k, m) of an occupied band m
// collects the empty bands of all those rows.
constexpr int kShortRow = 16;

// Column groups: for every k, the transitions of its short rows grouped by m,
// listed in perm[colbeg[k][m] .. colend[k][m]); the groups of k occupy the
// start of k's own range of the list.  The order inside a group does not
// change any result (every transition is one MFMA row of its own).
__global__ void k_cols(const long long *koff, const int *tn, const int *tm, int nb_max,
                       long long t_lo, long long t_hi, const long long *rowbeg,
                       const long long *rowend, long long *colbeg, long long *colend,
                       long long *perm) {
  extern __shared__ int cnt[];  // [nb_max] counts, then [nb_max] cursors
  int *cur = cnt + nb_max;
  const int k = blockIdx.x;
  const long long t0 = koff[k] > t_lo ? koff[k] : t_lo;
  const long long t1 = koff[k + 1] < t_hi ? koff[k + 1] : t_hi;
  for (int i = threadIdx.x; i < 2 * nb_max; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  if (t1 <= t0) {  // no transition of k in the range: empty groups
    for (int m = threadIdx.x; m < nb_max; m += blockDim.x)
      colbeg[(size_t)k * nb_max + m] = colend[(size_t)k * nb_max + m] = 0;
    return;
  }
  auto is_short = [&](long long t) {
    const size_t r = (size_t)k * nb_max + tn[t];
    return rowend[r] - rowbeg[r] < kShortRow;
  };
  for (long long t = t0 + threadIdx.x; t < t1; t += blockDim.x)
    if (is_short(t)) atomicAdd(&cnt[tm[t]], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int m = 0; m < nb_max; ++m) {
      colbeg[(size_t)k * nb_max + m] = t0 - t_lo + acc;
      colend[(size_t)k * nb_max + m] = t0 - t_lo + acc + cnt[m];
      cur[m] = acc;
      acc += cnt[m];
    }
  }
  __syncthreads();
  for (long long t = t0 + threadIdx.x; t < t1; t += blockDim.x)
    if (is_short(t)) perm[t0 - t_lo + atomicAdd(&cur[tm[t]], 1)] = t;
}

// One wavefront per group of transitions that share one side: a row group
// (k, n) (COL false) or a column group (k, m) (COL true).  Row group: with
// G2 in the basis of k',
//   rho[m][G] = sum_{G2} c_mk'(G2) U[G2][G],   U[G2][G] = conj(c_nk)(G2 - G - G_s);
// column group: with G1 = G2 - G - G_s in the basis of k,
//   rho[n][G] = sum_{G1} conj(c_nk)(G1) V[G1][G],   V[G1][G] = c_mk'(G1 + G + G_s).
// Both are complex matrix products on the FP64 16x16x4 MFMA, four real
// products per K-step of four plane waves: the A rows are the coefficients of
// the group's 16 transitions, the B operand is gathered per lane through the
// Miller-index lookup box of the fixed side, which sits in LDS next to that
// side's coefficients (zero outside its basis).  The output element j of
// lane l is transition row l/16 + 4 j, G column l%16; transition t is
// stored in row t - t_lo of P.  W wavefronts share one
// group (and its LDS) and take its 16-transition tiles in turn: W = 1 where
// the LDS of a group is small enough for several groups per CU, W = 8 (two
// per SIMD) where it is not (about 6300 plane waves: 149 KB, one group per
// CU).  The Miller indices of the A side, which every K-step needs before its
// lookups, are staged in LDS too (MS) when they fit, else loaded one K-step
// ahead.
template <int FMT, bool COL, int W, bool MS>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(2, 2)))
    k_pair_density(const double2 *coef, const int *miller, const int *npw, int nb_max,
                   int npw_max, const int *tn, const int *tm, const long long *gbeg,
                   const long long *gend, const long long *perm, const int *kpmap,
                   const int *gsmap, const int *gbasis, int n_g, int ld, const int *lut, long box,
                   int M0, int M1, int M2, void *P, long long t_lo, long long n_rows) {
  extern __shared__ double2 cfix[];             // [npw_max] the fixed side
  int *lutf = (int *)(cfix + npw_max);          // [box] lookup of its k-point
  unsigned *mia = (unsigned *)(lutf + box);     // [npw_max] A-side indices (MS)
  const int band = blockIdx.x, k = blockIdx.y;
  const size_t grp = (size_t)k * nb_max + band;
  const long long p0 = gbeg[grp], p1 = gend[grp];
  if (p1 <= p0) return;
  if (!COL && p1 - p0 < kShortRow) return;  // these run in column groups
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kp = kpmap[k];
  const int kf = COL ? kp : k;  // k-point of the fixed side (and of the lookup)
  const int ka = COL ? k : kp;  // k-point of the A rows (and of the K index)
  const int gs0 = gsmap[3 * k], gs1 = gsmap[3 * k + 1], gs2 = gsmap[3 * k + 2];
  const int npf = npw[kf], npa = npw[ka];
  const double2 *cf = coef + ((size_t)kf * nb_max + band) * npw_max;
  for (int i = threadIdx.x; i < npf; i += 64 * W) {
    const double2 c = cf[i];
    cfix[i] = COL ? c : make_double2(c.x, -c.y);
  }
  for (long i = threadIdx.x; i < box; i += 64 * W) lutf[i] = lut[(size_t)kf * box + i];
  const int W1 = 2 * M1 + 1, W2 = 2 * M2 + 1;
  const int *ma = miller + (size_t)ka * npw_max * 3;
  // Miller triple of plane wave j of the A side, offset into the lookup box
  // and packed as three 10-bit fields
  auto packed_m = [&](int j) {
    return (unsigned)(ma[3 * j] + M0) | ((unsigned)(ma[3 * j + 1] + M1) << 10) |
           ((unsigned)(ma[3 * j + 2] + M2) << 20);
  };
  if constexpr (MS)
    for (int i = threadIdx.x; i < npa; i += 64 * W) mia[i] = packed_m(i);
  __syncthreads();
  const double2 *ca = coef + (size_t)ka * nb_max * npw_max;
  const int *ta = COL ? tn : tm;  // band of the A row of a transition
  const int r = lane & 15, kq = lane >> 4;
  const int n_gt = ld / 16;
  // transition of group slot p
  auto trans = [&](long long p) { return COL ? perm[p] : p; };
  for (long long q0 = p0 + 16 * wave; q0 < p1; q0 += 16 * W) {
    // this lane's A row: the transition of slot q0 + r (zero past the group)
    const bool row_ok = q0 + r < p1;
    const double2 *crow = ca + (size_t)(row_ok ? ta[trans(q0 + r)] : 0) * npw_max;
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
      // step's MFMAs cover); conjugated for a column group
      auto load_a = [&](int j0) {
        const int j = j0 + kq;
        const double2 c = j < npa && row_ok ? crow[j] : make_double2(0.0, 0.0);
        return COL ? make_double2(c.x, -c.y) : c;
      };
      double2 a_next = load_a(0);
      unsigned pm_next = MS ? 0u : packed_m(std::min((int)kq, npa - 1));
      for (int j0 = 0; j0 < npa; j0 += 4) {
        const int j = j0 + kq;
        const double2 a = a_next;
        a_next = load_a(j0 + 4);
        const int jc = std::min(j, npa - 1);
        unsigned pm;
        if constexpr (MS) {
          pm = mia[jc];
        } else {
          pm = pm_next;
          pm_next = packed_m(std::min(j + 4, npa - 1));
        }
        const int m0 = (int)(pm & 1023u), m1 = (int)((pm >> 10) & 1023u), m2 = (int)(pm >> 20);
        // B operands of every tile: all lookups first, then all values, with
        // no branches (out-of-range entries read slot 0 and are zeroed); the
        // lookup index is G2 - G - G_s (row group) or G1 + G + G_s (column)
        int li[NQ];
        bool ok[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int g = (gt0 + q) * 16 + r;
          const int f0 = (int)(gp[q] & 1023u) - 512, f1 = (int)((gp[q] >> 10) & 1023u) - 512,
                    f2 = (int)(gp[q] >> 20) - 512;
          const int x0 = COL ? m0 + f0 : m0 - f0;
          const int x1 = COL ? m1 + f1 : m1 - f1;
          const int x2 = COL ? m2 + f2 : m2 - f2;
          ok[q] = j < npa && g < n_g && x0 >= 0 && x0 <= 2 * M0 && x1 >= 0 && x1 < W1 &&
                  x2 >= 0 && x2 < W2;
          li[q] = ok[q] ? ((x0 * W1 + x1) * W2 + x2) : 0;
        }
        int idx[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) idx[q] = lutf[li[q]];
        double2 u[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const bool hit = ok[q] && idx[q] >= 0;
          const double2 v = cfix[hit ? idx[q] : 0];
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
          const long long p = q0 + kq + 4 * e;
          if (p < p1)
            store<FMT>(P, trans(p) - t_lo, (gt0 + q) * 16 + r, ld, n_rows, acr[q][e],
                       aci[q][e]);
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

}  // extern "C"

namespace tdx {
namespace {

// Device tables of one call, carved from one workspace: the Miller lookup
// boxes, the (k, n) row and (k, m) column ranges, the column permutation and
// the k + q maps.
struct PdWork {
  int *lut;
  long long *rb, *re, *cb, *ce, *perm;
  int *kp, *gs;
};

size_t pd_work_layout(const tdx_states *st, long long n_rows, void *base, PdWork *w) {
  const int nk = st->n_k, nb_max = st->nb_max;
  const long box = (long)(2 * st->mmax[0] + 1) * (2 * st->mmax[1] + 1) * (2 * st->mmax[2] + 1);
  auto r256 = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t lut = r256(sizeof(int) * (size_t)nk * box);
  // row starts and ends back to back (one fill clears both), then the
  // column-group starts and ends
  const size_t tab = r256(sizeof(long long) * 2 * (size_t)nk * nb_max);
  const size_t perm = r256(sizeof(long long) * (size_t)std::max<long long>(n_rows, 1));
  const size_t maps = r256(sizeof(int) * 4 * (size_t)nk);
  if (w) {
    char *p = (char *)base;
    w->lut = (int *)p;
    p += lut;
    w->rb = (long long *)p;
    w->re = w->rb + (size_t)nk * nb_max;
    w->cb = (long long *)(p + tab);
    w->ce = w->cb + (size_t)nk * nb_max;
    p += 2 * tab;
    w->perm = (long long *)p;
    p += perm;
    w->kp = (int *)p;
    w->gs = w->kp + nk;
  }
  return lut + 2 * tab + perm + maps;
}

int pd_check(const tdx_states *st, const int qj[3], const tdx_translist *tl, int64_t t_begin,
             int64_t t_end, const int *gbasis, int n_g, int prec, const void *P) {
  TDX_REQUIRE(st && qj && tl && gbasis && P, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(prec >= TDX_PREC_FP64 && prec <= TDX_PREC_BF16X3, TDX_ERR_INVALID_ARG, "bad prec");
  TDX_REQUIRE(n_g > 0 && t_begin >= 0 && t_begin <= t_end && t_end <= tl->capacity,
              TDX_ERR_SHAPE, "bad sizes");
  for (int i = 0; i < 3; ++i)
    TDX_REQUIRE(st->mmax[i] < 200, TDX_ERR_SHAPE, "Miller range %d too large", st->mmax[i]);
  TDX_REQUIRE(st->npw_max * sizeof(double2) +
                      sizeof(int) * (size_t)(2 * st->mmax[0] + 1) * (2 * st->mmax[1] + 1) *
                          (2 * st->mmax[2] + 1) <=
                  150 * 1024,
              TDX_ERR_SHAPE, "plane-wave basis of %d and its lookup box exceed LDS",
              st->npw_max);
  return TDX_OK;
}

// Every launch of one pair-density call, with its tables in `work`: no host
// copy, memset or synchronisation, so a caller may capture it in a graph.
int pd_enqueue(const tdx_states *st, const int qj[3], const tdx_translist *tl, int64_t t_begin,
               int64_t t_end, const int *gbasis, int n_g, int prec, void *P, void *work,
               hipStream_t s) {
  const long long n_trans = t_end - t_begin;
  if (n_trans == 0) return TDX_OK;
  const int nk = st->n_k, nb_max = st->nb_max;
  const int M0 = st->mmax[0], M1 = st->mmax[1], M2 = st->mmax[2];
  const long box = (long)(2 * M0 + 1) * (2 * M1 + 1) * (2 * M2 + 1);
  PdWork w;
  pd_work_layout(st, n_trans, work, &w);
  hipLaunchKernelGGL(k_kq_map, dim3((nk + 255) / 256), dim3(256), 0, s, st->kgrid[0],
                     st->kgrid[1], st->kgrid[2], qj[0], qj[1], qj[2], w.kp, w.gs);
  TDX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_fill<int>, dim3(1024), dim3(256), 0, s, w.lut, (long long)nk * box, -1);
  TDX_HIP(hipGetLastError());
  // every row start and end (re follows rb directly); k_cols writes every
  // column-group entry itself
  hipLaunchKernelGGL(k_fill<long long>, dim3(1024), dim3(256), 0, s, w.rb,
                     2LL * nk * nb_max, 0LL);
  TDX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_lut, dim3((st->npw_max + 255) / 256, nk), dim3(256), 0, s, st->miller,
                     st->npw, st->npw_max, nk, M0, M1, M2, w.lut, box);
  TDX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_rows, dim3(nk), dim3(256), 0, s, (const long long *)tl->k_offsets, tl->n,
                     nb_max, (long long)t_begin, (long long)t_end, w.rb, w.re);
  TDX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_cols, dim3(nk), dim3(256), sizeof(int) * 2 * nb_max, s,
                     (const long long *)tl->k_offsets, tl->n, tl->m, nb_max, (long long)t_begin,
                     (long long)t_end, w.rb, w.re, w.cb, w.ce, w.perm);
  TDX_HIP(hipGetLastError());
  const int ld = ld_of(n_g);
  const size_t lds0 = sizeof(double2) * st->npw_max + sizeof(int) * (size_t)box;
  dim3 grid(nb_max, nk);
  // eight wavefronts per group when fewer than four groups fit in a CU's LDS
  const bool wide = lds0 > 40 * 1024;
  // the A side's Miller indices in LDS as well when they fit
  const bool ms = lds0 + sizeof(unsigned) * st->npw_max <= 150 * 1024;
  const size_t lds = ms ? lds0 + sizeof(unsigned) * st->npw_max : lds0;
  // long rows, then the column groups of the short ones (disjoint outputs)
#define TDX_PD3(F, COL, W, MS, B, E)                                                           \
  TDX_HIP(hipFuncSetAttribute((const void *)k_pair_density<F, COL, W, MS>,                     \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));          \
  hipLaunchKernelGGL((k_pair_density<F, COL, W, MS>), grid, dim3(64 * W), lds, s,              \
                     (const double2 *)st->coef, st->miller, st->npw, nb_max, st->npw_max,      \
                     tl->n, tl->m, B, E, w.perm, w.kp, w.gs, gbasis, n_g, ld, w.lut, box, M0,  \
                     M1, M2, P, (long long)t_begin, n_trans);                                  \
  TDX_HIP(hipGetLastError())
#define TDX_PD2(F, COL, W, B, E)       \
  if (ms) {                            \
    TDX_PD3(F, COL, W, true, B, E);    \
  } else {                             \
    TDX_PD3(F, COL, W, false, B, E);   \
  }
#define TDX_PD1(F, COL, B, E)       \
  if (wide) {                       \
    TDX_PD2(F, COL, 8, B, E)        \
  } else {                          \
    TDX_PD2(F, COL, 1, B, E)        \
  }
#define TDX_PD(F)                   \
  TDX_PD1(F, false, w.rb, w.re)     \
  TDX_PD1(F, true, w.cb, w.ce)
  if (prec == TDX_PREC_FP64) {
    TDX_PD(TDX_PREC_FP64);
  } else if (prec == TDX_PREC_FP32) {
    TDX_PD(TDX_PREC_FP32);
  } else {
    hipLaunchKernelGGL(k_zero_pad, dim3(64), dim3(256), 0, s, (unsigned int *)P, n_trans, ld);
    TDX_HIP(hipGetLastError());
    TDX_PD(TDX_PREC_BF16X3);
  }
#undef TDX_PD
#undef TDX_PD1
#undef TDX_PD2
#undef TDX_PD3
  return TDX_OK;
}

}  // namespace
}  // namespace tdx

extern "C" {

size_t tdx_pair_density_work_bytes(const tdx_states *st, int64_t n_trans) {
  if (!st || n_trans < 0) return 0;
  return pd_work_layout(st, n_trans, nullptr, nullptr);
}

int tdx_pair_density_async(tdx_ctx *ctx, const tdx_states *st, const int qj[3],
                           const tdx_translist *tl, int64_t t_begin, int64_t t_end,
                           const int *gbasis, int n_g, int prec, void *P, void *work,
                           size_t work_bytes, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && work, TDX_ERR_INVALID_ARG, "null argument");
  TDX_TRY(pd_check(st, qj, tl, t_begin, t_end, gbasis, n_g, prec, P));
  TDX_REQUIRE(work_bytes >= pd_work_layout(st, t_end - t_begin, nullptr, nullptr), TDX_ERR_SHAPE,
              "work buffer of %zu bytes below tdx_pair_density_work_bytes", work_bytes);
  return pd_enqueue(st, qj, tl, t_begin, t_end, gbasis, n_g, prec, P, work, as_stream(stream));
}

int tdx_pair_density_range(tdx_ctx *ctx, const tdx_states *st, const int qj[3],
                           const tdx_translist *tl, int64_t t_begin, int64_t t_end,
                           const int *gbasis, int n_g, int prec, void *P, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx, TDX_ERR_INVALID_ARG, "null argument");
  TDX_TRY(pd_check(st, qj, tl, t_begin, t_end, gbasis, n_g, prec, P));
  TDX_TRY(check_device(ctx));
  if (t_end == t_begin) return TDX_OK;
  void *w;
  TDX_TRY(ws_get(ctx, WS_DENS, pd_work_layout(st, t_end - t_begin, nullptr, nullptr), &w));
  return pd_enqueue(st, qj, tl, t_begin, t_end, gbasis, n_g, prec, P, w, as_stream(stream));
}

int tdx_pair_density(tdx_ctx *ctx, const tdx_states *st, const int qj[3], const tdx_translist *tl,
                     int64_t n_trans, const int *gbasis, int n_g, int prec, void *P,
                     tdx_stream stream) {
  return tdx_pair_density_range(ctx, st, qj, tl, 0, n_trans, gbasis, n_g, prec, P, stream);
}

}  // extern "C"
