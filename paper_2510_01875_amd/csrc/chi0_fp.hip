// FP32 and FP64 chi0 contractions on the 16x16x4 FP32 / FP64 MFMA of gfx950.
//
// The complex contraction is one real GEMM as in the split-BF16 tile: one
// K-step of 4 covers 2 transitions with (re, im) interleaved.  With
// a = w_t(w) rho_t(G) and b = rho_t(G'):
//   A[G][2t + p]   = (Re a, Im a),   A_rot[G][2t + p] = (Im a, -Re a),
//   B[2t + p][G']  = (Re b, Im b),
// A B accumulates Re chi0 and A_rot B accumulates Im chi0, in the form's
// precision (E = float or double).  FP32 accumulators are folded into the
// tile's FP64 partial every 128 chunks; slices are reduced in FP64 in a fixed
// order (bitwise reproducible).  The FP32 form takes its weights in FP32
// (w - delta in FP64 first), the FP64 form entirely in FP64.
//
// Lane l of an MFMA holds A[l%16][l/16] and B[l/16][l%16]: transition
// 2s + (l/16)/2, component (l/16)%2.  A is formed in registers from the rho
// row and the weight, once per K-step and frequency, and reused over every
// column block of the tile; an MFMA of this shape runs long enough that the
// formation costs nothing.  The pair-density rows ([T][ld] complex, no
// padding) are copied into LDS by global-to-LDS transfers of 16 bytes per
// lane: per chunk the tile's 16 rows (for A) and its 16 NSUB columns (for B)
// of CHUNK transitions, double-buffered; rows past the end of the list are
// clamped to the last one (their weights are zero).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "chi0_tile.h"
#include "internal.h"

namespace tdx {
namespace {

template <class E>
struct Vec4;
template <>
struct Vec4<float> {
  typedef f32x4 T;
};
template <>
struct Vec4<double> {
  typedef double T __attribute__((ext_vector_type(4)));
};

template <class E, int WPW, int SUB, int CHUNK>
struct CfgFp {
  static constexpr int kW = sizeof(E) / 4;          // 32-bit words per real
  static constexpr int kThreads = 256;
  static constexpr int kWBlock = 4 * WPW;           // frequencies per workgroup
  static constexpr int kSub = SUB;
  static constexpr int kCols = 16 * SUB;            // G' per tile
  static constexpr int kChunk = CHUNK;
  static constexpr int kSteps = CHUNK / 2;          // K-steps of two transitions
  static constexpr int kBWords = CHUNK * kCols * 2 * kW;  // [t][16 NSUB] complex
  static constexpr int kRhoWords = CHUNK * 16 * 2 * kW;   // [t][16] complex
  static constexpr int kWtWords = CHUNK * kWBlock * 2 * kW;
  static constexpr int kBufWords = kBWords + kRhoWords + kWtWords;
  static constexpr bool kWPart = CHUNK * kWBlock < 256;
  static constexpr int kNW = kWPart ? 1 : CHUNK * kWBlock / 256;
  static_assert(256 % kWBlock == 0 && CHUNK % 16 == 0, "tile must divide the block");
};

constexpr int kFpFoldChunks = 128;  // chunks summed in FP32 between folds

// FP64 weights of one chunk (the FP64 form): the same formulas as the FP32
// store, in FP64 throughout.
template <class C>
__device__ inline void store_weights_f64(const Weights<C> &pw, double2 *wt, double om, bool w_ok,
                                         double eta, int paired, int tid, long long tc,
                                         long long t_hi) {
  const int tw = tid / C::kWBlock, wi = tid % C::kWBlock;
#pragma unroll
  for (int i = 0; i < C::kNW; ++i) {
    const int tl = tw + (C::kThreads / C::kWBlock) * i;
    if (C::kWPart && tl >= C::kChunk) break;
    const bool ok = tc + tl < t_hi && w_ok;
    const double d = pw.d[i];
    double2 v;
    if (paired) {
      // 2 df delta / D, D = (w - delta)(w + delta) - eta^2 + 2 i w eta
      const double dr = (om - d) * (om + d) - eta * eta, di = 2.0 * om * eta;
      const double sc = 2.0 * pw.f[i] * d / fma(dr, dr, di * di);
      v = make_double2(sc * dr, -sc * di);
    } else {
      // df / (x + i eta) = df (x - i eta) / (x^2 + eta^2), x = w - delta
      const double x = om - d;
      const double sc = pw.f[i] / fma(x, x, eta * eta);
      v = make_double2(sc * x, -sc * eta);
    }
    wt[wt_index<C>(tl, wi)] = ok ? v : make_double2(0.0, 0.0);
  }
}

// LDS transfers of one chunk: the B rows (CHUNK x 16 NSUB complex, row
// stride 16 NSUB) and the rho rows (CHUNK x 16), in 1 KB pieces dealt to the
// waves in turn.  Lane l of piece j copies LDS bytes 1024 j + 16 l; its
// source row and byte within the row are fixed per slot.
template <class C, int NSUB>
struct DmaPlanFp {
  static constexpr int kRowB = 16 * NSUB * 8 * C::kW, kRowR = 16 * 8 * C::kW;  // bytes per row
  static constexpr int kB = C::kChunk * kRowB / 1024, kR = C::kChunk * kRowR / 1024;
  static constexpr int kT = kB + kR, kSlots = (kT + 3) / 4;
  int row[kSlots];       // row of the chunk the lane copies from
  unsigned col[kSlots];  // byte offset within that row (from col0 or row0)
  int dst[kSlots];       // word offset in a buffer
  bool is_r[kSlots], ok[kSlots];

  __device__ inline DmaPlanFp(int wave, int lane) {
#pragma unroll
    for (int i = 0; i < kSlots; ++i) {
      const int x = 4 * i + wave;  // uniform across the wave
      ok[i] = x < kT;
      is_r[i] = x >= kB;
      const int j = is_r[i] ? std::min(x, kT - 1) - kB : x;
      const int o = 1024 * j + 16 * lane;
      const int rb = is_r[i] ? kRowR : kRowB;
      row[i] = o / rb;
      col[i] = (unsigned)(o % rb);
      dst[i] = (is_r[i] ? C::kBWords : 0) + 256 * j;
    }
  }

  __device__ inline void issue(const unsigned char *P, int ld, int col0, int row0, long long tc,
                               long long t_max, unsigned int *buf) const {
#pragma unroll
    for (int i = 0; i < kSlots; ++i) {
      if (!ok[i]) continue;  // uniform across the wave
      const long long t = std::min(tc + row[i], t_max);
      const unsigned char *src =
          P + ((size_t)t * ld + (is_r[i] ? row0 : col0)) * 8 * C::kW + col[i];
      dma16(src, buf + dst[i]);
    }
  }
};

// One tile: rows row0..row0+15, columns col0..col0+16 NSUB-1, frequencies
// w0..w0+kWBlock-1, transitions [t_lo, t_hi).
template <class E, int WPW, int SUB, int CHUNK, int NSUB>
__device__ __attribute__((always_inline)) void chi0_tile_fp(
    unsigned int *lds, const void *P, int ld, const double *delta, const double *df, int paired,
    long long n_trans, long long t_lo, long long t_hi, const double *omega, int n_w, double eta,
    int n_g, int w0, int row0, int col0, double2 *part) {
  typedef CfgFp<E, WPW, SUB, CHUNK> C;
  typedef typename Vec4<E>::T V;
  typedef typename std::conditional<sizeof(E) == 8, double2, float2>::type E2;
  constexpr bool kF64 = sizeof(E) == 8;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int tau = lane >> 5, comp = (lane >> 4) & 1, c16 = lane & 15;

  V ar[WPW][NSUB], ai[WPW][NSUB];
#pragma unroll
  for (int i = 0; i < WPW; ++i)
#pragma unroll
    for (int b = 0; b < NSUB; ++b) {
      ar[i][b] = V{0, 0, 0, 0};
      ai[i][b] = V{0, 0, 0, 0};
    }

  const unsigned char *Pb = (const unsigned char *)P;
  const long long t_max = n_trans - 1;
  const DmaPlanFp<C, NSUB> dma(wave, lane);
  Weights<C> pw;
  const int wi = w0 + tid % C::kWBlock;
  const bool w_ok = wi < n_w;
  const double om = omega[std::min(wi, n_w - 1)];
  auto store = [&](unsigned int *buf, long long tc) {
    unsigned int *w = buf + C::kBWords + C::kRhoWords;
    if constexpr (kF64)
      store_weights_f64<C>(pw, (double2 *)w, om, w_ok, eta, paired, tid, tc, t_hi);
    else
      store_weights<C>(pw, (float2 *)w, om, w_ok, eta, paired, tid, tc, t_hi);
  };
  dma.issue(Pb, ld, col0, row0, t_lo, t_max, lds);
  load_weights<C>(pw, delta, df, t_lo, t_max, tid);
  store(lds, t_lo);
  wait_vm();
  __syncthreads();
  int cur = 0;
  bool first = true;
  // FP64 sums need no fold until the end of the slice
  constexpr long long kRun = kF64 ? (1LL << 62) : (long long)kFpFoldChunks * CHUNK;
  for (long long rs = t_lo; rs < t_hi; rs += kRun) {
    const long long re = std::min(t_hi, rs + kRun);
    for (long long tc = rs; tc < re; tc += CHUNK) {
      const long long nx = tc + CHUNK;
      const bool more = nx < t_hi;
      if (more) {
        load_weights<C>(pw, delta, df, nx, t_max, tid);
        dma.issue(Pb, ld, col0, row0, nx, t_max, lds + (cur ^ 1) * C::kBufWords);
      }
      const unsigned int *buf = lds + cur * C::kBufWords;
      const E *bq = (const E *)buf;
      const E2 *rq = (const E2 *)(buf + C::kBWords);
      const E2 *wt = (const E2 *)(buf + C::kBWords + C::kRhoWords);
#pragma unroll 2
      for (int s = 0; s < C::kSteps; ++s) {
        const int tl = 2 * s + tau;
        const E2 rho = rq[tl * 16 + c16];
        E a[WPW], r[WPW];
#pragma unroll
        for (int i = 0; i < WPW; ++i) {
          const E2 w = wt[wt_index<C>(tl, wave * WPW + i)];
          const E are = w.x * rho.x - w.y * rho.y;
          const E aim = w.x * rho.y + w.y * rho.x;
          a[i] = comp ? aim : are;
          r[i] = comp ? -are : aim;
        }
#pragma unroll
        for (int b = 0; b < NSUB; ++b) {
          const E bv = bq[(tl * 16 * NSUB + b * 16 + c16) * 2 + comp];
#pragma unroll
          for (int i = 0; i < WPW; ++i) {
            if constexpr (kF64) {
              ar[i][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bv, ar[i][b], 0, 0, 0);
              ai[i][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(r[i], bv, ai[i][b], 0, 0, 0);
            } else {
              ar[i][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], bv, ar[i][b], 0, 0, 0);
              ai[i][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(r[i], bv, ai[i][b], 0, 0, 0);
            }
          }
        }
      }
      if (more) store(lds + (cur ^ 1) * C::kBufWords, nx);
      wait_vm();
      __syncthreads();
      cur ^= 1;
    }
    fold<WPW, NSUB, V, kF64>(ar, ai, part, n_w, n_g, w0, row0, col0, lane, wave, first);
    first = false;
  }
}

template <class E, int WPW, int SUB, int CHUNK, int NSUB = SUB>
__device__ __attribute__((always_inline)) void chi0_tile_fp_n(
    int nsub, unsigned int *lds, const void *P, int ld, const double *delta, const double *df,
    int paired, long long n_trans, long long t_lo, long long t_hi, const double *omega, int n_w,
    double eta, int n_g, int w0, int row0, int col0, double2 *part) {
  if constexpr (NSUB > 1) {
    if (nsub < NSUB) {
      chi0_tile_fp_n<E, WPW, SUB, CHUNK, NSUB - 1>(nsub, lds, P, ld, delta, df, paired, n_trans,
                                                    t_lo, t_hi, omega, n_w, eta, n_g, w0, row0,
                                                    col0, part);
      return;
    }
  }
  chi0_tile_fp<E, WPW, SUB, CHUNK, NSUB>(lds, P, ld, delta, df, paired, n_trans, t_lo, t_hi,
                                         omega, n_w, eta, n_g, w0, row0, col0, part);
}

// One tile per workgroup; logical tile = (frequency block fastest, then
// (G block, G' block), then slice), XCD-aware as in the split-BF16 grid.
template <class E, int WPW, int SUB, int CHUNK>
__global__ void __launch_bounds__(256, 2)
    k_chi0_fp(const void *P, int ld, const double *delta, const double *df, int paired,
              long long n_trans, long long slice_len, const double *omega, int n_w, double eta,
              int n_g, int ncb, double2 *part) {
  typedef CfgFp<E, WPW, SUB, CHUNK> C;
  extern __shared__ unsigned int lds[];
  const int nx = gridDim.x, ny = gridDim.y;
  const int id = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
  const int L = xcd_logical(id, nx * ny * gridDim.z);
  const int bx = L % nx, by = (L / nx) % ny, bz = L / (nx * ny);
  const int gb = by / ncb, gc = by % ncb;
  const long long t_lo = (long long)bz * slice_len;
  const long long t_hi = std::min(n_trans, t_lo + slice_len);
  const int col0 = gc * C::kCols;
  chi0_tile_fp_n<E, WPW, SUB, CHUNK>(std::min(SUB, (ld - col0) / 16), lds, P, ld, delta, df,
                                     paired, n_trans, t_lo, t_hi, omega, n_w, eta, n_g,
                                     bx * C::kWBlock, gb * 16, col0,
                                     part + (size_t)bz * n_w * n_g * n_g);
}

template <class E, int WPW, int SUB, int CHUNK>
int launch_fp(const void *P, int ld, const double *delta, const double *df, int paired,
              long long n_trans, long long slice_len, int slices, const double *omega, int n_w,
              double eta, int n_g, double2 *part, hipStream_t s) {
  typedef CfgFp<E, WPW, SUB, CHUNK> C;
  const void *fn = (const void *)k_chi0_fp<E, WPW, SUB, CHUNK>;
  const size_t lds = (size_t)2 * C::kBufWords * 4;
  const int nblk = ld / 16, ncb = (ld + C::kCols - 1) / C::kCols;
  dim3 grid((n_w + C::kWBlock - 1) / C::kWBlock, nblk * ncb, (unsigned)slices);
  TDX_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((k_chi0_fp<E, WPW, SUB, CHUNK>), grid, dim3(256), lds, s, P, ld, delta, df,
                     paired, n_trans, slice_len, omega, n_w, eta, n_g, ncb, part);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}


// Tile variants: (frequencies per wave, column blocks, transitions per
// chunk); variant 0 of each precision is the default.
struct FpVariant {
  int wpw, sub, chunk;
  int (*launch)(const void *, int, const double *, const double *, int, long long, long long,
                int, const double *, int, double, int, double2 *, hipStream_t);
};

#define TDX_FPV(E, W, S, K) FpVariant{W, S, K, launch_fp<E, W, S, K>}
const FpVariant kVarF32[] = {TDX_FPV(float, 4, 3, 32), TDX_FPV(float, 4, 2, 32),
                             TDX_FPV(float, 4, 4, 32), TDX_FPV(float, 2, 3, 32),
                             TDX_FPV(float, 2, 6, 32)};
const FpVariant kVarF64[] = {TDX_FPV(double, 2, 3, 16), TDX_FPV(double, 2, 2, 16),
                             TDX_FPV(double, 2, 4, 16), TDX_FPV(double, 1, 3, 16),
                             TDX_FPV(double, 1, 6, 16)};
#undef TDX_FPV

const FpVariant &fp_variant(bool f64, int v) { return f64 ? kVarF64[v] : kVarF32[v]; }

}  // namespace

int chi0_fp_variant_count(bool f64) {
  return f64 ? (int)(sizeof(kVarF64) / sizeof(kVarF64[0]))
             : (int)(sizeof(kVarF32) / sizeof(kVarF32[0]));
}

// Tile shape of variant v of the FP32 (f64 = false) or FP64 contraction:
// frequencies and G' columns per workgroup, transitions per chunk (slices
// are multiples of it).
void chi0_fp_shape(bool f64, int v, int *wblock, int *cols, int *chunk) {
  const FpVariant &V = fp_variant(f64, v);
  *wblock = 4 * V.wpw;
  *cols = 16 * V.sub;
  *chunk = V.chunk;
}

int chi0_fp_launch(bool f64, int v, const void *P, int ld, const double *delta, const double *df,
                   int paired, long long n_trans, long long slice_len, int slices,
                   const double *omega, int n_w, double eta, int n_g, double2 *part,
                   hipStream_t s) {
  return fp_variant(f64, v).launch(P, ld, delta, df, paired, n_trans, slice_len, slices, omega,
                                   n_w, eta, n_g, part, s);
}

}  // namespace tdx
