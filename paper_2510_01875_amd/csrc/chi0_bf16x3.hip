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
// A tile is 16 G x (16 SUB) G' for 4 WPW frequencies (4 waves x WPW) over one
// slice of transitions.  Per chunk of CHUNK transitions the B fragments
// (already in lane order and already rotated for the imaginary part), the
// FP32 rho rows and the weights are staged in LDS; the next chunk's global
// loads are in flight while the current chunk runs (two LDS buffers).  Each
// slice sums in FP32; slices are reduced in FP64 in a fixed order, so results
// do not depend on which workgroup ran which tile.
//
// Two launch forms share the tile routine: a grid with one tile per
// workgroup, and a persistent grid that pulls tiles of many q-vectors from a
// longest-first work queue (one launch for a ragged batch).
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>

#include "chi0_batch.h"
#include "internal.h"

namespace tdx {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int WPW, int SUB, int CHUNK>
struct Cfg {
  static constexpr int kWBlock = 4 * WPW;  // frequencies per tile
  static constexpr int kCols = 16 * SUB;   // G' per tile
  static constexpr int kChunk = CHUNK;
  static constexpr int kSteps = CHUNK / 16;
  static constexpr int kBWords = kSteps * SUB * 4 * 64 * 4;  // [step][sub][comp][lane][4]
  static constexpr int kRhoWords = CHUNK * 16 * 2;           // [t][row] float2
  static constexpr int kWtWords = CHUNK * kWBlock * 2;       // [t][w] float2
  static constexpr int kBufWords = kBWords + kRhoWords + kWtWords;
  static constexpr size_t kLds = 2 * (size_t)kBufWords * 4;
  static constexpr int kNB = CHUNK * kCols / 256;    // B entries per thread
  static constexpr int kNA = CHUNK * 16 / 256;       // rho entries per thread
  // weights per thread; when the chunk holds fewer than 256 weights only the
  // first CHUNK * kWBlock threads store one
  static constexpr bool kWPart = CHUNK * kWBlock < 256;
  static constexpr int kNW = kWPart ? 1 : CHUNK * kWBlock / 256;
  static_assert(256 % kCols == 0 && 256 % kWBlock == 0, "tile must divide the block");
  static_assert(kNB >= 1 && kNA >= 1, "chunk too small");
};

__device__ inline bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// (re | im << 16) -> (-im | re << 16)
__device__ inline unsigned int rot_neg(unsigned int w) { return ((w >> 16) ^ 0x8000u) | (w << 16); }

__device__ inline unsigned int cvt_pk(float a, float b) {
  return __builtin_bit_cast(unsigned int, __builtin_convertvector((f32x2){a, b}, bf16x2));
}

__device__ inline float lo_f(unsigned int w) { return __uint_as_float(w << 16); }
__device__ inline float hi_f(unsigned int w) { return __uint_as_float(w & 0xffff0000u); }

template <class C>
struct Prefetch {
  uint2 b[C::kNB];
  uint2 a[C::kNA];
  double d[C::kNW], f[C::kNW];
};

// Global loads of one chunk into registers.  Full chunks (every row inside
// the slice, the common case) load with no predicate; the ragged last chunk
// of the list clamps its rows into the array and store_chunk zeroes them.
// Loads are unconditional so they stay in flight until the values are stored.
template <class C, bool FULL>
__device__ inline void load_chunk(Prefetch<C> &pf, const uint2 *P, size_t ld, int colc, int row0,
                                  const double *delta, const double *df, long long tc,
                                  long long n_trans, int tid) {
  const int tb = tid / C::kCols;
#pragma unroll
  for (int i = 0; i < C::kNB; ++i) {
    const long long t0 = tc + tb + (256 / C::kCols) * i;
    const long long t = FULL ? t0 : std::min(t0, n_trans - 1);
    pf.b[i] = P[(size_t)t * ld + colc];
  }
  const int ta = tid >> 4, ca = tid & 15;
#pragma unroll
  for (int i = 0; i < C::kNA; ++i) {
    const long long t0 = tc + ta + 16 * i;
    const long long t = FULL ? t0 : std::min(t0, n_trans - 1);
    pf.a[i] = P[(size_t)t * ld + row0 + ca];
  }
  const int tw = tid / C::kWBlock;
#pragma unroll
  for (int i = 0; i < C::kNW; ++i) {
    const long long t0 = tc + tw + (256 / C::kWBlock) * i;
    const long long t = (FULL && !C::kWPart) ? t0 : std::min(t0, n_trans - 1);
    pf.d[i] = delta[t];
    pf.f[i] = df[t];
  }
}

template <class C, bool FULL>
__device__ inline void store_chunk(const Prefetch<C> &pf, unsigned int *buf, double om, bool w_ok,
                                   double eta, int tid, long long tc, long long t_hi,
                                   bool col_ok) {
  unsigned int *bw = buf;
  float2 *rq = (float2 *)(buf + C::kBWords);
  float2 *wt = (float2 *)(buf + C::kBWords + C::kRhoWords);
  const int c = tid % C::kCols, b = c >> 4, tb = tid / C::kCols;
#pragma unroll
  for (int i = 0; i < C::kNB; ++i) {
    const int tl = tb + (256 / C::kCols) * i;
    const int s = tl >> 4, kq = (tl & 15) >> 2, jj = tl & 3, l = kq * 16 + (c & 15);
    const bool ok = col_ok && (FULL || tc + tl < t_hi);
    const unsigned int x = ok ? pf.b[i].x : 0u, y = ok ? pf.b[i].y : 0u;
    const int base = ((s * (C::kCols / 16) + b) * 4) * 256 + l * 4 + jj;
    bw[base] = x;
    bw[base + 256] = y;
    bw[base + 512] = rot_neg(x);
    bw[base + 768] = rot_neg(y);
  }
  const int ta = tid >> 4, ca = tid & 15;
#pragma unroll
  for (int i = 0; i < C::kNA; ++i) {
    const int tl = ta + 16 * i;
    const bool ok = FULL || tc + tl < t_hi;
    const uint2 q = pf.a[i];
    rq[tl * 16 + ca] = ok ? make_float2(lo_f(q.x) + lo_f(q.y), hi_f(q.x) + hi_f(q.y))
                          : make_float2(0.f, 0.f);
  }
  // weights df / (w - delta + i eta) in FP64, stored in FP32
  const int tw = tid / C::kWBlock, wi = tid % C::kWBlock;
#pragma unroll
  for (int i = 0; i < C::kNW; ++i) {
    const int tl = tw + (256 / C::kWBlock) * i;
    if (C::kWPart && tl >= C::kChunk) break;
    const bool ok = (FULL || tc + tl < t_hi) && w_ok;
    const double x = om - pf.d[i];
    const double sc = pf.f[i] / fma(x, x, eta * eta);
    wt[tl * C::kWBlock + wi] =
        ok ? make_float2((float)(sc * x), (float)(-sc * eta)) : make_float2(0.f, 0.f);
  }
}

// One tile: rows row0..row0+15, columns col0..col0+kCols-1, frequencies
// w0..w0+kWBlock-1, transitions [t_lo, t_hi).  Writes the FP32 slice sum into
// part (the slice's [n_w][n_g][n_g] block).
template <int WPW, int SUB, int CHUNK>
__device__ __attribute__((always_inline)) void chi0_tile(unsigned int *lds, const uint2 *P, int ld, const double *delta,
                          const double *df, long long n_trans, long long t_lo, long long t_hi,
                          const double *omega, int n_w, double eta, int n_g, int w0, int row0,
                          int col0, double2 *part) {
  typedef Cfg<WPW, SUB, CHUNK> C;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, kq = lane >> 4;

  f32x4 ar[WPW][SUB], ai[WPW][SUB];
#pragma unroll
  for (int i = 0; i < WPW; ++i)
#pragma unroll
    for (int b = 0; b < SUB; ++b) {
      ar[i][b] = f32x4{0, 0, 0, 0};
      ai[i][b] = f32x4{0, 0, 0, 0};
    }

  Prefetch<C> pf;
  const int cc = col0 + tid % C::kCols;
  const int colc = std::min(cc, ld - 1);
  const bool col_ok = cc < ld;
  const int wi = w0 + tid % C::kWBlock;
  const bool w_ok = wi < n_w;
  const double om = omega[std::min(wi, n_w - 1)];
  const size_t lds_ = (size_t)ld;
  if (t_lo + CHUNK <= t_hi) {
    load_chunk<C, true>(pf, P, lds_, colc, row0, delta, df, t_lo, n_trans, tid);
    store_chunk<C, true>(pf, lds, om, w_ok, eta, tid, t_lo, t_hi, col_ok);
  } else {
    load_chunk<C, false>(pf, P, lds_, colc, row0, delta, df, t_lo, n_trans, tid);
    store_chunk<C, false>(pf, lds, om, w_ok, eta, tid, t_lo, t_hi, col_ok);
  }
  __syncthreads();
  int cur = 0;
  for (long long tc = t_lo; tc < t_hi; tc += CHUNK) {
    const long long nx = tc + CHUNK;
    const bool more = nx < t_hi, full = nx + CHUNK <= t_hi;
    if (more) {
      if (full)
        load_chunk<C, true>(pf, P, lds_, colc, row0, delta, df, nx, n_trans, tid);
      else
        load_chunk<C, false>(pf, P, lds_, colc, row0, delta, df, nx, n_trans, tid);
    }
    const unsigned int *buf = lds + cur * C::kBufWords;
    const u32x4 *bfr = (const u32x4 *)buf;
    const float2 *rq = (const float2 *)(buf + C::kBWords);
    const float2 *wt = (const float2 *)(buf + C::kBWords + C::kRhoWords);
#pragma unroll
    for (int s = 0; s < C::kSteps; ++s) {
      const int tb = s * 16 + 4 * kq;
      float2 rho[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) rho[j] = rq[(tb + j) * 16 + r];
      u32x4 ah[WPW], al[WPW];
#pragma unroll
      for (int i = 0; i < WPW; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float2 w = wt[(tb + j) * C::kWBlock + wave * WPW + i];
          const float are = fmaf(w.x, rho[j].x, -w.y * rho[j].y);
          const float aim = fmaf(w.x, rho[j].y, w.y * rho[j].x);
          const unsigned int h = cvt_pk(are, aim);
          ah[i][j] = h;
          al[i][j] = cvt_pk(are - lo_f(h), aim - hi_f(h));
        }
      }
#pragma unroll
      for (int b = 0; b < SUB; ++b) {
        const u32x4 *bp = bfr + ((s * SUB + b) * 4) * 64 + lane;
        const bf16x8 bhr = as_bf16x8(bp[0]), blr = as_bf16x8(bp[64]);
        const bf16x8 bhi = as_bf16x8(bp[128]), bli = as_bf16x8(bp[192]);
#pragma unroll
        for (int i = 0; i < WPW; ++i) {
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
      unsigned int *nb = lds + (cur ^ 1) * C::kBufWords;
      if (full)
        store_chunk<C, true>(pf, nb, om, w_ok, eta, tid, nx, t_hi, col_ok);
      else
        store_chunk<C, false>(pf, nb, om, w_ok, eta, tid, nx, t_hi, col_ok);
    }
    __syncthreads();
    cur ^= 1;
  }
  // D[row][col]: element j of lane l is row 4*(l/16)+j, column l%16
#pragma unroll
  for (int i = 0; i < WPW; ++i) {
    const int w = w0 + wave * WPW + i;
    if (w >= n_w) continue;
#pragma unroll
    for (int b = 0; b < SUB; ++b) {
      const int col = col0 + b * 16 + (lane & 15);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = row0 + 4 * (lane >> 4) + j;
        if (row < n_g && col < n_g)
          part[((size_t)w * n_g + row) * n_g + col] =
              make_double2((double)ar[i][b][j], (double)ai[i][b][j]);
      }
    }
  }
}

// One tile per workgroup: x = frequency block, y = (G block, G' block), z = slice.
template <int WPW, int SUB, int CHUNK>
__global__ void __launch_bounds__(256, 2)
    k_chi0_bf16x3(const uint2 *P, int ld, const double *delta, const double *df,
                  long long n_trans, long long slice_len, const double *omega, int n_w,
                  double eta, int n_g, int ncb, double2 *part) {
  typedef Cfg<WPW, SUB, CHUNK> C;
  extern __shared__ unsigned int lds[];
  const int gb = blockIdx.y / ncb, gc = blockIdx.y % ncb;
  const long long t_lo = (long long)blockIdx.z * slice_len;
  const long long t_hi = std::min(n_trans, t_lo + slice_len);
  chi0_tile<WPW, SUB, CHUNK>(lds, P, ld, delta, df, n_trans, t_lo, t_hi, omega, n_w, eta, n_g,
                             blockIdx.x * C::kWBlock, gb * 16, gc * C::kCols,
                             part + (size_t)blockIdx.z * n_w * n_g * n_g);
}

// Persistent form: every workgroup takes tiles from the queue until it is
// empty.  The queue counter is a device integer zeroed before the launch;
// every workgroup leaves once the counter passes the tile count.
template <int WPW, int SUB, int CHUNK>
__global__ void __launch_bounds__(256, 2)
    k_chi0_bf16x3_persistent(const BatchItem *items, const BatchTile *tiles, int n_tiles,
                             int *counter) {
  typedef Cfg<WPW, SUB, CHUNK> C;
  extern __shared__ unsigned int lds[];
  __shared__ int s_idx;
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1);
    __syncthreads();
    const int idx = s_idx;
    __syncthreads();
    if (idx >= n_tiles) break;
    const BatchTile tl = tiles[idx];
    const BatchItem it = items[tl.item];
    const long long t_lo = tl.slice * it.slice_len;
    const long long t_hi = std::min(it.n_trans, t_lo + it.slice_len);
    chi0_tile<WPW, SUB, CHUNK>(lds, (const uint2 *)it.P, it.ld, it.delta, it.df, it.n_trans,
                               t_lo, t_hi, it.omega, it.n_w, it.eta, it.n_g,
                               tl.wblk * C::kWBlock, tl.gb * 16, tl.gc * C::kCols,
                               it.part + (size_t)tl.slice * it.n_w * it.n_g * it.n_g);
  }
}

struct Variant {
  int wpw, sub, chunk;
  size_t lds;
  const void *grid_fn;
  const void *pers_fn;
};

#define TDX_V(W, S, K)                                                                   \
  Variant {                                                                              \
    W, S, K, Cfg<W, S, K>::kLds, (const void *)k_chi0_bf16x3<W, S, K>,                   \
        (const void *)k_chi0_bf16x3_persistent<W, S, K>                                  \
  }
const Variant kVariants[] = {TDX_V(4, 4, 32), TDX_V(2, 8, 16), TDX_V(4, 2, 32),
                             TDX_V(2, 4, 32)};
#undef TDX_V

}  // namespace

int bf16x3_variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }

void bf16x3_variant_shape(int v, int *wblock, int *cols) {
  *wblock = 4 * kVariants[v].wpw;
  *cols = 16 * kVariants[v].sub;
}

int bf16x3_launch_grid(int v, const void *P, int ld, const double *delta, const double *df,
                       long long n_trans, long long slice_len, int slices, const double *omega,
                       int n_w, double eta, int n_g, double2 *part, hipStream_t s) {
  const Variant &V = kVariants[v];
  const int nblk = ld / 16;
  int ncb = (ld + 16 * V.sub - 1) / (16 * V.sub);
  dim3 grid((n_w + 4 * V.wpw - 1) / (4 * V.wpw), nblk * ncb, (unsigned)slices);
  TDX_HIP(hipFuncSetAttribute(V.grid_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)V.lds));
  void *args[] = {(void *)&P,       (void *)&ld,        (void *)&delta, (void *)&df,
                  (void *)&n_trans, (void *)&slice_len, (void *)&omega, (void *)&n_w,
                  (void *)&eta,     (void *)&n_g,       (void *)&ncb,   (void *)&part};
  TDX_HIP(hipLaunchKernel(V.grid_fn, grid, dim3(256), args, V.lds, s));
  return TDX_OK;
}

int bf16x3_launch_persistent(int v, const BatchItem *items, const BatchTile *tiles, int n_tiles,
                             int *counter, int n_blocks, hipStream_t s) {
  const Variant &V = kVariants[v];
  TDX_HIP(hipFuncSetAttribute(V.pers_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)V.lds));
  void *args[] = {(void *)&items, (void *)&tiles, (void *)&n_tiles, (void *)&counter};
  TDX_HIP(hipLaunchKernel(V.pers_fn, dim3(n_blocks), dim3(256), args, V.lds, s));
  return TDX_OK;
}

}  // namespace tdx
