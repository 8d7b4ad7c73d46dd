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
// slice of transitions.  The pair densities arrive in a layout made for this
// kernel: per quad of transitions and column, the 16-byte groups hi, lo,
// rot(hi), rot(lo) (rot(re, im) = (-im, re)), so that one 16-byte-per-lane
// global-to-LDS transfer fills one lane-ordered B fragment, and the FP32 rho
// rows for the left operand.  Per chunk of CHUNK transitions the fragments
// and rho rows are copied into LDS with no register staging and no
// arithmetic; only the weights pass through registers.  The next chunk's
// transfers are in flight while the current chunk runs (two LDS buffers).  Sums
// run in FP32 over 256 chunks and are folded into the tile's FP64 partial;
// slices are reduced in FP64 in a fixed order, so results do not depend on
// which workgroup ran which tile.
//
// Two launch forms share the tile routine: a grid with one tile per
// workgroup, and a persistent grid that walks the longest-first tile list of
// many q-vectors (one launch for a ragged batch).
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
  // weights per thread; when the chunk holds fewer than 256 weights only the
  // first CHUNK * kWBlock threads store one
  static constexpr bool kWPart = CHUNK * kWBlock < 256;
  static constexpr int kNW = kWPart ? 1 : CHUNK * kWBlock / 256;
  static_assert(256 % kWBlock == 0 && CHUNK % 16 == 0, "tile must divide the block");
};

constexpr int kFoldChunks = 256;  // chunks summed in FP32 between folds

__device__ inline bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ inline unsigned int cvt_pk(float a, float b) {
  return __builtin_bit_cast(unsigned int, __builtin_convertvector((f32x2){a, b}, bf16x2));
}

__device__ inline float lo_f(unsigned int w) { return __uint_as_float(w << 16); }
__device__ inline float hi_f(unsigned int w) { return __uint_as_float(w & 0xffff0000u); }

// LDS index (float2 units) of rho(tl, row) and of the weight (tl, w): the
// four transition groups kq that one MFMA K-step reads side by side are
// adjacent, so a read instruction touches consecutive words.
__device__ inline int rho_index(int tl, int row) {
  return (((tl >> 4) * 4 + (tl & 3)) * 4 + ((tl & 15) >> 2)) * 16 + row;
}
template <class C>
__device__ inline int wt_index(int tl, int w) {
  return (((tl >> 4) * 4 + (tl & 3)) * C::kWBlock + w) * 4 + ((tl & 15) >> 2);
}

typedef __attribute__((address_space(3))) void lds_void;

// 16 bytes per lane from global memory straight into LDS: lane l writes
// dst + 16 l (dst uniform across the wave).  No registers are involved.
__device__ inline void dma16(const void *src, unsigned int *dst) {
  __builtin_amdgcn_global_load_lds(src, (lds_void *)dst, 16, 0, 0);
}

// Wait for this wave's outstanding global loads, LDS transfers included.
__device__ inline void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0f70); }  // vmcnt(0)

// Stage the B fragments and the FP32 rho rows of the chunk starting at
// transition tc (a multiple of 16) into buf by LDS DMA.  The pair-density
// buffer carries a zero chunk past its last transition, so whole chunks are
// read without clamping; each transfer is a wave-uniform base plus a
// per-lane offset fixed for the tile (lane_b, lane_r).
//  - B: block (s, b, comp) is the lane-ordered fragment of K-step s,
//    16-column block b and component comp (hi, lo, rot hi, rot lo); wave w
//    stages comp = w of every block.  Lane (kq = l/16, c16 = l%16) copies the
//    16-byte word group of transitions tc + 16 s + 4 kq .. +3 at column
//    col0 + 16 b + c16: lane_b = (4 kq ld + c16) * 16 bytes.
//  - rho: block d holds float2 slots 64 d .. 64 d + 63 of the layout
//    rho_index; lane l copies rows row0 + 2 m, +1 (m = l & 7) of transition
//    tc + 16 (d/2) + 2 (d&1) + h + 4 kq2 (h = l/32, kq2 = l/8 & 3):
//    lane_r = ((h + 4 kq2) ld + 2 m) * 8 bytes.
template <class C>
__device__ inline void dma_chunk(const unsigned char *P4, const unsigned char *R, int ld,
                                 long long tc, int col0, int row0, int nsub, unsigned int *buf,
                                 int wave, unsigned lane_b, unsigned lane_r) {
#pragma unroll
  for (int m = 0; m < C::kSteps * (C::kCols / 16); ++m) {
    const int s = m / (C::kCols / 16), b = m % (C::kCols / 16);
    if (b >= nsub) continue;  // uniform across the workgroup
    const unsigned char *base =
        P4 + ((((size_t)(tc >> 2) + 4 * s) * 4 + wave) * ld + col0 + 16 * b) * 16;
    dma16(base + lane_b, buf + (m * 4 + wave) * 256);
  }
  for (int d = wave; d < C::kChunk / 8; d += 4) {
    const unsigned char *base =
        R + ((size_t)(tc + 16 * (d >> 1) + 2 * (d & 1)) * ld + row0) * 8;
    dma16(base + lane_r, buf + C::kBWords + d * 256);
  }
}

// Weights df / (w - delta + i eta) of one chunk: loads into registers ...
template <class C>
struct Weights {
  double d[C::kNW], f[C::kNW];
};

template <class C>
__device__ inline void load_weights(Weights<C> &pw, const double *delta, const double *df,
                                    long long tc, long long t_max, int tid) {
  const int tw = tid / C::kWBlock;
#pragma unroll
  for (int i = 0; i < C::kNW; ++i) {
    const int tl = std::min(tw + (256 / C::kWBlock) * i, C::kChunk - 1);
    const long long t = std::min(tc + tl, t_max);
    pw.d[i] = delta[t];
    pw.f[i] = df[t];
  }
}

// ... and into LDS: w - delta in FP64 (it may cancel), the rest in FP32
// (relative error ~1e-7, far below the 2^-16 of the split products); zero
// past the end of the slice or of the frequency grid.
template <class C>
__device__ inline void store_weights(const Weights<C> &pw, unsigned int *buf, double om,
                                     bool w_ok, float eta, int tid, long long tc,
                                     long long t_hi) {
  float2 *wt = (float2 *)(buf + C::kBWords + C::kRhoWords);
  const int tw = tid / C::kWBlock, wi = tid % C::kWBlock;
#pragma unroll
  for (int i = 0; i < C::kNW; ++i) {
    const int tl = tw + (256 / C::kWBlock) * i;
    if (C::kWPart && tl >= C::kChunk) break;
    const bool ok = tc + tl < t_hi && w_ok;
    const float x = (float)(om - pw.d[i]);
    const float sc = (float)pw.f[i] * __builtin_amdgcn_rcpf(fmaf(x, x, eta * eta));
    wt[wt_index<C>(tl, wi)] = ok ? make_float2(sc * x, -sc * eta) : make_float2(0.f, 0.f);
  }
}

// Fold the FP32 accumulators into the tile's FP64 partial in global memory
// (the workgroup owns that region): the first fold stores, later ones add.
template <int WPW, int SUB>
__device__ inline void fold(f32x4 (&ar)[WPW][SUB], f32x4 (&ai)[WPW][SUB], double2 *part, int n_w,
                            int n_g, int w0, int row0, int col0, int lane, int wave, bool first) {
#pragma unroll
  for (int i = 0; i < WPW; ++i) {
    const int w = w0 + wave * WPW + i;
#pragma unroll
    for (int b = 0; b < SUB; ++b) {
      const int col = col0 + b * 16 + (lane & 15);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        // D[row][col]: element j of lane l is row 4*(l/16)+j, column l%16
        const int row = row0 + 4 * (lane >> 4) + j;
        if (w < n_w && row < n_g && col < n_g) {
          double2 *d = part + ((size_t)w * n_g + row) * n_g + col;
          double2 v = make_double2((double)ar[i][b][j], (double)ai[i][b][j]);
          if (!first) {
            const double2 o = *d;
            v.x += o.x;
            v.y += o.y;
          }
          *d = v;
        }
      }
      ar[i][b] = f32x4{0, 0, 0, 0};
      ai[i][b] = f32x4{0, 0, 0, 0};
    }
  }
}

// One tile: rows row0..row0+15, columns col0..col0+kCols-1, frequencies
// w0..w0+kWBlock-1, transitions [t_lo, t_hi).  Sums run in FP32 for at most
// kFoldChunks chunks and are folded into part (the slice's [n_w][n_g][n_g]
// block, FP64) between runs.
template <int WPW, int SUB, int CHUNK>
__device__ __attribute__((always_inline)) void chi0_tile(
    unsigned int *lds, const void *P, const void *R, int ld, const double *delta,
    const double *df, long long n_trans, long long t_lo, long long t_hi, const double *omega,
    int n_w, double eta, int n_g, int w0, int row0, int col0, double2 *part) {
  typedef Cfg<WPW, SUB, CHUNK> C;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int kq = lane >> 4;

  f32x4 ar[WPW][SUB], ai[WPW][SUB];
#pragma unroll
  for (int i = 0; i < WPW; ++i)
#pragma unroll
    for (int b = 0; b < SUB; ++b) {
      ar[i][b] = f32x4{0, 0, 0, 0};
      ai[i][b] = f32x4{0, 0, 0, 0};
    }

  const unsigned char *P4 = (const unsigned char *)P, *Rr = (const unsigned char *)R;
  const long long t_max = n_trans - 1;
  const unsigned lane_b = (unsigned)(4 * kq * ld + (lane & 15)) * 16u;
  const unsigned lane_r = (unsigned)(((lane >> 5) + 4 * ((lane >> 3) & 3)) * ld + 2 * (lane & 7)) * 8u;
  Weights<C> pw;
  const int wi = w0 + tid % C::kWBlock;
  const bool w_ok = wi < n_w;
  const double om = omega[std::min(wi, n_w - 1)];
  const float etaf = (float)eta;
  // 16-column blocks of this tile inside the padded basis (ld is a multiple
  // of 16); blocks past it are neither staged nor multiplied
  const int nsub = std::min(SUB, (ld - col0) / 16);
  dma_chunk<C>(P4, Rr, ld, t_lo, col0, row0, nsub, lds, wave, lane_b, lane_r);
  load_weights<C>(pw, delta, df, t_lo, t_max, tid);
  store_weights<C>(pw, lds, om, w_ok, etaf, tid, t_lo, t_hi);
  wait_vm();
  __syncthreads();
  int cur = 0;
  bool first = true;
  constexpr long long kRun = (long long)kFoldChunks * CHUNK;
  for (long long rs = t_lo; rs < t_hi; rs += kRun) {
    const long long re = std::min(t_hi, rs + kRun);
    for (long long tc = rs; tc < re; tc += CHUNK) {
      const long long nx = tc + CHUNK;
      const bool more = nx < t_hi;
      if (more) {
        dma_chunk<C>(P4, Rr, ld, nx, col0, row0, nsub, lds + (cur ^ 1) * C::kBufWords, wave,
                     lane_b, lane_r);
        load_weights<C>(pw, delta, df, nx, t_max, tid);
      }
      const unsigned int *buf = lds + cur * C::kBufWords;
      const u32x4 *bfr = (const u32x4 *)buf;
      const float2 *rq = (const float2 *)(buf + C::kBWords);
      const float2 *wt = (const float2 *)(buf + C::kBWords + C::kRhoWords);
  #pragma unroll
      for (int s = 0; s < C::kSteps; ++s) {
        float2 rho[4];
  #pragma unroll
        for (int j = 0; j < 4; ++j) rho[j] = rq[(s * 4 + j) * 64 + lane];
        u32x4 ah[WPW], al[WPW];
  #pragma unroll
        for (int i = 0; i < WPW; ++i) {
  #pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float2 w = wt[((s * 4 + j) * C::kWBlock + wave * WPW + i) * 4 + kq];
            const float are = fmaf(w.x, rho[j].x, -w.y * rho[j].y);
            const float aim = fmaf(w.x, rho[j].y, w.y * rho[j].x);
            const unsigned int h = cvt_pk(are, aim);
            ah[i][j] = h;
            al[i][j] = cvt_pk(are - lo_f(h), aim - hi_f(h));
          }
        }
  #pragma unroll
        for (int b = 0; b < SUB; ++b) {
          if (b < nsub) {  // uniform across the workgroup
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
      }
      if (more) store_weights<C>(pw, lds + (cur ^ 1) * C::kBufWords, om, w_ok, etaf, tid, nx, t_hi);
      wait_vm();
      __syncthreads();
      cur ^= 1;
    }
    fold<WPW, SUB>(ar, ai, part, n_w, n_g, w0, row0, col0, lane, wave, first);
    first = false;
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs (id % 8), each with
// its own L2.  Logical tile L runs on workgroup (L % per) * 8 + L / per with
// per = total / 8, so every XCD runs a contiguous range of logical tiles and
// neighbouring tiles, which read the same pair-density rows, share an L2.
__device__ inline int xcd_logical(int id, int total) {
  const int per = total / 8;
  if (id >= per * 8) return id;  // ragged tail keeps its place
  return (id % 8) * per + id / 8;
}

// One tile per workgroup; logical tile = (frequency block fastest, then
// (G block, G' block), then slice).  OCC = workgroups per CU (2 for every
// listed shape: one wave per SIMD leaves LDS and dependency latency exposed,
// measured at about 60 % of the two-wave rate for 16 x 128 and 16 x 144
// tiles that fill the 512-entry register file).
template <int WPW, int SUB, int CHUNK, int OCC>
__global__ void __launch_bounds__(256, OCC)
    k_chi0_bf16x3(const void *P, const void *R, int ld, const double *delta, const double *df,
                  long long n_trans, long long slice_len, const double *omega, int n_w,
                  double eta, int n_g, int ncb, double2 *part) {
  typedef Cfg<WPW, SUB, CHUNK> C;
  extern __shared__ unsigned int lds[];
  const int nx = gridDim.x, ny = gridDim.y;
  const int id = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
  const int L = xcd_logical(id, nx * ny * gridDim.z);
  const int bx = L % nx, by = (L / nx) % ny, bz = L / (nx * ny);
  const int gb = by / ncb, gc = by % ncb;
  const long long t_lo = (long long)bz * slice_len;
  const long long t_hi = std::min(n_trans, t_lo + slice_len);
  chi0_tile<WPW, SUB, CHUNK>(lds, P, R, ld, delta, df, n_trans, t_lo, t_hi, omega, n_w, eta, n_g,
                             bx * C::kWBlock, gb * 16, gc * C::kCols,
                             part + (size_t)bz * n_w * n_g * n_g);
}

// Persistent form: a fixed grid (OCC workgroups per CU) walks the
// longest-first tile list in rounds of gridDim.x tiles (XCD-aware within a
// round), so every workgroup runs a similar amount of work and leaves when it
// passes the end.  No LDS beyond the tile's double buffer (two workgroups still fit per
// CU) and no atomics; the assignment is deterministic.
template <int WPW, int SUB, int CHUNK, int OCC>
__global__ void __launch_bounds__(256, OCC)
    k_chi0_bf16x3_persistent(const BatchItem *items, const BatchTile *tiles, int n_tiles) {
  typedef Cfg<WPW, SUB, CHUNK> C;
  extern __shared__ unsigned int lds[];
  const int G = gridDim.x;
  for (int base = 0; base < n_tiles; base += G) {
    // round `base`: logical tiles base..base+G-1, a contiguous block per XCD
    const int idx = base + xcd_logical(blockIdx.x, G);
    if (idx >= n_tiles) break;
    const BatchTile tl = tiles[idx];
    const BatchItem it = items[tl.item];
    const long long t_lo = tl.slice * it.slice_len;
    const long long t_hi = std::min(it.n_trans, t_lo + it.slice_len);
    chi0_tile<WPW, SUB, CHUNK>(lds, it.P, it.R, it.ld, it.delta, it.df, it.n_trans,
                               t_lo, t_hi, it.omega, it.n_w, it.eta, it.n_g,
                               tl.wblk * C::kWBlock, tl.gb * 16, tl.gc * C::kCols,
                               it.part + (size_t)tl.slice * it.n_w * it.n_g * it.n_g);
    __syncthreads();  // the next tile's prologue rewrites the LDS buffers
  }
}

struct Variant {
  int wpw, sub, chunk, occ;
  size_t lds;
  const void *grid_fn;
  const void *pers_fn;
};

#define TDX_V(W, S, K, O)                                                                \
  Variant {                                                                              \
    W, S, K, O, Cfg<W, S, K>::kLds, (const void *)k_chi0_bf16x3<W, S, K, O>,             \
        (const void *)k_chi0_bf16x3_persistent<W, S, K, O>                               \
  }
const Variant kVariants[] = {TDX_V(4, 4, 32, 2), TDX_V(2, 8, 16, 2), TDX_V(4, 2, 32, 2),
                             TDX_V(2, 4, 32, 2)};
#undef TDX_V

}  // namespace

int bf16x3_variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }

void bf16x3_variant_shape(int v, int *wblock, int *cols) {
  *wblock = 4 * kVariants[v].wpw;
  *cols = 16 * kVariants[v].sub;
}

int bf16x3_variant_occupancy(int v) { return kVariants[v].occ; }

int bf16x3_launch_grid(int v, const void *P, const void *R, int ld, const double *delta,
                       const double *df,
                       long long n_trans, long long slice_len, int slices, const double *omega,
                       int n_w, double eta, int n_g, double2 *part, hipStream_t s) {
  const Variant &V = kVariants[v];
  const int nblk = ld / 16;
  int ncb = (ld + 16 * V.sub - 1) / (16 * V.sub);
  dim3 grid((n_w + 4 * V.wpw - 1) / (4 * V.wpw), nblk * ncb, (unsigned)slices);
  TDX_HIP(hipFuncSetAttribute(V.grid_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)V.lds));
  void *args[] = {(void *)&P,       (void *)&R,         (void *)&ld,
                  (void *)&delta,   (void *)&df,
                  (void *)&n_trans, (void *)&slice_len, (void *)&omega, (void *)&n_w,
                  (void *)&eta,     (void *)&n_g,       (void *)&ncb,   (void *)&part};
  TDX_HIP(hipLaunchKernel(V.grid_fn, grid, dim3(256), args, V.lds, s));
  return TDX_OK;
}

int bf16x3_launch_persistent(int v, const BatchItem *items, const BatchTile *tiles, int n_tiles,
                             int n_blocks, hipStream_t s) {
  const Variant &V = kVariants[v];
  TDX_HIP(hipFuncSetAttribute(V.pers_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)V.lds));
  void *args[] = {(void *)&items, (void *)&tiles, (void *)&n_tiles};
  TDX_HIP(hipLaunchKernel(V.pers_fn, dim3(n_blocks), dim3(256), args, V.lds, s));
  return TDX_OK;
}

}  // namespace tdx
